// mrlbm2d.hip -- the two-dimensional adaptive MR-LBM step on the GPU (the multi-dimensional
// extension of the paper's conclusion: projection as the mean over the four children, the
// tensor product of the centered prediction, eps_l = 2^{d (l - J)} eps, enlargement rule (b)
// at 2^{mu_bar + d} eps_l), with a D2Q4 scheme for a scalar conservation law.
//
// Layout: dense levels in device memory. Level l (J_min <= l <= J) holds q planes of
// N_l x N_l values (index (h * N_l + i) * N_l + j, i along x) and, below J, one byte per cell
// for "split" (the cell has four children). A step is a sequence of level-wide phases:
// projection up the tree, details and thresholds, the two enlargement rules, the grading
// sweep from fine to coarse, the data transfer from coarse to fine, the leaves collision, the
// projection of the collided values, the reconstruction on the finest level (only of the cells
// the stream reads) and the compact stream (for each leaf and velocity the difference of the
// strips entering and leaving it). A phase whose levels are independent runs as one launch
// over all of them; a level-serial phase runs one launch per fine level and sweeps the coarse
// levels in a single workgroup.
// Every expression is written in the order the FP64 checks use, with no contraction into
// fused multiply-adds (the build passes -ffp-contract=off), so that the threshold decisions
// and the values agree bit for bit.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "mrlbm.h"

namespace {

constexpr int Q2 = 4;  // D2Q4: (+x, -x, +y, -y)

struct P2 {
    int jmin, J, gamma, mu_bar, bc, physics;
    double eps, lam, lam2, s1, s2, s3, oms1, oms2, oms3, Vx, Vy;
    double c[3];
};

__device__ __forceinline__ int bci(int i, int n, int bc) {
    if (bc == MRLBM_PERIODIC) return i & (n - 1);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// value of plane h at cell (i + di, j + dj) of a level of n x n cells
__device__ __forceinline__ double at(const double* f, int h, int n, int i, int j, int bc) {
    return f[((size_t)h * n + bci(i, n, bc)) * n + bci(j, n, bc)];
}

// The terms of the tensor-product prediction of the four children of (i, j) on plane h:
// child (2i + a, 2j + b) is ((f + sa Qx) + sb Qy) + sa sb Qxy with sa = (-1)^a, sb = (-1)^b
struct Terms {
    double f, qx, qy, qxy;
};

__device__ Terms predict_terms(const P2& p, const double* f, int h, int n, int i, int j) {
    const int bc = p.bc;
    double qx = 0.0, qy = 0.0, qxy = 0.0;
    for (int al = 1; al <= p.gamma; ++al) {
        const double tx = p.c[al - 1] * (at(f, h, n, i + al, j, bc) - at(f, h, n, i - al, j, bc));
        const double ty = p.c[al - 1] * (at(f, h, n, i, j + al, bc) - at(f, h, n, i, j - al, bc));
        qx = al == 1 ? tx : qx + tx;
        qy = al == 1 ? ty : qy + ty;
    }
    bool first = true;
    for (int al = 1; al <= p.gamma; ++al)
        for (int be = 1; be <= p.gamma; ++be) {
            const double cc = p.c[al - 1] * p.c[be - 1];
            const double t = cc * ((at(f, h, n, i + al, j + be, bc) - at(f, h, n, i + al, j - be, bc)) -
                                   (at(f, h, n, i - al, j + be, bc) - at(f, h, n, i - al, j - be, bc)));
            qxy = first ? t : qxy + t;
            first = false;
        }
    return Terms{f[((size_t)h * n + i) * n + j], qx, qy, qxy};
}

__device__ __forceinline__ double child_value(const Terms& q, int a, int b) {
    const double sa = a ? -1.0 : 1.0, sb = b ? -1.0 : 1.0;
    return ((q.f + sa * q.qx) + sb * q.qy) + (sa * sb) * q.qxy;
}

// D2Q4 collision (the oracle's fixed order)
__device__ void collide4(const P2& p, double* f) {
    const double u = ((f[0] + f[1]) + f[2]) + f[3];
    const double m1 = p.lam * (f[0] - f[1]);
    const double m2 = p.lam * (f[2] - f[3]);
    const double m3 = p.lam2 * ((f[0] + f[1]) - (f[2] + f[3]));
    double px, py;
    if (p.physics == MRLBM_ADVECTION) {
        px = p.Vx * u;
        py = p.Vy * u;
    } else {
        px = (u * u) * 0.5;
        py = (u * u) * 0.5;
    }
    const double m1s = p.oms1 * m1 + p.s1 * px;
    const double m2s = p.oms2 * m2 + p.s2 * py;
    const double m3s = p.oms3 * m3;
    const double a = m1s / p.lam, b = m2s / p.lam, c = m3s / p.lam2;
    const double e = 0.5 * (u + c), o = 0.5 * (u - c);
    f[0] = 0.5 * (e + a);
    f[1] = 0.5 * (e - a);
    f[2] = 0.5 * (o + b);
    f[3] = 0.5 * (o - b);
}

__global__ void k2_init(P2 p, const double* u0, double* FJ) {
    const int n = 1 << p.J;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)n * n) return;
    const double u = u0[k];
    double px, py;
    if (p.physics == MRLBM_ADVECTION) {
        px = p.Vx * u;
        py = p.Vy * u;
    } else {
        px = (u * u) * 0.5;
        py = (u * u) * 0.5;
    }
    const double a = px / p.lam, b = py / p.lam, c = 0.0 / p.lam2;
    const double e = 0.5 * (u + c), o = 0.5 * (u - c);
    const size_t nn = (size_t)n * n;
    FJ[k] = 0.5 * (e + a);
    FJ[nn + k] = 0.5 * (e - a);
    FJ[2 * nn + k] = 0.5 * (o + b);
    FJ[3 * nn + k] = 0.5 * (o - b);
}

__global__ void k2_fill(uint8_t* s, size_t n, uint8_t v) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) s[k] = v;
}

// ---- The phases, per cell: k is the cell's index on its level (or its parent's, as stated).
// Each phase runs as one kernel per level, as one kernel over several levels at once where
// the levels are independent, or, for the level-serial phases on the coarse levels, in one
// workgroup that sweeps them with a barrier between levels.

// projection of the split cell k of level l from level l + 1
__device__ void project_at(int l, const uint8_t* split, const double* fine, double* coarse, size_t k) {
    const int n = 1 << l;
    if (k >= (size_t)n * n || !split[k]) return;
    const int i = (int)(k / n), j = (int)(k % n);
    const int m = 2 * n;
    // every load before the stores (the compiler cannot tell the arrays apart)
    double v[Q2];
    for (int h = 0; h < Q2; ++h) {
        const double* g = fine + (size_t)h * m * m;
        const double a = g[(size_t)(2 * i) * m + 2 * j], b = g[(size_t)(2 * i + 1) * m + 2 * j];
        const double c = g[(size_t)(2 * i) * m + 2 * j + 1], d = g[(size_t)(2 * i + 1) * m + 2 * j + 1];
        v[h] = (((a + b) + c) + d) * 0.25;
    }
    for (int h = 0; h < Q2; ++h) coarse[((size_t)h * n + i) * n + j] = v[h];
}

// details of cell k of level l: keep (T_eps) and rule-(b) flags, and the new tree's split flag,
// which starts as keep (the enlargement adds to it); true when a detail is not a number
__device__ bool details_at(const P2& p, int l, const uint8_t* split, const double* coarse, const double* fine,
                           uint8_t* keep, uint8_t* ruleb, uint8_t* nsplit, size_t k) {
    const int n = 1 << l;
    if (k >= (size_t)n * n) return false;
    keep[k] = 0;
    ruleb[k] = 0;
    nsplit[k] = 0;
    if (!split[k]) return false;
    const int i = (int)(k / n), j = (int)(k % n);
    const int m = 2 * n;
    double D = 0.0;
    bool bad = false;
    for (int h = 0; h < Q2; ++h) {
        const Terms q = predict_terms(p, coarse, h, n, i, j);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                const double pr = child_value(q, a, b);
                const double d = fabs(fine[((size_t)h * m + 2 * i + a) * m + 2 * j + b] - pr);
                bad = bad || (d != d);
                D = d > D ? d : D;
            }
    }
    const double thr = ldexp(p.eps, 2 * (l + 1 - p.J));
    const double thrb = ldexp(thr, p.mu_bar + 2);
    const bool kb = bad || D >= thr;
    keep[k] = kb;
    nsplit[k] = kb;
    ruleb[k] = kb && (l + 1 < p.J) && (bad || D >= thrb);
    return bad;
}

// rule (a): the kept cells' children put their sigma-box (sigma = 1) into R, i.e. their parents
// p -+ 1 split; rule (b): the four children of a flagged cell split
__device__ void enlarge_at(const P2& p, int l, const uint8_t* keep, const uint8_t* ruleb, uint8_t* nsplit_l,
                           uint8_t* nsplit_l1, size_t k) {
    const int n = 1 << l;
    if (k >= (size_t)n * n || !keep[k]) return;
    const int i = (int)(k / n), j = (int)(k % n);
    const int m = 2 * n;
    // children 2i..2i+1 shifted by -1..1 at level l + 1: parents i - 1 .. i + 1
    for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj) {
            const int ci = bci(2 * i + (di < 0 ? -1 : (di > 0 ? 2 : 0)), m, p.bc);
            const int cj = bci(2 * j + (dj < 0 ? -1 : (dj > 0 ? 2 : 0)), m, p.bc);
            nsplit_l[(size_t)(ci >> 1) * n + (cj >> 1)] = 1;
        }
    if (ruleb[k] && nsplit_l1)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) nsplit_l1[(size_t)(2 * i + a) * m + 2 * j + b] = 1;
}

// grading at level a: every split (a, p) puts its gamma-box into R (the parents split)
__device__ void grade_at(int a, int gamma, int bc, const uint8_t* sa, uint8_t* sa1, size_t k) {
    const int n = 1 << a;
    if (k >= (size_t)n * n || !sa[k]) return;
    const int i = (int)(k / n), j = (int)(k % n);
    const int h = n >> 1;
    for (int di = -gamma; di <= gamma; ++di)
        for (int dj = -gamma; dj <= gamma; ++dj) sa1[(size_t)(bci(i + di, n, bc) >> 1) * h + (bci(j + dj, n, bc) >> 1)] = 1;
}

// transfer at level l + 1: the children of cells split in the new tree and not in the old one
// are predicted (one thread per parent of level l)
__device__ void transfer_at(const P2& p, int l, const uint8_t* old_split_l, const uint8_t* new_split_l,
                            const double* coarse, double* fine, size_t k) {
    const int n = 1 << l, m = 2 * n;
    if (k >= (size_t)n * n || !new_split_l[k] || old_split_l[k]) return;
    const int i = (int)(k / n), j = (int)(k % n);
    Terms q[Q2];  // every load before the stores
    for (int h = 0; h < Q2; ++h) q[h] = predict_terms(p, coarse, h, n, i, j);
    for (int h = 0; h < Q2; ++h)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) fine[((size_t)h * m + 2 * i + a) * m + 2 * j + b] = child_value(q[h], a, b);
}

__device__ __forceinline__ bool collide_cell(const P2& p, double* F, size_t nn, size_t k) {
    double f[Q2];
    for (int h = 0; h < Q2; ++h) f[h] = F[h * nn + k];
    collide4(p, f);
    bool bad = false;
    for (int h = 0; h < Q2; ++h) {
        bad = bad || (f[h] != f[h]);
        F[h * nn + k] = f[h];
    }
    return bad;
}

// leaves collision at level l (cells of R not split): k is a parent of level l - 1, which
// collides those of its four children that are leaves when it is split (level j_min, with no
// parent level: k is the cell); returns the leaves collided, bad set when a value is not a number
__device__ int collide_at(const P2& p, int l, const uint8_t* split_lm1, const uint8_t* split_l, double* F, size_t t,
                          bool& bad) {
    const int n = 1 << l;
    const size_t nn = (size_t)n * n;
    int cnt = 0;
    if (!split_lm1) {
        if (t < nn && !(split_l && split_l[t])) {
            bad = collide_cell(p, F, nn, t);
            cnt = 1;
        }
    } else {
        const int m = n >> 1;
        if (t < (size_t)m * m && split_lm1[t]) {
            const int pi = (int)(t / m), pj = (int)(t % m);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const size_t k = (size_t)(2 * pi + a) * n + 2 * pj + b;
                    if (split_l && split_l[k]) continue;
                    bad = collide_cell(p, F, nn, k) || bad;
                    ++cnt;
                }
        }
    }
    return cnt;
}

// the same for four parents of level l - 1 per thread (t: the group), whose split flags one
// 32-bit load reads (a level of at least four parents; the flag arrays are 256-byte aligned)
__device__ int collide_quad_at(const P2& p, int l, const uint8_t* split_lm1, const uint8_t* split_l, double* F,
                               size_t t, bool& bad) {
    const int n = 1 << l, m = n >> 1;
    const size_t nn = (size_t)n * n;
    if (t >= (size_t)m * m / 4) return 0;
    const uint32_t w = reinterpret_cast<const uint32_t*>(split_lm1)[t];
    if (!w) return 0;
    int cnt = 0;
    for (int e = 0; e < 4; ++e) {
        if (!((w >> (8 * e)) & 0xFFu)) continue;
        const size_t q = 4 * t + e;
        const int pi = (int)(q / m), pj = (int)(q % m);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                const size_t k = (size_t)(2 * pi + a) * n + 2 * pj + b;
                if (split_l && split_l[k]) continue;
                bad = collide_cell(p, F, nn, k) || bad;
                ++cnt;
            }
    }
    return cnt;
}

// the leaf count of a wave into the step's total (one atomic per wave; at most 16 per thread)
__device__ void count_leaves(int cnt, unsigned long long* nleaf) {
    const unsigned long long c = (unsigned long long)__popcll(__ballot(cnt & 1)) +
                                 2ull * __popcll(__ballot(cnt & 2)) + 4ull * __popcll(__ballot(cnt & 4)) +
                                 8ull * __popcll(__ballot(cnt & 8)) + 16ull * __popcll(__ballot(cnt & 16));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(nleaf, c);
}

// leaf count of the step into the running total (cnt[0]: this step, cnt[1]: all steps)
__global__ void k2_tally(unsigned long long* cnt) {
    if (threadIdx.x == 0) cnt[1] += cnt[0];
}

// Flags of the children a parent's reconstruction must form: bit a (a = 0, 1) the children
// (2i + a, .) on the x-velocity planes, bit 2 + b the children (., 2j + b) on the y-velocity
// planes; NEED_ALL every child on every plane.
constexpr uint8_t NEED_ALL = 15;

// reconstruction from level l to l + 1: G_{l+1} = prediction of G_l, stored values on R (one
// thread per parent of level l: the children of a split cell are in R, the others predicted).
// With need_l, only the children and planes it flags (the others are left as they were).
__device__ void reconstruct_at(const P2& p, int l, const uint8_t* split_l, const uint8_t* need_l, const double* Gl,
                               const double* Fl1, double* Gl1, size_t k) {
    const int n = 1 << l, m = 2 * n;
    if (k >= (size_t)n * n) return;
    const int nb = need_l ? need_l[k] : NEED_ALL;
    if (!nb) return;
    const int i = (int)(k / n), j = (int)(k % n);
    const bool inR = split_l[k] != 0;
    // every load before the stores (the compiler cannot tell the arrays apart)
    double v[Q2][4];
    for (int h = 0; h < Q2; ++h) {
        const int hb = h < 2 ? (nb & 3) : (nb >> 2);
        if (!hb) continue;
        if (inR) {
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) v[h][2 * a + b] = Fl1[((size_t)h * m + 2 * i + a) * m + 2 * j + b];
        } else {
            const Terms q = predict_terms(p, Gl, h, n, i, j);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) v[h][2 * a + b] = child_value(q, a, b);
        }
    }
    for (int h = 0; h < Q2; ++h) {
        const int hb = h < 2 ? (nb & 3) : (nb >> 2);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                if ((hb >> (h < 2 ? a : b)) & 1) Gl1[((size_t)h * m + 2 * i + a) * m + 2 * j + b] = v[h][2 * a + b];
    }
}

// A run's per-level arrays by value (J <= 12), index l - j_min: values, the current tree's
// split flags (the old tree before the transfer, the new one after it), the new tree's, the
// keep and rule-(b) flags and the reconstruction flags.
constexpr int MAXL2 = 13;
struct Lv2 {
    double* F[MAXL2];
    const uint8_t* split[MAXL2];
    uint8_t* nsplit[MAXL2];
    uint8_t* keep[MAXL2];
    uint8_t* ruleb[MAXL2];
    uint8_t* need[MAXL2];
};


// Which children of the parents of level J - 1 the stream reads. On an x-velocity plane a
// leaf's stream reads the finest cells of its first and last columns and the cells just
// outside them; those outside cells lie in the last or first column of the neighbouring
// leaves (dyadic squares meet edge to edge), so the x planes are read exactly in the first
// and last columns of every leaf, and the y planes in the first and last rows. The children
// of a split parent are finest leaves (their own first and last columns and rows); for the
// other parents the flags follow from their place in the coarser leaf that holds them.
__global__ void k2_need_finest(P2 p, Lv2 L, uint8_t* need) {
    const int J = p.J, n = 1 << (J - 1);
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)n * n) return;
    const int i = (int)(k / n), j = (int)(k % n);
    uint8_t v = NEED_ALL;
    if (!L.split[J - 1 - p.jmin][k]) {
        // the leaf holding the cell: its finest ancestor level whose parent is split
        int l = J - 1;
        while (l > p.jmin && !L.split[l - 1 - p.jmin][(size_t)(i >> (J - l)) * ((size_t)1 << (l - 1)) + (j >> (J - l))]) --l;
        const int h = 1 << (J - 1 - l);  // the leaf's side in level-(J - 1) cells
        const int a = i & (h - 1), b = j & (h - 1);
        v = (uint8_t)((a == 0) | ((a == h - 1) << 1) | ((b == 0) << 2) | ((b == h - 1) << 3));
    }
    need[k] = v;
}

// need_{l-1} from need_l: G_l is needed at the children of a parent of level l - 1 when one
// of them lies in the (2 gamma + 1)^2 prediction box of a flagged, unsplit parent of level l
// (whose children are predicted from G_l). A plane's prediction reads that plane only, so the
// x planes and the y planes are flagged apart (all children of the x planes: bits 0-1, of the
// y planes: bits 2-3). The four children's boxes together cover the (2 gamma + 2)^2 cells from
// (2i - gamma, 2j - gamma); a gather, so every entry is written. (k: the parent of level l - 1)
__device__ void need_up_at(const P2& p, int l, const uint8_t* split_l, const uint8_t* need_l, uint8_t* need_lm1,
                           size_t k) {
    const int n = 1 << l, m = n >> 1;
    if (k >= (size_t)m * m) return;
    const int i = (int)(k / m), j = (int)(k % m);
    const int G = p.gamma;
    int v = 0;
    for (int di = -G; di <= G + 1 && v != NEED_ALL; ++di) {
        const size_t row = (size_t)bci(2 * i + di, n, p.bc) * n;
        for (int dj = -G; dj <= G + 1; ++dj) {
            const size_t q = row + bci(2 * j + dj, n, p.bc);
            const int nq = need_l[q];
            if (nq && !split_l[q]) v |= ((nq & 3) ? 3 : 0) | ((nq & 12) ? 12 : 0);
        }
    }
    need_lm1[k] = (uint8_t)v;
}

// compact stream of the leaf (l, i, j) from the finest reconstruction G (N_J x N_J): per
// velocity h0 <= h < h1 the strip of finest values entering the leaf minus the strip leaving
// it (each velocity reads and writes its own plane only)
__device__ void stream_leaf(const P2& p, int l, int i, int j, const double* G, double* F, int h0 = 0, int h1 = Q2) {
    const int n = 1 << l, NJ = 1 << p.J, L = 1 << (p.J - l);
    const size_t k = (size_t)i * n + j;
    const size_t nn = (size_t)n * n, NN = (size_t)NJ * NJ;
    const int x0 = i * L, y0 = j * L, bc = p.bc;
    const int wx[Q2] = {1, -1, 0, 0}, wy[Q2] = {0, 0, 1, -1};
    double out[Q2];
    for (int h = h0; h < h1; ++h) {
        const double* g = G + h * NN;
        if (l == p.J) {
            out[h] = g[(size_t)bci(x0 - wx[h], NJ, bc) * NJ + bci(y0 - wy[h], NJ, bc)];
            continue;
        }
        double acc = 0.0;
        // the terms are summed in strip order; the loads of the unrolled iterations go ahead
#pragma unroll 8
        for (int t = 0; t < L; ++t) {
            double a, b;
            if (wx[h] != 0) {
                const int y = bci(y0 + t, NJ, bc);
                a = g[(size_t)bci(wx[h] > 0 ? x0 - 1 : x0, NJ, bc) * NJ + y];
                b = g[(size_t)bci(wx[h] > 0 ? x0 + L - 1 : x0 + L, NJ, bc) * NJ + y];
            } else {
                const int x = bci(x0 + t, NJ, bc);
                a = g[(size_t)x * NJ + bci(wy[h] > 0 ? y0 - 1 : y0, NJ, bc)];
                b = g[(size_t)x * NJ + bci(wy[h] > 0 ? y0 + L - 1 : y0 + L, NJ, bc)];
            }
            const bool pos = (wx[h] + wy[h]) > 0;
            const double term = pos ? (a - b) : -(a - b);
            acc = t == 0 ? term : acc + term;
        }
        out[h] = F[h * nn + k] + ldexp(acc, -2 * (p.J - l));
    }
    for (int h = h0; h < h1; ++h) F[h * nn + k] = out[h];
}

// the leaves of level l < J, or of a J with no coarser level: one thread per cell, or with
// per_velocity one per cell and velocity (long strips: the four sums side by side)
__device__ void stream_cells_at(const P2& p, int l, const uint8_t* split_lm1, const uint8_t* split_l, const double* G,
                                double* F, bool per_velocity, size_t t) {
    const int n = 1 << l;
    const size_t k = per_velocity ? t / Q2 : t;
    if (k >= (size_t)n * n) return;
    const int i = (int)(k / n), j = (int)(k % n);
    if (split_lm1 && !split_lm1[(size_t)(i >> 1) * (n >> 1) + (j >> 1)]) return;  // not in R
    if (split_l && split_l[k]) return;                                              // not a leaf
    if (per_velocity) {
        const int h = (int)(t % Q2);
        stream_leaf(p, l, i, j, G, F, h, h + 1);
    } else {
        stream_leaf(p, l, i, j, G, F);
    }
}

// The value of v in lane t of the wave (t a constant).
__device__ __forceinline__ double lane_value(double v, int t) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, t);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), t);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// the leaves of level l with strips of 64 cells or more: one wave per cell and velocity. The
// lanes load 64 strip positions at a time and every lane folds their terms in strip order, so
// the sum is the one stream_leaf forms.
// (t: the thread of the level; the level's threads start at a multiple of 64)
__device__ void stream_strips_at(const P2& p, int l, const uint8_t* split_lm1, const uint8_t* split_l, const double* G,
                                 double* F, size_t t) {
    const int n = 1 << l, NJ = 1 << p.J, L = 1 << (p.J - l);
    const size_t wv = t >> 6;
    const int lane = (int)(t & 63);
    const size_t k = wv / Q2;
    const int h = (int)(wv % Q2);
    if (k >= (size_t)n * n) return;
    const int i = (int)(k / n), j = (int)(k % n);
    if (split_lm1 && !split_lm1[(size_t)(i >> 1) * (n >> 1) + (j >> 1)]) return;  // not in R
    if (split_l && split_l[k]) return;                                              // not a leaf
    const size_t nn = (size_t)n * n, NN = (size_t)NJ * NJ;
    const int x0 = i * L, y0 = j * L, bc = p.bc;
    const int wx = h == 0 ? 1 : (h == 1 ? -1 : 0), wy = h == 2 ? 1 : (h == 3 ? -1 : 0);
    const bool pos = (wx + wy) > 0;
    const double* g = G + h * NN;
    double acc = 0.0;
    for (int c = 0; c < L; c += 64) {
        const int t = c + lane;
        double a, b;
        if (wx != 0) {
            const int y = bci(y0 + t, NJ, bc);
            a = g[(size_t)bci(wx > 0 ? x0 - 1 : x0, NJ, bc) * NJ + y];
            b = g[(size_t)bci(wx > 0 ? x0 + L - 1 : x0 + L, NJ, bc) * NJ + y];
        } else {
            const int x = bci(x0 + t, NJ, bc);
            a = g[(size_t)x * NJ + bci(wy > 0 ? y0 - 1 : y0, NJ, bc)];
            b = g[(size_t)x * NJ + bci(wy > 0 ? y0 + L - 1 : y0 + L, NJ, bc)];
        }
        const double term = pos ? (a - b) : -(a - b);
#pragma unroll
        for (int u = 0; u < 64; ++u) {
            const double x = lane_value(term, u);
            acc = (c == 0 && u == 0) ? x : acc + x;
        }
    }
    if (lane == 0) F[h * nn + k] = F[h * nn + k] + ldexp(acc, -2 * (p.J - l));
}

// the leaves of the finest level J > jmin (strips of one cell): one thread per parent of level
// J - 1, which streams its four children when it is split (split parents cluster along fronts,
// so grouping parents per thread would serialise their streams)
__global__ void k2_stream_finest(P2 p, const uint8_t* split_jm1, const double* G, double* F) {
    const int n = 1 << p.J, np = n >> 1;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)np * np || !split_jm1[k]) return;
    const int pi = (int)(k / np), pj = (int)(k % np);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) stream_leaf(p, p.J, 2 * pi + a, 2 * pj + b, G, F);
}

// Threads of one launch over several levels: level l0 + i owns the threads off[i] .. off[i+1] - 1
// (each a multiple of the workgroup size, so that no workgroup spans two levels).
struct Sweep {
    int l0, nl;
    unsigned long long off[MAXL2 + 1];
};

__device__ __forceinline__ int sweep_level(const Sweep& sw, unsigned long long t, unsigned long long& k) {
    int i = 0;
    while (i + 1 < sw.nl && t >= sw.off[i + 1]) ++i;
    k = t - sw.off[i];
    return sw.l0 + i;
}

__device__ __forceinline__ unsigned long long gtid() { return (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ unsigned long long cells_of(int l) { return 1ull << (2 * l); }

// ---- one level per launch
__global__ void k2_project(int l, const uint8_t* split, const double* fine, double* coarse) {
    project_at(l, split, fine, coarse, gtid());
}
__global__ void k2_grade(int a, int gamma, int bc, const uint8_t* sa, uint8_t* sa1) { grade_at(a, gamma, bc, sa, sa1, gtid()); }
__global__ void k2_transfer(P2 p, int l, const uint8_t* old_split_l, const uint8_t* new_split_l, const double* coarse,
                            double* fine) {
    transfer_at(p, l, old_split_l, new_split_l, coarse, fine, gtid());
}
__global__ void k2_need_up(P2 p, int l, const uint8_t* split_l, const uint8_t* need_l, uint8_t* need_lm1) {
    need_up_at(p, l, split_l, need_l, need_lm1, gtid());
}
__global__ void k2_reconstruct(P2 p, int l, const uint8_t* split_l, const uint8_t* need_l, const double* Gl,
                               const double* Fl1, double* Gl1) {
    reconstruct_at(p, l, split_l, need_l, Gl, Fl1, Gl1, gtid());
}

// ---- the independent levels of a phase in one launch
// Levels of at least four cells take four consecutive cells per thread in the level-wide
// sweeps: one 32-bit load of their flags (the byte arrays are 256-byte aligned) skips the
// group when none of them is split (details) or kept (enlargement).
__device__ __forceinline__ bool quad_level(int l) { return l >= 1; }

__global__ void k2_details_all(P2 p, Sweep sw, Lv2 L, int* nan_flag) {
    unsigned long long k;
    const int l = sweep_level(sw, gtid(), k);
    const int li = l - p.jmin;
    if (!quad_level(l)) {
        if (details_at(p, l, L.split[li], L.F[li], L.F[li + 1], L.keep[li], L.ruleb[li], L.nsplit[li], k)) *nan_flag = 1;
        return;
    }
    if (k >= cells_of(l) / 4) return;
    if (!reinterpret_cast<const uint32_t*>(L.split[li])[k]) {
        reinterpret_cast<uint32_t*>(L.keep[li])[k] = 0u;
        reinterpret_cast<uint32_t*>(L.ruleb[li])[k] = 0u;
        reinterpret_cast<uint32_t*>(L.nsplit[li])[k] = 0u;
        return;
    }
    bool bad = false;
    for (int e = 0; e < 4; ++e)
        bad = details_at(p, l, L.split[li], L.F[li], L.F[li + 1], L.keep[li], L.ruleb[li], L.nsplit[li], 4 * k + e) || bad;
    if (bad) *nan_flag = 1;
}
__global__ void k2_enlarge_all(P2 p, Sweep sw, Lv2 L) {
    unsigned long long k;
    const int l = sweep_level(sw, gtid(), k);
    const int li = l - p.jmin;
    uint8_t* nl1 = l + 1 < p.J ? L.nsplit[li + 1] : nullptr;
    if (!quad_level(l)) {
        enlarge_at(p, l, L.keep[li], L.ruleb[li], L.nsplit[li], nl1, k);
        return;
    }
    if (k >= cells_of(l) / 4 || !reinterpret_cast<const uint32_t*>(L.keep[li])[k]) return;
    for (int e = 0; e < 4; ++e) enlarge_at(p, l, L.keep[li], L.ruleb[li], L.nsplit[li], nl1, 4 * k + e);
}
__global__ void k2_collide_all(P2 p, Sweep sw, Lv2 L, unsigned long long* nleaf, int* nan_flag) {
    unsigned long long k;
    const int l = sweep_level(sw, gtid(), k);
    const int li = l - p.jmin;
    bool bad = false;
    const int cnt = l > p.jmin && l >= 2
                        ? collide_quad_at(p, l, L.split[li - 1], l < p.J ? L.split[li] : nullptr, L.F[li], k, bad)
                        : collide_at(p, l, l > p.jmin ? L.split[li - 1] : nullptr, l < p.J ? L.split[li] : nullptr,
                                     L.F[li], k, bad);
    count_leaves(cnt, nleaf);
    if (bad) *nan_flag = 1;
}
__global__ void k2_stream_cells_all(P2 p, Sweep sw, Lv2 L, const double* G) {
    unsigned long long k;
    const int l = sweep_level(sw, gtid(), k);
    const int li = l - p.jmin;
    stream_cells_at(p, l, l > p.jmin ? L.split[li - 1] : nullptr, l < p.J ? L.split[li] : nullptr, G, L.F[li],
                    p.J - l >= 4, k);
}
__global__ void k2_stream_strips_all(P2 p, Sweep sw, Lv2 L, const double* G) {
    unsigned long long k;
    const int l = sweep_level(sw, gtid(), k);
    const int li = l - p.jmin;
    stream_strips_at(p, l, l > p.jmin ? L.split[li - 1] : nullptr, L.split[li], G, L.F[li], k);
}

// ---- the coarse levels of a level-serial phase in one workgroup: levels of at most 4096 cells
// for the light phases, of at most 256 for the reconstruction and its flags, whose cells each
// wait on several dependent loads (one workgroup hides little of that latency)
constexpr int COARSE_CELLS = 4096;
constexpr int COARSE_CELLS_HEAVY = 256;
constexpr int COARSE_THREADS = 1024;

__global__ __launch_bounds__(COARSE_THREADS) void k2_project_coarse(Lv2 L, int jmin, int lhi, int llo) {
    for (int l = lhi; l >= llo; --l) {
        const size_t nn = (size_t)1 << (2 * l);
        for (size_t k = threadIdx.x; k < nn; k += blockDim.x) project_at(l, L.split[l - jmin], L.F[l + 1 - jmin], L.F[l - jmin], k);
        __syncthreads();
    }
}
__global__ __launch_bounds__(COARSE_THREADS) void k2_grade_coarse(P2 p, Lv2 L, int ahi, int alo) {
    for (int a = ahi; a >= alo; --a) {
        const size_t nn = (size_t)1 << (2 * a);
        for (size_t k = threadIdx.x; k < nn; k += blockDim.x)
            grade_at(a, p.gamma, p.bc, L.nsplit[a - p.jmin], L.nsplit[a - 1 - p.jmin], k);
        __syncthreads();
    }
}
__global__ __launch_bounds__(COARSE_THREADS) void k2_transfer_coarse(P2 p, Lv2 L, int llo, int lhi) {
    for (int l = llo; l <= lhi; ++l) {
        const int li = l - p.jmin;
        const size_t nn = (size_t)1 << (2 * l);
        for (size_t k = threadIdx.x; k < nn; k += blockDim.x) transfer_at(p, l, L.split[li], L.nsplit[li], L.F[li], L.F[li + 1], k);
        __syncthreads();
    }
}
__global__ __launch_bounds__(COARSE_THREADS) void k2_need_up_coarse(P2 p, Lv2 L, int lhi, int llo) {
    for (int l = lhi; l >= llo; --l) {
        const int li = l - p.jmin;
        const size_t nn = (size_t)1 << (2 * (l - 1));
        for (size_t k = threadIdx.x; k < nn; k += blockDim.x) need_up_at(p, l, L.split[li], L.need[li], L.need[li - 1], k);
        __syncthreads();
    }
}
// G of level j_min is its stored values; then levels llo = j_min .. lhi, G alternating between ga
// and gb (level l + 1 lands in gb when l - j_min is even)
__global__ __launch_bounds__(COARSE_THREADS) void k2_reconstruct_coarse(P2 p, Lv2 L, int lhi, int use_need, double* ga,
                                                                        double* gb) {
    const size_t n0 = (size_t)Q2 << (2 * p.jmin);
    for (size_t k = threadIdx.x; k < n0; k += blockDim.x) ga[k] = L.F[0][k];
    __syncthreads();
    for (int l = p.jmin; l <= lhi; ++l) {
        const int li = l - p.jmin;
        const size_t nn = (size_t)1 << (2 * l);
        for (size_t k = threadIdx.x; k < nn; k += blockDim.x)
            reconstruct_at(p, l, L.split[li], use_need ? L.need[li] : nullptr, ga, L.F[li + 1], gb, k);
        __syncthreads();
        double* t = ga;
        ga = gb;
        gb = t;
    }
}

// conserved moment u on the finest level from the reconstruction
__global__ void k2_moment(int NJ, const double* G, double* out) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t NN = (size_t)NJ * NJ;
    if (k >= NN) return;
    out[k] = ((G[k] + G[NN + k]) + G[2 * NN + k]) + G[3 * NN + k];
}

struct Run2D {
    P2 p;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<double*> F;      // per level, q x N_l x N_l
    std::vector<uint8_t*> split; // per level < J
    std::vector<uint8_t*> nsplit, keep, ruleb;
    std::vector<uint8_t*> need;  // per level < J: parents whose children the stream needs
    double* G0 = nullptr;        // reconstruction ping-pong (finest size)
    double* G1 = nullptr;
    double* out = nullptr;       // finest conserved moment
    unsigned long long* d_nleaf = nullptr;
    int* d_nan = nullptr;
    long long steps = 0, leaf_updates = 0, leaves = 0;
    bool numeric = false;
    std::string err;
    std::vector<void*> allocs;
};

thread_local std::string g_err2d;

int fail2d(Run2D* r, hipError_t st, const char* what) {
    r->err = std::string(what) + ": " + hipGetErrorString(st);
    return st == hipErrorOutOfMemory ? MRLBM_ENOMEM : MRLBM_EDEVICE;
}

unsigned blocks(size_t n) { return (unsigned)((n + 255) / 256); }

void free2d(Run2D* r) {
    if (!r) return;
    for (void* a : r->allocs) (void)hipFree(a);
    if (r->own_stream && r->stream) (void)hipStreamDestroy(r->stream);
    delete r;
}

int validate2d(const mrlbm2d_params* q, std::string* why) {
    auto bad = [&](const char* m) {
        if (why) *why = m;
        return (int)MRLBM_EINVAL;
    };
    if (!q) return bad("params is NULL");
    if (q->abi_version != MRLBM_ABI_VERSION) return bad("abi_version mismatch");
    if (q->physics != MRLBM_ADVECTION && q->physics != MRLBM_BURGERS) return bad("physics: advection or Burgers");
    if (q->bc != MRLBM_PERIODIC && q->bc != MRLBM_CLAMP) return bad("bc must be PERIODIC or CLAMP");
    if (!(q->lambda > 0.0) || !isfinite(q->lambda)) return bad("lambda must be finite and > 0");
    for (int i = 0; i < 3; ++i)
        if (!(q->s[i] > 0.0 && q->s[i] <= 2.0)) return bad("relaxation rates must lie in (0, 2]");
    if (!isfinite(q->V[0]) || !isfinite(q->V[1])) return bad("V must be finite");
    if (q->gamma < 1 || q->gamma > 3) return bad("gamma must be 1, 2 or 3");
    if (q->j_min < 0 || q->j_min > q->j_max) return bad("need 0 <= j_min <= j_max");
    if (q->j_max > 12) {
        if (why) *why = "j_max beyond 12";
        return MRLBM_ECAPACITY;
    }
    if (q->bc == MRLBM_PERIODIC && (1 << q->j_min) < 2 * q->gamma + 1)
        return bad("periodic coarsest level needs 2^j_min >= 2 gamma + 1");
    if (q->mu_bar < 0 || q->mu_bar > 30) return bad("mu_bar must be in 0..30");
    if (!(q->eps >= 0.0) || !isfinite(q->eps)) return bad("eps must be finite and >= 0");
    return MRLBM_OK;
}

Lv2 levels2d(const Run2D* r) {
    Lv2 L{};
    const int nlev = r->p.J - r->p.jmin;
    for (int li = 0; li <= nlev; ++li) {
        L.F[li] = r->F[li];
        if (li < nlev) {
            L.split[li] = r->split[li];
            L.nsplit[li] = r->nsplit[li];
            L.keep[li] = r->keep[li];
            L.ruleb[li] = r->ruleb[li];
            L.need[li] = r->need[li];
        }
    }
    return L;
}

// A launch over levels lo..hi with cnt(l) threads each: returns the total thread count.
template <class C>
unsigned long long make_sweep(int lo, int hi, C cnt, Sweep& sw) {
    sw.l0 = lo;
    sw.nl = hi - lo + 1;
    unsigned long long o = 0;
    for (int i = 0; i < sw.nl; ++i) {
        sw.off[i] = o;
        o += ((unsigned long long)cnt(lo + i) + 255ull) / 256ull * 256ull;
    }
    sw.off[sw.nl] = o;
    return o;
}

// The finest level of at most `cells` cells (the coarse single-workgroup kernels' range).
int coarse_top(int cells = COARSE_CELLS) {
    int l = 0;
    while (((size_t)1 << (2 * (l + 1))) <= (size_t)cells) ++l;
    return l;
}

size_t cells2(int l) { return (size_t)1 << (2 * l); }

// projection up the tree of the current split flags: the fine levels one launch each, the
// coarse ones in one workgroup
void project2d(Run2D* r, const Lv2& L) {
    const int J = r->p.J, jmin = r->p.jmin, lc = coarse_top();
    for (int l = J - 1; l >= jmin && l > lc; --l)
        hipLaunchKernelGGL(k2_project, dim3(blocks(cells2(l))), dim3(256), 0, r->stream, l, L.split[l - jmin],
                           (const double*)L.F[l + 1 - jmin], L.F[l - jmin]);
    const int top = std::min(lc, J - 1);
    if (top >= jmin) hipLaunchKernelGGL(k2_project_coarse, dim3(1), dim3(COARSE_THREADS), 0, r->stream, L, jmin, top, jmin);
}

// the reconstruction of the finest level into G0 / G1 (use_need: only what the stream reads);
// returns the buffer that holds it
double* reconstruct2d(Run2D* r, const Lv2& L, int use_need) {
    const P2& p = r->p;
    const int J = p.J, jmin = p.jmin, lc = coarse_top(COARSE_CELLS_HEAVY);
    double* ga = r->G0;
    double* gb = r->G1;
    const int top = std::min(lc, J - 1);
    hipLaunchKernelGGL(k2_reconstruct_coarse, dim3(1), dim3(COARSE_THREADS), 0, r->stream, p, L, top, use_need, ga, gb);
    if (top >= jmin && (top - jmin) % 2 == 0) std::swap(ga, gb);
    for (int l = std::max(jmin, lc + 1); l < J; ++l) {
        hipLaunchKernelGGL(k2_reconstruct, dim3(blocks(cells2(l))), dim3(256), 0, r->stream, p, l, L.split[l - jmin],
                           use_need ? (const uint8_t*)L.need[l - jmin] : (const uint8_t*)nullptr, (const double*)ga,
                           (const double*)L.F[l + 1 - jmin], gb);
        std::swap(ga, gb);
    }
    return ga;
}

int step2d(Run2D* r) {
    const P2& p = r->p;
    const int J = p.J, jmin = p.jmin, lc = coarse_top();
    hipStream_t s = r->stream;
    Lv2 L = levels2d(r);
    Sweep sw;
    // 1. projection of f^n up the tree
    project2d(r, L);
    if (J > jmin) {
        // 2. details, T_eps and rule-(b) flags; the new tree starts as the kept cells
        auto quad = [](int l) { return l >= 1 ? cells2(l) / 4 : cells2(l); };  // as quad_level
        unsigned long long nt = make_sweep(jmin, J - 1, quad, sw);
        hipLaunchKernelGGL(k2_details_all, dim3((unsigned)(nt / 256)), dim3(256), 0, s, p, sw, L, r->d_nan);
        // 3. enlargement, rules (a) and (b)
        nt = make_sweep(jmin, J - 1, quad, sw);
        hipLaunchKernelGGL(k2_enlarge_all, dim3((unsigned)(nt / 256)), dim3(256), 0, s, p, sw, L);
        // 4. grading, fine to coarse
        for (int a = J - 1; a > jmin && a > lc; --a)
            hipLaunchKernelGGL(k2_grade, dim3(blocks(cells2(a))), dim3(256), 0, s, a, p.gamma, p.bc,
                               (const uint8_t*)r->nsplit[a - jmin], r->nsplit[a - 1 - jmin]);
        int top = std::min(lc, J - 1);
        if (top > jmin) hipLaunchKernelGGL(k2_grade_coarse, dim3(1), dim3(COARSE_THREADS), 0, s, p, L, top, jmin + 1);
        // 5. transfer, coarse to fine
        if (top >= jmin) hipLaunchKernelGGL(k2_transfer_coarse, dim3(1), dim3(COARSE_THREADS), 0, s, p, L, jmin, top);
        for (int l = std::max(jmin, lc + 1); l < J; ++l)
            hipLaunchKernelGGL(k2_transfer, dim3(blocks(cells2(l))), dim3(256), 0, s, p, l, (const uint8_t*)r->split[l - jmin],
                               (const uint8_t*)r->nsplit[l - jmin], (const double*)r->F[l - jmin], r->F[l + 1 - jmin]);
    }
    // the new tree replaces the old one
    std::swap(r->split, r->nsplit);
    L = levels2d(r);
    // 6. leaves collision (d_nleaf[0] counts this step's leaves)
    if (hipMemsetAsync(r->d_nleaf, 0, sizeof(unsigned long long), s) != hipSuccess) return MRLBM_EDEVICE;
    {
        const unsigned long long nt =
            make_sweep(jmin, J, [jmin](int l) { return l > jmin ? (l >= 2 ? cells2(l - 1) / 4 : cells2(l - 1)) : cells2(l); }, sw);
        hipLaunchKernelGGL(k2_collide_all, dim3((unsigned)(nt / 256)), dim3(256), 0, s, p, sw, L, r->d_nleaf, r->d_nan);
    }
    hipLaunchKernelGGL(k2_tally, dim3(1), dim3(64), 0, s, r->d_nleaf);
    // 7. projection of the collided values
    project2d(r, L);
    // 8. the reconstruction, formed only where the stream reads it: the flags go from the
    // finest level's first and last columns and rows of the leaves up through the prediction boxes
    if (J > jmin) {
        hipLaunchKernelGGL(k2_need_finest, dim3(blocks(cells2(J - 1))), dim3(256), 0, s, p, L, r->need[J - 1 - jmin]);
        const int lh = coarse_top(COARSE_CELLS_HEAVY);
        for (int l = J - 1; l > jmin && l > lh; --l)
            hipLaunchKernelGGL(k2_need_up, dim3(blocks(cells2(l - 1))), dim3(256), 0, s, p, l, (const uint8_t*)r->split[l - jmin],
                               (const uint8_t*)r->need[l - jmin], r->need[l - 1 - jmin]);
        const int top = std::min(lh, J - 1);
        if (top > jmin) hipLaunchKernelGGL(k2_need_up_coarse, dim3(1), dim3(COARSE_THREADS), 0, s, p, L, top, jmin + 1);
    }
    const double* G = reconstruct2d(r, L, 1);
    // 9. stream: strips of 64 cells or more a wave per cell and velocity, 16 or more a thread per
    // cell and velocity, shorter ones a thread per cell; the finest leaves per parent
    const int ls = J - 6;  // the finest level with strips of 64 cells
    if (ls >= jmin) {
        const unsigned long long nt = make_sweep(jmin, ls, [](int l) { return cells2(l) * Q2 * 64; }, sw);
        hipLaunchKernelGGL(k2_stream_strips_all, dim3((unsigned)(nt / 256)), dim3(256), 0, s, p, sw, L, G);
    }
    if (J - 1 >= std::max(jmin, ls + 1)) {
        const int J_ = J;
        const unsigned long long nt = make_sweep(
            std::max(jmin, ls + 1), J - 1, [J_](int l) { return cells2(l) * (J_ - l >= 4 ? Q2 : 1); }, sw);
        hipLaunchKernelGGL(k2_stream_cells_all, dim3((unsigned)(nt / 256)), dim3(256), 0, s, p, sw, L, G);
    }
    if (J > jmin) {
        hipLaunchKernelGGL(k2_stream_finest, dim3(blocks(cells2(J - 1))), dim3(256), 0, s, p, r->split[J - 1 - jmin], G,
                           r->F[J - jmin]);
    } else {
        const unsigned long long nt = make_sweep(J, J, cells2, sw);
        hipLaunchKernelGGL(k2_stream_cells_all, dim3((unsigned)(nt / 256)), dim3(256), 0, s, p, sw, L, G);
    }
    hipError_t st = hipGetLastError();
    if (st != hipSuccess) return fail2d(r, st, "step launch");
    r->steps += 1;
    return MRLBM_OK;
}

// After the steps of a call: this step's leaves, the running total and the NaN flag.
int finish2d(Run2D* r) {
    unsigned long long cnt[2] = {0, 0};
    int nan = 0;
    hipError_t st = hipMemcpyAsync(cnt, r->d_nleaf, sizeof(cnt), hipMemcpyDeviceToHost, r->stream);
    if (st == hipSuccess) st = hipMemcpyAsync(&nan, r->d_nan, sizeof(int), hipMemcpyDeviceToHost, r->stream);
    if (st == hipSuccess) st = hipStreamSynchronize(r->stream);
    if (st != hipSuccess) return fail2d(r, st, "step");
    if (r->steps > 0) r->leaves = (long long)cnt[0];
    r->leaf_updates = (long long)cnt[1];
    if (nan) {
        r->numeric = true;
        return MRLBM_ENUMERIC;
    }
    return MRLBM_OK;
}

}  // namespace

struct mrlbm2d_s {
    Run2D* r;
};

extern "C" {

int mrlbm2d_validate(const mrlbm2d_params* p) { return validate2d(p, nullptr); }

int mrlbm2d_create(const mrlbm2d_params* q, const double* u0, void* hip_stream, mrlbm2d_t* out) {
    if (!out) return MRLBM_EINVAL;
    *out = nullptr;
    g_err2d.clear();
    std::string why;
    int rc = validate2d(q, &why);
    if (rc != MRLBM_OK) {
        g_err2d = why;
        return rc;
    }
    if (!u0) {
        g_err2d = "initial data pointer is NULL";
        return MRLBM_EINVAL;
    }
    const size_t NJ = (size_t)1 << q->j_max;
    for (size_t k = 0; k < NJ * NJ; ++k)
        if (!isfinite(u0[k])) {
            g_err2d = "initial data must be finite";
            return MRLBM_EINVAL;
        }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        g_err2d = "no HIP device";
        return MRLBM_EDEVICE;
    }
    Run2D* r = new (std::nothrow) Run2D();
    if (!r) return MRLBM_ENOMEM;
    P2& p = r->p;
    memset(&p, 0, sizeof(p));
    p.jmin = q->j_min;
    p.J = q->j_max;
    p.gamma = q->gamma;
    p.mu_bar = q->mu_bar;
    p.bc = q->bc;
    p.physics = q->physics;
    p.eps = q->eps;
    p.lam = q->lambda;
    p.lam2 = q->lambda * q->lambda;
    p.s1 = q->s[0];
    p.s2 = q->s[1];
    p.s3 = q->s[2];
    p.oms1 = 1.0 - q->s[0];
    p.oms2 = 1.0 - q->s[1];
    p.oms3 = 1.0 - q->s[2];
    p.Vx = q->V[0];
    p.Vy = q->V[1];
    if (q->gamma == 1) {
        p.c[0] = -1.0 / 8.0;
    } else if (q->gamma == 2) {
        p.c[0] = -22.0 / 128.0;
        p.c[1] = 3.0 / 128.0;
    } else {
        p.c[0] = -201.0 / 1024.0;  // c3 with the sign that makes the stencil exact on degree 5
        p.c[1] = 11.0 / 256.0;
        p.c[2] = -5.0 / 1024.0;
    }
    hipError_t st;
    auto dalloc = [&](void** ptr, size_t bytes) {
        st = hipMalloc(ptr, bytes);
        if (st == hipSuccess) r->allocs.push_back(*ptr);
        return st == hipSuccess;
    };
    auto fail = [&](const char* what) {
        const int code = fail2d(r, st, what);
        g_err2d = r->err;
        free2d(r);
        return code;
    };
    if (hip_stream) {
        r->stream = (hipStream_t)hip_stream;
    } else {
        if ((st = hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking)) != hipSuccess) return fail("hipStreamCreate");
        r->own_stream = true;
    }
    for (int l = p.jmin; l <= p.J; ++l) {
        const size_t nn = ((size_t)1 << l) << l;
        void* f = nullptr;
        if (!dalloc(&f, sizeof(double) * Q2 * nn)) return fail("hipMalloc(levels)");
        if ((st = hipMemsetAsync(f, 0, sizeof(double) * Q2 * nn, r->stream)) != hipSuccess) return fail("hipMemset");
        r->F.push_back(static_cast<double*>(f));
        if (l < p.J) {
            void* a[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
            for (int t = 0; t < 5; ++t)
                if (!dalloc(&a[t], nn)) return fail("hipMalloc(split)");
            r->split.push_back(static_cast<uint8_t*>(a[0]));
            r->nsplit.push_back(static_cast<uint8_t*>(a[1]));
            r->keep.push_back(static_cast<uint8_t*>(a[2]));
            r->ruleb.push_back(static_cast<uint8_t*>(a[3]));
            r->need.push_back(static_cast<uint8_t*>(a[4]));
            hipLaunchKernelGGL(k2_fill, dim3(blocks(nn)), dim3(256), 0, r->stream, r->split.back(), nn, (uint8_t)1);
        }
    }
    void *g0 = nullptr, *g1 = nullptr, *o = nullptr, *nl = nullptr, *nf = nullptr, *ud = nullptr;
    if (!dalloc(&g0, sizeof(double) * Q2 * NJ * NJ) || !dalloc(&g1, sizeof(double) * Q2 * NJ * NJ) ||
        !dalloc(&o, sizeof(double) * NJ * NJ) || !dalloc(&nl, 2 * sizeof(unsigned long long)) || !dalloc(&nf, sizeof(int)) ||
        !dalloc(&ud, sizeof(double) * NJ * NJ))
        return fail("hipMalloc(work)");
    r->G0 = static_cast<double*>(g0);
    r->G1 = static_cast<double*>(g1);
    r->out = static_cast<double*>(o);
    r->d_nleaf = static_cast<unsigned long long*>(nl);
    r->d_nan = static_cast<int*>(nf);
    if ((st = hipMemsetAsync(r->d_nan, 0, sizeof(int), r->stream)) != hipSuccess ||
        (st = hipMemsetAsync(r->d_nleaf, 0, 2 * sizeof(unsigned long long), r->stream)) != hipSuccess ||
        (st = hipMemcpyAsync(ud, u0, sizeof(double) * NJ * NJ, hipMemcpyHostToDevice, r->stream)) != hipSuccess)
        return fail("upload");
    hipLaunchKernelGGL(k2_init, dim3(blocks(NJ * NJ)), dim3(256), 0, r->stream, p, (const double*)ud, r->F.back());
    if ((st = hipStreamSynchronize(r->stream)) != hipSuccess) return fail("init");
    r->leaves = (long long)(NJ * NJ);
    mrlbm2d_t h = new (std::nothrow) mrlbm2d_s{r};
    if (!h) {
        free2d(r);
        return MRLBM_ENOMEM;
    }
    *out = h;
    return MRLBM_OK;
}

int mrlbm2d_step(mrlbm2d_t h, int32_t nsteps) {
    if (!h || nsteps < 0) return MRLBM_EINVAL;
    Run2D* r = h->r;
    if (r->numeric) return MRLBM_ENUMERIC;
    for (int t = 0; t < nsteps; ++t) {
        const int rc = step2d(r);
        if (rc != MRLBM_OK) return rc;
    }
    return finish2d(r);
}

int mrlbm2d_step_timed(mrlbm2d_t h, int32_t nsteps, float* ms) {
    if (!h || nsteps < 0 || !ms) return MRLBM_EINVAL;
    Run2D* r = h->r;
    if (r->numeric) return MRLBM_ENUMERIC;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t st = hipEventCreate(&a);
    if (st == hipSuccess) st = hipEventCreate(&b);
    if (st == hipSuccess) st = hipEventRecord(a, r->stream);
    int rc = st == hipSuccess ? MRLBM_OK : fail2d(r, st, "timing events");
    for (int t = 0; t < nsteps && rc == MRLBM_OK; ++t) rc = step2d(r);
    if (rc == MRLBM_OK && (st = hipEventRecord(b, r->stream)) != hipSuccess) rc = fail2d(r, st, "timing events");
    if (rc == MRLBM_OK) rc = finish2d(r);
    if ((rc == MRLBM_OK || rc == MRLBM_ENUMERIC) && hipEventElapsedTime(ms, a, b) != hipSuccess) *ms = 0.f;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return rc;
}

int mrlbm2d_moments(mrlbm2d_t h, double* out, int64_t cap) {
    if (!h || !out) return MRLBM_EINVAL;
    Run2D* r = h->r;
    if (r->numeric) return MRLBM_ENUMERIC;
    const P2& p = r->p;
    const size_t NJ = (size_t)1 << p.J;
    if (cap < (int64_t)(NJ * NJ)) return MRLBM_ECAPACITY;
    hipStream_t s = r->stream;
    const Lv2 L = levels2d(r);
    project2d(r, L);
    const double* ga = reconstruct2d(r, L, 0);
    hipLaunchKernelGGL(k2_moment, dim3(blocks(NJ * NJ)), dim3(256), 0, s, (int)NJ, (const double*)ga, r->out);
    hipError_t st = hipMemcpyAsync(out, r->out, sizeof(double) * NJ * NJ, hipMemcpyDeviceToHost, s);
    if (st == hipSuccess) st = hipStreamSynchronize(s);
    if (st != hipSuccess) return fail2d(r, st, "moments");
    return MRLBM_OK;
}

int mrlbm2d_split(mrlbm2d_t h, int32_t level, uint8_t* out, int64_t cap) {
    if (!h || !out) return MRLBM_EINVAL;
    Run2D* r = h->r;
    if (level < r->p.jmin || level >= r->p.J) return MRLBM_EINVAL;
    const size_t nn = ((size_t)1 << level) << level;
    if (cap < (int64_t)nn) return MRLBM_ECAPACITY;
    hipError_t st = hipMemcpyAsync(out, r->split[level - r->p.jmin], nn, hipMemcpyDeviceToHost, r->stream);
    if (st == hipSuccess) st = hipStreamSynchronize(r->stream);
    if (st != hipSuccess) return fail2d(r, st, "split");
    return MRLBM_OK;
}

int mrlbm2d_stats(mrlbm2d_t h, int64_t* steps, int64_t* leaves, int64_t* leaf_updates) {
    if (!h || !steps || !leaves || !leaf_updates) return MRLBM_EINVAL;
    *steps = h->r->steps;
    *leaves = h->r->leaves;
    *leaf_updates = h->r->leaf_updates;
    return MRLBM_OK;
}

void mrlbm2d_destroy(mrlbm2d_t h) {
    if (!h) return;
    if (h->r && h->r->stream) (void)hipStreamSynchronize(h->r->stream);
    free2d(h->r);
    delete h;
}

const char* mrlbm2d_last_error(mrlbm2d_t h) {
    if (!h) return g_err2d.c_str();
    return h->r->err.c_str();
}

}  // extern "C"
