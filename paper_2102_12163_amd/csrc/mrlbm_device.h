// mrlbm_device.h -- device-side building blocks of the MR-LBM step for CDNA4 (gfx950).
//
// Data layout of one run (home copy in HBM, owned by the host library):
//   values   two compact arrays of q planes x (2^(J+1) - 2^Jmin) slots of type T; the
//            cells of R(Lambda) occupy slots 0..#R-1, level by level (see rank_of).
//   split    one bit per cell of levels Jmin..J-1, "cell (l, p) has children"; 64-bit words,
//            levels below 64 cells use one partial word.
//   list     complete leaves of the current tree in spatial order, key (l << 27) | k.
//   pairs    reconstructed finest values on both sides of every leaf interface (used when
//            a run does not fit the workgroup's LDS).
//
// Inside a workgroup the tree lives in LDS as bit words; wavefront lane i owns bit i of a
// word, so a wave processes 64 cells of one level per iteration and __ballot turns 64
// per-lane decisions back into one word.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace mrl {

constexpr int MAXQ = 6;
constexpr int PERIODIC = 0;
constexpr int CLAMP = 1;
constexpr int ADVECTION = 0, BURGERS = 1, SHALLOW_WATER = 2, EULER = 3;

// Scheme constants, evaluated once on the host in double precision with the same
// expressions as the paper's formulas (see the host library for each one).
struct Coef {
    double lam, lam2, V, alam2, g2, gam, k3, gm1, k5;
    double lam3, lam4, blam2;  // D1Q5: lambda^3, lambda^4, beta lambda^2
    double s[MAXQ], oms[MAXQ];
    double ilam, ilam2;  // 1 / lam and 1 / lam^2 (exact when lam_pow2)
    double ilam3, ilam4; // 1 / lam^3 and 1 / lam^4 (exact when lam_pow2)
    int physics, qc;
    int lam_pow2;        // lam is a power of two: dividing by lam or lam^2 is an exact scaling
};

struct Desc {
    int jmin, jmax, gamma, mu_bar, bc, q, qc, nm;
    int recon;  // 1: reconstructed collision (Sec. 4.3.1), 0: leaves collision (Sec. 4.5)
    double eps;
    double c[3];
    Coef cf;
    void* va;
    void* vb;
    uint64_t* split;
    uint32_t* list;
    void* pairs;
    uint8_t* gtree;  // the run's tree arrays in device memory, for runs too large for LDS (else null)
    // refinement predictor (shared by the runs of a handle)
    const uint16_t* mlp;    // bfloat16 parameters, or null
    int pmode;              // 0 off, 1 learned rule (b) with judge, 2 record training samples
    int sample_cap;
    double gate;            // the network decides only pairs with D < gate * rule-(b) threshold
    float* samples;         // [sample_cap][33]: 32 features and the label
    unsigned int* nsamples;
};

struct State {
    long long steps, leaf_updates, n_leaves;
    int cur;    // which HBM value array holds the home copy
    int flags;  // bit 0: NaN met
    int n_r;    // #R(Lambda) of the current tree
    int pad;
    long long misses, redos;  // predictor: judged misses and redone steps
};

#define DEV __device__ __forceinline__

__host__ __device__ inline int nwords(int l) { return l >= 6 ? (1 << (l - 6)) : 1; }
// Number of words of the levels jmin..l-1: one word per level below 6, 2^(m-6) at level m >= 6.
__host__ __device__ inline int wbase(int jmin, int l) {
    int s = 0;
    const int e1 = l < 6 ? l : 6;
    if (e1 > jmin) s += e1 - jmin;
    const int b2 = jmin > 6 ? jmin : 6;
    if (l > b2) s += (1 << (l - 6)) - (1 << (b2 - 6));
    return s;
}

// Level of word index w of the level-major bit arrays (levels jmin..), and its index inside
// the level: levels below 6 hold one word each, level l >= 6 holds 2^(l-6) words.
DEV int level_of_word(int jmin, int w, int* lw) {
    const int small = jmin < 6 ? 6 - jmin : 0;
    if (w < small) {
        *lw = 0;
        return jmin + w;
    }
    const int m = w - small + (jmin > 6 ? (1 << (jmin - 6)) : 1);
    const int l = 6 + (31 - __clz(m));
    *lw = m - (1 << (l - 6));
    return l;
}

DEV int bcx(int i, int n, int bc) {
    if (bc == PERIODIC) return i & (n - 1);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

DEV uint64_t lowmask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

// 32 parent bits -> 64 child bits (each bit doubled).
// Bit i of a 16-bit value to bit 2i (32-bit operations: the compiler fuses each shift-or-mask
// step into one three-input bit operation).
DEV uint32_t spread16(uint32_t y) {
    y = (y | (y << 8)) & 0x00FF00FFu;
    y = (y | (y << 4)) & 0x0F0F0F0Fu;
    y = (y | (y << 2)) & 0x33333333u;
    y = (y | (y << 1)) & 0x55555555u;
    return y;
}
// 32 parent bits (low half of x) -> 64 child bits, each parent bit to both its children.
DEV uint64_t spread32(uint64_t x) {
    uint32_t lo = spread16((uint32_t)x & 0xFFFFu);
    uint32_t hi = spread16(((uint32_t)x) >> 16);
    lo |= lo << 1;
    hi |= hi << 1;
    return ((uint64_t)hi << 32) | lo;
}

// 32 child bits -> 16 parent bits (OR of each sibling pair).
DEV uint32_t compress32(uint32_t x) {
    uint32_t y = (x | (x >> 1)) & 0x55555555u;
    y = (y | (y >> 1)) & 0x33333333u;
    y = (y | (y >> 2)) & 0x0F0F0F0Fu;
    y = (y | (y >> 4)) & 0x00FF00FFu;
    y = (y | (y >> 8)) & 0x0000FFFFu;
    return y;
}
// 64 child bits -> 32 parent bits (OR of each sibling pair).
DEV uint64_t compress64(uint64_t x) {
    return (uint64_t)(compress32((uint32_t)x) | (compress32((uint32_t)(x >> 32)) << 16));
}

DEV bool getbit(const uint64_t* A, int wbl, int k) { return (A[wbl + (k >> 6)] >> (k & 63)) & 1ull; }

// Word w of R(Lambda) at level l: all of level Jmin, else the children of split cells.
DEV uint64_t r_word(const uint64_t* split, int jmin, int l, int w) {
    if (l == jmin) return lowmask(1 << l);
    uint64_t x = split[wbase(jmin, l - 1) + (w >> 1)] >> ((w & 1) * 32);
    return spread32(x);
}

// Word x of level l dilated by r cells, given its left and right neighbour words xl, xr
// (levels of at least 64 cells; zero for a clamped edge): bit i set iff some cell i + s,
// |s| <= r, is set. Levels of fewer than 64 cells are one word, wrapped or clamped in place.
DEV uint64_t dilate_val(uint64_t x, uint64_t xl, uint64_t xr, int l, int r, int bc) {
    const int N = 1 << l;
    uint64_t d = x;
    if (N >= 64) {
        for (int s = 1; s <= r; ++s) {
            d |= (x << s) | (xl >> (64 - s));
            d |= (x >> s) | (xr << (64 - s));
        }
    } else {
        const uint64_t m = lowmask(N);
        for (int s = 1; s <= r; ++s) {
            if (bc == PERIODIC) {
                const int sm = s % N;
                if (sm) {
                    d |= ((x << sm) | (x >> (N - sm))) & m;
                    d |= ((x >> sm) | (x << (N - sm))) & m;
                }
            } else {
                d |= (x << s) & m;
                d |= x >> s;
            }
        }
    }
    return d;
}

// Word w of level l dilated by r cells: bit i set iff some cell bc(i + s), |s| <= r, is set.
// Clamp reads as zero fill (the clamped neighbours add nothing beyond the cell itself).
DEV uint64_t dilate_word(const uint64_t* A, int wbl, int l, int w, int r, int bc) {
    const int N = 1 << l;
    const uint64_t x = A[wbl + w];
    uint64_t xl = 0ull, xr = 0ull;
    if (N >= 64) {
        const int nw = N >> 6;
        if (bc == PERIODIC) {
            xl = A[wbl + ((w - 1) & (nw - 1))];
            xr = A[wbl + ((w + 1) & (nw - 1))];
        } else {
            xl = w > 0 ? A[wbl + w - 1] : 0ull;
            xr = w < nw - 1 ? A[wbl + w + 1] : 0ull;
        }
    }
    return dilate_val(x, xl, xr, l, r, bc);
}

// Inclusive prefix sum over the 64 lanes of a wave with data-parallel-primitive moves:
// within each row of 16 lanes by shifts of 1, 2, 4 and 8 (lanes shifted in from outside the
// row read zero), then row 0's total into row 1 and row 2's into row 3 (row broadcast of lane
// 15), then the total of rows 0-1 into rows 2 and 3 (row broadcast of lane 31).
DEV uint32_t wave_scan(uint32_t x) {
    x += __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xF, 0xF, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xF, 0xF, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xF, 0xF, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xF, 0xF, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0u, x, 0x142, 0xA, 0xF, false);  // row_bcast:15, rows 1, 3
    x += __builtin_amdgcn_update_dpp(0u, x, 0x143, 0xC, 0xF, false);  // row_bcast:31, rows 2, 3
    return x;
}

// 64-bit value of the previous lane (lane 0: zero) and of the next lane (lane 63: zero), by
// whole-wave DPP shifts; the 32-bit value of the other lane of each even/odd lane pair.
DEV uint64_t from_prev_lane(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)v, 0x138, 0xF, 0xF, false);  // wave_shr:1
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(v >> 32), 0x138, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}
DEV uint64_t from_next_lane(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)v, 0x130, 0xF, 0xF, false);  // wave_shl:1
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(v >> 32), 0x130, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}
DEV uint32_t from_pair_lane(uint32_t v) {
    return __builtin_amdgcn_update_dpp(0u, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
}

// Lane src's 64-bit value, as a wave-uniform value (src uniform).
DEV uint64_t readlane64(uint64_t v, int src) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, src);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// 64-bit lane exchange inside a wave (two 32-bit halves).
DEV uint64_t shfl64(uint64_t v, int src) {
    const int lo = __shfl((int)(uint32_t)v, src, 64);
    const int hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// ------------------------------------------------------------------ schemes
// Population order: D1Q2 (+lambda, -lambda); D1Q3 (0, +lambda, -lambda); D1Q2^k blocks
// (+lambda, -lambda) per conserved quantity; D1Q5 (0, lambda, -lambda, 2 lambda, -2 lambda).
// Q populations, NM of them moving (mv(m): population of the m-th moving one), w(h) the
// velocity of population h in units of lambda, SIG = max |w| (the stencil radius sigma).
template <int S> struct Sch;
template <> struct Sch<0> {
    static constexpr int Q = 2, NM = 2, SIG = 1;
    __host__ __device__ static constexpr int mv(int m) { return m; }
    __host__ __device__ static constexpr int w(int h) { return h == 0 ? 1 : -1; }
};
template <> struct Sch<1> {
    static constexpr int Q = 3, NM = 2, SIG = 1;
    __host__ __device__ static constexpr int mv(int m) { return m + 1; }
    __host__ __device__ static constexpr int w(int h) { return h == 0 ? 0 : (h == 1 ? 1 : -1); }
};
template <> struct Sch<2> {
    static constexpr int Q = 4, NM = 4, SIG = 1;
    __host__ __device__ static constexpr int mv(int m) { return m; }
    __host__ __device__ static constexpr int w(int h) { return (h & 1) ? -1 : 1; }
};
template <> struct Sch<3> {
    static constexpr int Q = 6, NM = 6, SIG = 1;
    __host__ __device__ static constexpr int mv(int m) { return m; }
    __host__ __device__ static constexpr int w(int h) { return (h & 1) ? -1 : 1; }
};
template <> struct Sch<4> {
    static constexpr int Q = 5, NM = 4, SIG = 2;
    __host__ __device__ static constexpr int mv(int m) { return m + 1; }
    __host__ __device__ static constexpr int w(int h) { return h == 0 ? 0 : (h == 1 ? 1 : (h == 2 ? -1 : (h == 3 ? 2 : -2))); }
};

// The stream of a leaf reads, for each moving population h and delta = 1..|w^h|, the
// reconstructed finest value at e + eta(h, delta) on both of its interfaces e (eq.
// AdaptiveStreamPhase; eta = -delta for w^h > 0, delta - 1 for w^h < 0). The interface
// values are stored as planes: moving population m owns |w| consecutive planes from
// plane_base(m), one per delta; PL planes in all.
template <int S> struct Planes {
    __host__ __device__ static constexpr int aw(int m) { return Sch<S>::w(Sch<S>::mv(m)) < 0 ? -Sch<S>::w(Sch<S>::mv(m))
                                                                               : Sch<S>::w(Sch<S>::mv(m)); }
    __host__ __device__ static constexpr int base(int m) { return m == 0 ? 0 : base(m - 1) + aw(m - 1); }
    static constexpr int PL = base(Sch<S>::NM);
    // offset of the finest cell of (m, delta) from the interface, eta(h, delta)
    __host__ __device__ static constexpr int eta(int m, int delta) { return Sch<S>::w(Sch<S>::mv(m)) > 0 ? -delta : delta - 1; }
};

template <int S> struct MovingPops { DEV static constexpr int h(int m) { return Sch<S>::mv(m); } };
template <int S> struct AllPops { DEV static constexpr int h(int m) { return m; } };

// Leaves collision (Sec. 4.5, eq. LeavesCollision) with the equilibria of Sec. 5: the
// conserved moments stay, every other moment relaxes m* = (1 - s) m + s m_eq. The
// expression order is fixed (it is the order the FP64 checks were written against).
// x / d; when d is a power of two, x * (1 / d) instead: the same correctly rounded value
// (both are the exact scaling of x), without the division sequence.
template <typename T>
DEV T div_by(T x, T d, T inv, bool pow2) {
    if (pow2) return x * inv;
    return x / d;
}

// D1Q5 (Sec. 5.2.1): the moments of f and the populations of moments (m0, m1, m2, m3, m4),
// through the even parts a = f1 + f2, b = f3 + f4 and the odd parts c = f1 - f2, d = f3 - f4.
template <typename T>
DEV void q5_moments(const Coef& c, const T* f, T* m) {
    m[0] = (((f[0] + f[1]) + f[2]) + f[3]) + f[4];
    m[1] = (T)c.lam * ((f[1] - f[2]) + (T)2 * (f[3] - f[4]));
    m[2] = (T)c.lam2 * ((f[1] + f[2]) + (T)4 * (f[3] + f[4]));
    m[3] = (T)c.lam3 * ((f[1] - f[2]) + (T)8 * (f[3] - f[4]));
    m[4] = (T)c.lam4 * ((f[1] + f[2]) + (T)16 * (f[3] + f[4]));
}
template <typename T>
DEV void q5_equilibria(const Coef& c, T m0, T m1, T* eq) {
    eq[0] = (m1 * m1) / m0 + (T)c.g2 * (m0 * m0);
    eq[1] = (T)c.alam2 * m1;
    eq[2] = (T)c.blam2 * eq[0];
}
template <typename T>
DEV void q5_populations(const Coef& c, T m0, T m1, T m2, T m3, T m4, T* f) {
    const bool p2 = c.lam_pow2 != 0;
    const T p1 = div_by(m1, (T)c.lam, (T)c.ilam, p2);
    const T q2 = div_by(m2, (T)c.lam2, (T)c.ilam2, p2);
    const T q3 = div_by(m3, (T)c.lam3, (T)c.ilam3, p2);
    const T q4 = div_by(m4, (T)c.lam4, (T)c.ilam4, p2);
    const T b = (q4 - q2) / (T)12;
    const T a = q2 - (T)4 * b;
    const T d = (q3 - p1) / (T)6;
    const T cc = p1 - (T)2 * d;
    const T half = (T)0.5;
    f[0] = (m0 - a) - b;
    f[1] = half * (a + cc);
    f[2] = half * (a - cc);
    f[3] = half * (b + d);
    f[4] = half * (b - d);
}
// relaxation of m2, m3, m4 towards eq (conserved m0, m1 stay)
template <typename T>
DEV void q5_relax(const Coef& c, T* f, const T* eq) {
    T m[5];
    q5_moments(c, f, m);
    const T m2s = (T)c.oms[0] * m[2] + (T)c.s[0] * eq[0];
    const T m3s = (T)c.oms[1] * m[3] + (T)c.s[1] * eq[1];
    const T m4s = (T)c.oms[2] * m[4] + (T)c.s[2] * eq[2];
    q5_populations(c, m[0], m[1], m2s, m3s, m4s, f);
}

template <typename T, int S>
DEV void collide(const Coef& c, T* f) {
    const T lam = (T)c.lam;
    const T ilam = (T)c.ilam;
    const bool p2 = c.lam_pow2 != 0;
    const T half = (T)0.5;
    if constexpr (S == 4) {
        T m[5], eq[3];
        q5_moments(c, f, m);
        q5_equilibria(c, m[0], m[1], eq);
        q5_relax(c, f, eq);
        (void)lam;
        (void)ilam;
        (void)p2;
        (void)half;
    } else if constexpr (S == 0) {
        const T u = f[0] + f[1];
        const T m1 = lam * (f[0] - f[1]);
        const T eq = c.physics == ADVECTION ? (T)c.V * u : (u * u) * half;
        const T m1s = (T)c.oms[0] * m1 + (T)c.s[0] * eq;
        const T r = div_by(m1s, lam, ilam, p2);
        f[0] = half * (u + r);
        f[1] = half * (u - r);
    } else if constexpr (S == 1) {
        const T lam2 = (T)c.lam2;
        const T m0 = (f[0] + f[1]) + f[2];
        const T m1 = lam * (f[1] - f[2]);
        const T m2 = lam2 * (f[1] + f[2]);
        T m1s, m2s;
        if (c.physics == BURGERS) {
            const T eq1 = (m0 * m0) * half;
            const T eq2 = (T)c.alam2 * m0;
            m1s = (T)c.oms[0] * m1 + (T)c.s[0] * eq1;
            m2s = (T)c.oms[1] * m2 + (T)c.s[1] * eq2;
        } else {
            const T eq2 = (m1 * m1) / m0 + (T)c.g2 * (m0 * m0);
            m1s = m1;
            m2s = (T)c.oms[0] * m2 + (T)c.s[0] * eq2;
        }
        const T a = div_by(m2s, lam2, (T)c.ilam2, p2);
        const T b = div_by(m1s, lam, ilam, p2);
        f[0] = m0 - a;
        f[1] = half * (a + b);
        f[2] = half * (a - b);
    } else {
        constexpr int NB = Sch<S>::Q / 2;
        T cc[NB], eq[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) cc[b] = f[2 * b] + f[2 * b + 1];
        if constexpr (S == 2) {
            eq[0] = cc[1];
            eq[1] = (cc[1] * cc[1]) / cc[0] + (T)c.g2 * (cc[0] * cc[0]);
        } else {
            eq[0] = cc[1];
            eq[1] = (T)c.k3 * ((cc[1] * cc[1]) / cc[0]) + (T)c.gm1 * cc[2];
            eq[2] = (T)c.gam * ((cc[2] * cc[1]) / cc[0]) + (T)c.k5 * (((cc[1] * cc[1]) * cc[1]) / (cc[0] * cc[0]));
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const T n = lam * (f[2 * b] - f[2 * b + 1]);
            const T ns = (T)c.oms[b] * n + (T)c.s[b] * eq[b];
            const T r = div_by(ns, lam, ilam, p2);
            f[2 * b] = half * (cc[b] + r);
            f[2 * b + 1] = half * (cc[b] - r);
        }
    }
}

// Number of non-conserved moments with an equilibrium (at most, for D1Q3: 2 for Burgers,
// 1 for shallow water).
template <int S> struct NEq { static constexpr int N = S == 0 ? 1 : ((S == 3 || S == 4) ? 3 : 2); };

// Equilibria of the non-conserved moments from the conserved moments of f, with the
// expressions of collide (Sec. 5).
template <typename T, int S>
DEV void eq_moments(const Coef& c, const T* f, T* eq) {
    const T half = (T)0.5;
    if constexpr (S == 4) {
        T m[5];
        q5_moments(c, f, m);
        q5_equilibria(c, m[0], m[1], eq);
        (void)half;
    } else if constexpr (S == 0) {
        const T u = f[0] + f[1];
        eq[0] = c.physics == ADVECTION ? (T)c.V * u : (u * u) * half;
    } else if constexpr (S == 1) {
        const T m0 = (f[0] + f[1]) + f[2];
        if (c.physics == BURGERS) {
            eq[0] = (m0 * m0) * half;
            eq[1] = (T)c.alam2 * m0;
        } else {
            const T m1 = (T)c.lam * (f[1] - f[2]);
            eq[0] = (m1 * m1) / m0 + (T)c.g2 * (m0 * m0);
            eq[1] = (T)0;
        }
    } else {
        constexpr int NB = Sch<S>::Q / 2;
        T cc[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) cc[b] = f[2 * b] + f[2 * b + 1];
        if constexpr (S == 2) {
            eq[0] = cc[1];
            eq[1] = (cc[1] * cc[1]) / cc[0] + (T)c.g2 * (cc[0] * cc[0]);
        } else {
            eq[0] = cc[1];
            eq[1] = (T)c.k3 * ((cc[1] * cc[1]) / cc[0]) + (T)c.gm1 * cc[2];
            eq[2] = (T)c.gam * ((cc[2] * cc[1]) / cc[0]) + (T)c.k5 * (((cc[1] * cc[1]) * cc[1]) / (cc[0] * cc[0]));
        }
    }
}

// collide with the non-conserved moments relaxed towards the given equilibria eq instead of
// f's own (Sec. 4.3.1, eq. reconstructedCollision, where eq is a leaf's mean over its finest
// cells); the conserved moments stay. relax_to(c, f, eq_moments(c, f)) is collide(c, f).
template <typename T, int S>
DEV void relax_to(const Coef& c, T* f, const T* eq) {
    const T lam = (T)c.lam;
    const T ilam = (T)c.ilam;
    const bool p2 = c.lam_pow2 != 0;
    const T half = (T)0.5;
    if constexpr (S == 4) {
        q5_relax(c, f, eq);
        (void)lam;
        (void)ilam;
        (void)p2;
        (void)half;
    } else if constexpr (S == 0) {
        const T u = f[0] + f[1];
        const T m1 = lam * (f[0] - f[1]);
        const T m1s = (T)c.oms[0] * m1 + (T)c.s[0] * eq[0];
        const T r = div_by(m1s, lam, ilam, p2);
        f[0] = half * (u + r);
        f[1] = half * (u - r);
    } else if constexpr (S == 1) {
        const T lam2 = (T)c.lam2;
        const T m0 = (f[0] + f[1]) + f[2];
        const T m1 = lam * (f[1] - f[2]);
        const T m2 = lam2 * (f[1] + f[2]);
        T m1s, m2s;
        if (c.physics == BURGERS) {
            m1s = (T)c.oms[0] * m1 + (T)c.s[0] * eq[0];
            m2s = (T)c.oms[1] * m2 + (T)c.s[1] * eq[1];
        } else {
            m1s = m1;
            m2s = (T)c.oms[0] * m2 + (T)c.s[0] * eq[0];
        }
        const T a = div_by(m2s, lam2, (T)c.ilam2, p2);
        const T b = div_by(m1s, lam, ilam, p2);
        f[0] = m0 - a;
        f[1] = half * (a + b);
        f[2] = half * (a - b);
    } else {
        constexpr int NB = Sch<S>::Q / 2;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const T cb = f[2 * b] + f[2 * b + 1];
            const T n = lam * (f[2 * b] - f[2 * b + 1]);
            const T ns = (T)c.oms[b] * n + (T)c.s[b] * eq[b];
            const T r = div_by(ns, lam, ilam, p2);
            f[2 * b] = half * (cb + r);
            f[2 * b + 1] = half * (cb - r);
        }
    }
}

// Populations at equilibrium for the conserved moments mc (Sec. 2.1.1, initial datum).
template <typename T, int S>
DEV void equilibrium(const Coef& c, const double* mc, T* f) {
    const double lam = c.lam;
    if constexpr (S == 4) {
        double eq[3], g[5];
        q5_equilibria<double>(c, mc[0], mc[1], eq);
        q5_populations<double>(c, mc[0], mc[1], eq[0], eq[1], eq[2], g);
        for (int h = 0; h < 5; ++h) f[h] = (T)g[h];
        (void)lam;
    } else if constexpr (S == 0) {
        const double u = mc[0];
        const double eq = c.physics == ADVECTION ? c.V * u : (u * u) * 0.5;
        const double r = eq / lam;
        f[0] = (T)(0.5 * (u + r));
        f[1] = (T)(0.5 * (u - r));
    } else if constexpr (S == 1) {
        const double m0 = mc[0];
        double eq1, eq2;
        if (c.physics == BURGERS) {
            eq1 = (m0 * m0) * 0.5;
            eq2 = c.alam2 * m0;
        } else {
            eq1 = mc[1];
            eq2 = (eq1 * eq1) / m0 + c.g2 * (m0 * m0);
        }
        const double a = eq2 / c.lam2;
        const double b = eq1 / lam;
        f[0] = (T)(m0 - a);
        f[1] = (T)(0.5 * (a + b));
        f[2] = (T)(0.5 * (a - b));
    } else {
        constexpr int NB = Sch<S>::Q / 2;
        double eq[NB];
        if constexpr (S == 2) {
            eq[0] = mc[1];
            eq[1] = (mc[1] * mc[1]) / mc[0] + c.g2 * (mc[0] * mc[0]);
        } else {
            eq[0] = mc[1];
            eq[1] = c.k3 * ((mc[1] * mc[1]) / mc[0]) + c.gm1 * mc[2];
            eq[2] = c.gam * ((mc[2] * mc[1]) / mc[0]) + c.k5 * (((mc[1] * mc[1]) * mc[1]) / (mc[0] * mc[0]));
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const double r = eq[b] / lam;
            f[2 * b] = (T)(0.5 * (mc[b] + r));
            f[2 * b + 1] = (T)(0.5 * (mc[b] - r));
        }
    }
}

// Conserved moments of one cell, evaluated in double.
template <typename T, int S>
DEV void conserved(const Coef& c, const T* f, double* mc) {
    if constexpr (S == 4) {
        double g[5], m[5];
        for (int h = 0; h < 5; ++h) g[h] = (double)f[h];
        q5_moments<double>(c, g, m);
        mc[0] = m[0];
        mc[1] = m[1];
    } else if constexpr (S == 0) {
        mc[0] = (double)f[0] + (double)f[1];
    } else if constexpr (S == 1) {
        mc[0] = ((double)f[0] + (double)f[1]) + (double)f[2];
        if (c.qc == 2) mc[1] = c.lam * ((double)f[1] - (double)f[2]);
    } else {
        constexpr int NB = Sch<S>::Q / 2;
#pragma unroll
        for (int b = 0; b < NB; ++b) mc[b] = (double)f[2 * b] + (double)f[2 * b + 1];
    }
}

// ------------------------------------------------------------------ compact storage
// Values of one tree are stored compactly: the cells of R(Lambda) are numbered level by
// level and, inside a level, by index (their "slot"); population h of slot s lives at
// p[h * stride + s]. R holds the R(Lambda) bits per 64-bit word and RP the number of
// R(Lambda) cells in all words before a word, so slot(l, k) = RP[w] + popcount of the R
// bits below k in its word w.
DEV int rank_of(const uint64_t* R, const uint32_t* RP, int jmin, int l, int k) {
    const int w = wbase(jmin, l) + (k >> 6);
    return (int)RP[w] + __popcll(R[w] & ((1ull << (k & 63)) - 1ull));
}
// Number of set bits of x below the calling lane's index (masked bit count).
DEV uint32_t popc_below_lane(uint64_t x) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(x >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)x, 0u));
}
// rank_of for the cell (l, 64 w + lane) of the calling lane.
DEV int rank_lane(const uint64_t* R, const uint32_t* RP, int jmin, int l, int w) {
    const int wi = wbase(jmin, l) + w;
    return (int)RP[wi] + (int)popc_below_lane(R[wi]);
}
DEV bool rbit(const uint64_t* R, int jmin, int l, int k) { return (R[wbase(jmin, l) + (k >> 6)] >> (k & 63)) & 1ull; }

template <typename T, typename P>
struct VP {
    P* p;
    int stride;
    DEV T ld(int h, int s) const { return (T)p[h * stride + s]; }
    DEV void st(int h, int s, T v) const { p[h * stride + s] = v; }
};

// ------------------------------------------------------------------ reconstruction
// Reconstructed values f-double-hat at the cells tA..tB (tB - tA <= 4 gamma) of level L
// (Sec. 3.3, reconstruction operator): starting at level L, a window of cells is followed
// towards coarser levels until every cell of the window lies in R(Lambda); then, level by
// level back to L, every window cell outside R(Lambda) is predicted from the parent level's
// window (Sec. 3.1) and every cell inside R(Lambda) takes its stored value. With unwrapped
// indices the level-l window is [((tA + 2G) >> (L - l)) - 2G, ((tB - 2G) >> (L - l)) + 2G], so
// a window position's parent position depends only on the parity of (tA + 2G) >> (L - l):
// the whole window stays in registers. Out-of-range cells under clamp copy the edge cell.
// Under clamp the targets must already be in range.
// c ? a : b on the values (a select of two registers, never a select of their addresses,
// which would keep a register array in scratch memory)
template <typename T>
DEV T pick(bool c, T a, T b) {
    typedef typename std::conditional<sizeof(T) == 8, unsigned long long, unsigned int>::type U;
    U ua, ub;
    __builtin_memcpy(&ua, &a, sizeof(T));
    __builtin_memcpy(&ub, &b, sizeof(T));
    const U m = c ? ~(U)0 : (U)0;
    const U r = (ua & m) | (ub & ~m);
    T out;
    __builtin_memcpy(&out, &r, sizeof(T));
    return out;
}

template <typename T, int G, int NP, class PM, int NO, class V>
DEV void chain(const V& Vx, const uint64_t* R, const uint32_t* RP, int jmin, int L, int bc, const T* cc, int tA,
               int tB, T* out, int lstart) {
    static_assert(NO <= 4 * G + 1, "the window holds at most 4 gamma + 1 cells");
    constexpr int WM = 4 * G + 1;
    // descent: the finest level whose whole window lies in R(Lambda); no level above lstart
    // qualifies (the caller knows a window cell there lies below a leaf)
    int l0 = lstart < L ? lstart : L;
    while (l0 > jmin) {
        const int sh = L - l0;
        const int lo = ((tA + 2 * G) >> sh) - 2 * G;
        const int hi = ((tB - 2 * G) >> sh) + 2 * G;
        const int N = 1 << l0;
        const int wbl = wbase(jmin, l0);
        bool all = true;
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            if (i <= hi - lo) {
                const int xx = bcx(lo + i, N, bc);
                all = all && ((R[wbl + (xx >> 6)] >> (xx & 63)) & 1ull);
            }
        }
        if (all) break;
        --l0;
    }
    T win[NP][WM];
    {
        const int sh = L - l0;
        const int lo = ((tA + 2 * G) >> sh) - 2 * G;
        const int hi = ((tB - 2 * G) >> sh) + 2 * G;
        const int N = 1 << l0;
        const int wbl = wbase(jmin, l0);
        if (lo >= 0 && hi < N) {
            // every window cell lies in R (the descent's condition, or level jmin) and R is
            // ranked by index within a level: one rank, then consecutive slots
            const int w = wbl + (lo >> 6);
            const int s0 = (int)RP[w] + __popcll(R[w] & ((1ull << (lo & 63)) - 1ull));
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                const bool ok = i <= hi - lo;
#pragma unroll
                for (int m = 0; m < NP; ++m) win[m][i] = ok ? Vx.ld(PM::h(m), s0 + i) : (T)0;
            }
        } else {
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                const int xx = bcx(lo + i, N, bc);
                const int w = wbl + (xx >> 6);
                const uint64_t rw = R[w];
                const bool ok = (i <= hi - lo) && ((rw >> (xx & 63)) & 1ull);
                const int s = ok ? (int)RP[w] + __popcll(rw & ((1ull << (xx & 63)) - 1ull)) : 0;
#pragma unroll
                for (int m = 0; m < NP; ++m) win[m][i] = ok ? Vx.ld(PM::h(m), s) : (T)0;
            }
        }
    }
    // ascent; once a window level holds no cell of R(Lambda), no finer window level does
    // (their parents lie inside it), and the rest is prediction only. The levels below L carry
    // the whole window; level L, taken after the loop by every lane at once, only the NO
    // output cells (tA .. tB, in range under clamp).
    bool anyr = true;
    for (int l = l0 + 1; l < L; ++l) {
        const int sh = L - l;
        const int u = (tA + 2 * G) >> sh;
        const int lo = u - 2 * G;
        const int hi = ((tB - 2 * G) >> sh) + 2 * G;
        const int N = 1 << l;
        const bool par = (u & 1) != 0;
        // children of the parents at window positions G..3G (prediction, Sec. 3.1): the even
        // child of parent G + j is kid[2j] = f + corr, the odd one kid[2j+1] = f - corr, and
        // window position i of this level is kid[i + parity]
        T kid[NP][WM + 1];
#pragma unroll
        for (int m = 0; m < NP; ++m)
#pragma unroll
            for (int j = 0; j <= 2 * G; ++j) {
                T acc = (T)0;
#pragma unroll
                for (int a = 1; a <= G; ++a) {
                    const T t = cc[a - 1] * (win[m][G + j + a] - win[m][G + j - a]);
                    acc = (a == 1) ? t : acc + t;
                }
                kid[m][2 * j] = win[m][G + j] + acc;
                kid[m][2 * j + 1] = win[m][G + j] - acc;
            }
        T nw[NP][WM];
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int m = 0; m < NP; ++m) nw[m][i] = pick(par, kid[m][i + 1], kid[m][i]);
        // window cells inside R(Lambda) take their stored values instead
        bool any = false;
        if (anyr) {
            const int wbl = wbase(jmin, l);
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                if (i <= hi - lo) {
                    const int xx = bcx(lo + i, N, bc);
                    const int w = wbl + (xx >> 6);
                    const uint64_t rw = R[w];
                    if ((rw >> (xx & 63)) & 1ull) {
                        any = true;
                        const int s = (int)RP[w] + __popcll(rw & ((1ull << (xx & 63)) - 1ull));
#pragma unroll
                        for (int m = 0; m < NP; ++m) nw[m][i] = Vx.ld(PM::h(m), s);
                    }
                }
            }
        }
        anyr = any;
        if (bc == CLAMP && (lo < 0 || hi >= N)) {
            const int e0 = -lo, e1 = N - 1 - lo;
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                const int x = lo + i;
                if (x < 0 || x >= N) {
                    const int src = x < 0 ? e0 : e1;
#pragma unroll
                    for (int m = 0; m < NP; ++m) {
                        T v = nw[m][0];
#pragma unroll
                        for (int j = 1; j < WM; ++j) v = (src == j) ? nw[m][j] : v;
                        nw[m][i] = v;
                    }
                }
            }
        }
#pragma unroll
        for (int m = 0; m < NP; ++m)
#pragma unroll
            for (int i = 0; i < WM; ++i) win[m][i] = nw[m][i];
    }
    if (l0 < L) {
        // level L: window position i is cell tA + i (lo = tA); its children come from the
        // parents at window positions G .. G + NO / 2 of level L - 1, the same arithmetic
        const int u = tA + 2 * G;
        const bool par = (u & 1) != 0;
        constexpr int NPAR = NO / 2 + 1;  // parents whose children reach positions 0 .. NO
        static_assert(NPAR <= 2 * G + 1, "the outputs lie inside the window");
        T kid[NP][2 * NPAR];
#pragma unroll
        for (int m = 0; m < NP; ++m)
#pragma unroll
            for (int j = 0; j < NPAR; ++j) {
                T acc = (T)0;
#pragma unroll
                for (int a = 1; a <= G; ++a) {
                    const T t = cc[a - 1] * (win[m][G + j + a] - win[m][G + j - a]);
                    acc = (a == 1) ? t : acc + t;
                }
                kid[m][2 * j] = win[m][G + j] + acc;
                kid[m][2 * j + 1] = win[m][G + j] - acc;
            }
        T nw[NP][NO];
#pragma unroll
        for (int i = 0; i < NO; ++i)
#pragma unroll
            for (int m = 0; m < NP; ++m) nw[m][i] = pick(par, kid[m][i + 1], kid[m][i]);
        if (anyr) {
            const int N = 1 << L;
            const int wbl = wbase(jmin, L);
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                const int xx = bcx(tA + i, N, bc);
                const int w = wbl + (xx >> 6);
                const uint64_t rw = R[w];
                if ((rw >> (xx & 63)) & 1ull) {
                    const int s = (int)RP[w] + __popcll(rw & ((1ull << (xx & 63)) - 1ull));
#pragma unroll
                    for (int m = 0; m < NP; ++m) nw[m][i] = Vx.ld(PM::h(m), s);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < NP; ++m)
#pragma unroll
            for (int j = 0; j < NO; ++j) out[m * NO + j] = nw[m][j];
    } else {
        // window position j is cell tA + j of level L (positions beyond tB - tA are not
        // meaningful)
#pragma unroll
        for (int m = 0; m < NP; ++m)
#pragma unroll
            for (int j = 0; j < NO; ++j) out[m * NO + j] = win[m][j];
    }
}

}  // namespace mrl
