// mrlbm_kernels.h -- the per-run workgroup engine: every phase of an MR-LBM time step as a
// block-cooperative function, and the kernels built from them.
//
// One workgroup advances one run (one instance of a batch); phases are separated by
// workgroup barriers only, so a launch of K steps for B runs is a single grid of B
// workgroups with no inter-workgroup synchronization.
#pragma once

#include "mrlbm_device.h"

namespace mrl {

enum : int { MODE_ADAPT = 1, MODE_SCHEME = 2 };

template <typename T, int S, int G>
struct Block {
    static constexpr int Q = Sch<S>::Q;
    static constexpr int NM = Sch<S>::NM;

    const Desc& d;
    int tid, NT, lane, wave, nwaves;
    int jmin, J, bc;
    int* wb;             // word base per level (LDS)
    uint64_t* split;     // current tree bits, levels jmin..J (LDS)
    uint64_t* nsplit;    // next tree bits
    uint64_t* keep;      // T_eps result
    uint64_t* ruleb;     // enlargement rule (b) hits
    uint64_t* E;         // finest-level leaf left edges
    uint32_t* scan;      // exclusive prefix of E popcounts
    uint32_t* red;       // small reduction scratch (one per wave + extras)
    T cc[3];

    DEV Block(const Desc& dd, int* wb_, uint64_t* lds, uint32_t* red_) : d(dd), wb(wb_), red(red_) {
        tid = threadIdx.x;
        NT = blockDim.x;
        lane = tid & 63;
        wave = tid >> 6;
        nwaves = NT >> 6;
        jmin = d.jmin;
        J = d.jmax;
        bc = d.bc;
        const int wt = wbase(jmin, J + 1);
        split = lds;
        nsplit = split + wt;
        keep = nsplit + wt;
        ruleb = keep + wt;
        E = ruleb + wt;
        const int nwJ = nwords(J);
        scan = reinterpret_cast<uint32_t*>(E + nwJ);
        for (int a = 0; a < 3; ++a) cc[a] = (T)d.c[a];
    }

    DEV int wtot() const { return wbase(jmin, J + 1); }

    // ----------------------------------------------------------- A1 / B2: projection
    // Every split cell takes half the sum of its two children, finest level first
    // (Sec. 3.1, Definition Projection operator).
    DEV void project_up(const Vals<T>& V) {
        for (int l = J - 1; l >= jmin; --l) {
            const int nw = nwords(l);
            for (int w = wave; w < nw; w += nwaves) {
                const uint64_t bits = split[wb[l] + w];
                if (!bits) continue;
                if ((bits >> lane) & 1ull) {
                    const int p = (w << 6) + lane;
#pragma unroll
                    for (int h = 0; h < Q; ++h)
                        V.at(l, h, p) = (T)0.5 * (V.at(l + 1, h, 2 * p) + V.at(l + 1, h, 2 * p + 1));
                }
            }
            __syncthreads();
        }
    }

    // ----------------------------------------------------------- A2-A4(b): details
    // For every split cell (l, p): d^h = f_{l+1,2p} - (f_{l,p} + sum_a c_a (f_{l,p+a} - f_{l,p-a}))
    // in double (Sec. 3.1-3.2), D = max_h |d^h|; keep iff D >= eps_{l+1} (Sec. 3.4, T_eps);
    // rule (b) iff kept, l+1 < J and D >= 2^(mu+1) eps_{l+1} (Sec. 4.2). One wave per word;
    // the 64 lane decisions become the keep / ruleb words through __ballot.
    DEV void details(const Vals<T>& V, int* nanflag) {
        int t = wave;
        for (int l = jmin; l < J; ++l) {
            const int nw = nwords(l);
            const int N = 1 << l;
            const double thr = ldexp(d.eps, l + 1 - J);
            const double thrb = ldexp(d.eps, d.mu_bar + 1 + l + 1 - J);
            const bool rb_level = (l + 1 < J);
            for (; t < nw; t += nwaves) {
                const uint64_t bits = split[wb[l] + t];
                uint64_t kw = 0, rw = 0;
                if (bits) {
                    bool kb = false, rbb = false;
                    if ((bits >> lane) & 1ull) {
                        const int p = (t << 6) + lane;
                        double D = 0.0;
                        bool bad = false;
#pragma unroll
                        for (int h = 0; h < Q; ++h) {
                            const double f0 = (double)V.at(l, h, p);
                            double acc = 0.0;
#pragma unroll
                            for (int a = 1; a <= G; ++a) {
                                const double fp = (double)V.at(l, h, bcx(p + a, N, bc));
                                const double fm = (double)V.at(l, h, bcx(p - a, N, bc));
                                const double tt = d.c[a - 1] * (fp - fm);
                                acc = (a == 1) ? tt : acc + tt;
                            }
                            const double pred = f0 + acc;
                            const double dd = (double)V.at(l + 1, h, 2 * p) - pred;
                            const double ad = fabs(dd);
                            bad = bad || (ad != ad);
                            D = ad > D ? ad : D;
                        }
                        if (bad) *nanflag = 1;
                        kb = bad || (D >= thr);
                        rbb = kb && rb_level && (bad || D >= thrb);
                    }
                    kw = __ballot(kb);
                    rw = __ballot(rbb);
                }
                if (lane == 0) {
                    keep[wb[l] + t] = kw;
                    ruleb[wb[l] + t] = rw;
                }
            }
            t -= nw;
        }
    }

    // ----------------------------------------------------------- A4: enlargement
    // Rule (a): every cell of R(T_eps) at level l+1 puts its neighbours within sigma into R,
    // i.e. their parents split: a dilation of keep[l] by ceil(sigma/2) at level l. Rule (b):
    // both children of a flagged cell are split. Levels below J only.
    DEV void enlarge() {
        const int ra = 1;  // ceil(sigma / 2) for sigma = 1 (every built-in scheme)
        int t = tid;
        for (int l = jmin; l <= J; ++l) {
            const int nw = nwords(l);
            for (; t < nw; t += NT) {
                uint64_t v = 0;
                if (l < J) {
                    v = dilate_word(keep, wb[l], l, t, ra, bc);
                    if (l > jmin) {
                        const uint64_t pb = ruleb[wb[l - 1] + (t >> 1)] >> ((t & 1) * 32);
                        v |= spread32(pb);
                    }
                }
                nsplit[wb[l] + t] = v;
            }
            t -= nw;
        }
        __syncthreads();
    }

    // ----------------------------------------------------------- A5: grading
    // Smallest graded tree (Sec. 3.3): a split cell (a, p), a > Jmin, needs (a, p + delta),
    // |delta| <= gamma, in R, so the parents of those cells are split. One sweep from the
    // finest level; delta = 0 also restores the tree property.
    DEV void grade() {
        for (int a = J - 1; a > jmin; --a) {
            const int pnw = nwords(a - 1);
            const int cnw = nwords(a);
            for (int pw = tid; pw < pnw; pw += NT) {
                const int c0 = 2 * pw, c1 = 2 * pw + 1;
                uint64_t v = 0;
                if (c0 < cnw) v |= compress64(dilate_word(nsplit, wb[a], a, c0, G, bc));
                if (c1 < cnw) v |= compress64(dilate_word(nsplit, wb[a], a, c1, G, bc)) << 32;
                nsplit[wb[a - 1] + pw] |= v;
            }
            __syncthreads();
        }
    }

    // ----------------------------------------------------------- A7: data transfer
    // Cells of R(Lambda^{n+1}) not in R(Lambda^n) are predicted from their parent level,
    // coarse to fine; all other cells keep their values (Sec. 4.1.1). Then the new tree
    // replaces the old one.
    DEV void transfer(const Vals<T>& V) {
        for (int l = jmin + 1; l <= J; ++l) {
            const int nw = nwords(l);
            const int Np = 1 << (l - 1);
            for (int w = wave; w < nw; w += nwaves) {
                const uint64_t nb = r_word(nsplit, wb, jmin, l, w) & ~r_word(split, wb, jmin, l, w);
                if (!nb) continue;
                if ((nb >> lane) & 1ull) {
                    const int c = (w << 6) + lane;
                    const int p = c >> 1;
                    const bool odd = c & 1;
#pragma unroll
                    for (int h = 0; h < Q; ++h) {
                        const T f0 = V.at(l - 1, h, p);
                        T acc = (T)0;
#pragma unroll
                        for (int a = 1; a <= G; ++a) {
                            const T tt = cc[a - 1] * (V.at(l - 1, h, bcx(p + a, Np, bc)) - V.at(l - 1, h, bcx(p - a, Np, bc)));
                            acc = (a == 1) ? tt : acc + tt;
                        }
                        V.at(l, h, c) = odd ? f0 - acc : f0 + acc;
                    }
                }
            }
            __syncthreads();
        }
        uint64_t* tmp = split;
        split = nsplit;
        nsplit = tmp;
    }

    // ----------------------------------------------------------- A6 + B1
    // Complete leaves = R(Lambda) minus split cells. Each leaf marks its left edge on the
    // finest lattice (so that ranks give spatial order) and, when collide is set, is
    // collided in place (Sec. 4.5). Returns nothing; the count is reduced through red[].
    DEV void leaves_mark(const Vals<T>& V, bool do_collide, int* nanflag) {
        int t = wave;
        int cnt = 0;
        for (int l = jmin; l <= J; ++l) {
            const int nw = nwords(l);
            for (; t < nw; t += nwaves) {
                const uint64_t lb = r_word(split, wb, jmin, l, t) & (l < J ? ~split[wb[l] + t] : ~0ull);
                if (!lb) continue;
                cnt += __popcll(lb);
                if ((lb >> lane) & 1ull) {
                    const int k = (t << 6) + lane;
                    const int e = k << (J - l);
                    atomicOr((unsigned long long*)&E[e >> 6], 1ull << (e & 63));
                    if (do_collide) {
                        T f[Q];
#pragma unroll
                        for (int h = 0; h < Q; ++h) f[h] = V.at(l, h, k);
                        collide<T, S>(d.cf, f);
                        bool bad = false;
#pragma unroll
                        for (int h = 0; h < Q; ++h) {
                            bad = bad || (f[h] != f[h]);
                            V.at(l, h, k) = f[h];
                        }
                        if (bad) *nanflag = 1;
                    }
                }
            }
            t -= nw;
        }
        if (lane == 0) atomicAdd(&red[0], (uint32_t)cnt);
        __syncthreads();
    }

    // Exclusive prefix of popcount(E[w]) over the finest words, block-wide.
    DEV void scan_edges() {
        const int nwJ = nwords(J);
        const int per = (nwJ + NT - 1) / NT;
        const int w0 = tid * per;
        uint32_t s = 0;
        for (int i = 0; i < per; ++i) {
            const int w = w0 + i;
            if (w < nwJ) s += (uint32_t)__popcll(E[w]);
        }
        // inclusive scan within the wave
        uint32_t x = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) red[1 + wave] = x;
        __syncthreads();
        if (tid == 0) {
            uint32_t run = 0;
            for (int wv = 0; wv < nwaves; ++wv) {
                const uint32_t v = red[1 + wv];
                red[1 + wv] = run;
                run += v;
            }
        }
        __syncthreads();
        uint32_t base = red[1 + wave] + x - s;
        for (int i = 0; i < per; ++i) {
            const int w = w0 + i;
            if (w < nwJ) {
                scan[w] = base;
                base += (uint32_t)__popcll(E[w]);
            }
        }
        __syncthreads();
    }

    // Leaf list in spatial order: rank of a leaf = number of leaf edges left of its own.
    DEV void write_list() {
        int t = wave;
        for (int l = jmin; l <= J; ++l) {
            const int nw = nwords(l);
            for (; t < nw; t += nwaves) {
                const uint64_t lb = r_word(split, wb, jmin, l, t) & (l < J ? ~split[wb[l] + t] : ~0ull);
                if (!lb) continue;
                if ((lb >> lane) & 1ull) {
                    const int k = (t << 6) + lane;
                    const int e = k << (J - l);
                    const uint64_t below = E[e >> 6] & ((1ull << (e & 63)) - 1ull);
                    const uint32_t rank = scan[e >> 6] + (uint32_t)__popcll(below);
                    d.list[rank] = ((uint32_t)l << 27) | (uint32_t)k;
                }
            }
            t -= nw;
        }
        __syncthreads();
    }

    // ----------------------------------------------------------- B3: stream
    // Interface i is the left edge of leaf i (i = n: the right end of the domain). Its two
    // reconstructed finest values (cells e-1 and e) serve both neighbouring leaves.
    DEV void pairs(const Vals<T>& V, int n) {
        const int NJ = 1 << J;
        T* P = reinterpret_cast<T*>(d.pairs);
        const int stride = NJ + 1;
        for (int i = tid; i <= n; i += NT) {
            int e = NJ;
            if (i < n) {
                const uint32_t key = d.list[i];
                const int l = key >> 27, k = key & ((1u << 27) - 1u);
                e = k << (J - l);
            }
            T a[NM], b[NM];
            pair_chain<T, G, NM, MovingPops<S>>(V, split, wb, jmin, J, bc, cc, e, a, b);
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                P[(2 * m) * stride + i] = a[m];
                P[(2 * m + 1) * stride + i] = b[m];
            }
        }
        __syncthreads();
    }

    // f^{n+1} of every leaf from its collided value and the interface pairs
    // (eq. AdaptiveStreamPhase; leaves at level J take the reconstructed neighbour).
    DEV void combine(const Vals<T>& V, const Vals<T>& Vn, int n) {
        const int NJ = 1 << J;
        const T* P = reinterpret_cast<const T*>(d.pairs);
        const int stride = NJ + 1;
        for (int i = tid; i < n; i += NT) {
            const uint32_t key = d.list[i];
            const int l = key >> 27, k = key & ((1u << 27) - 1u);
#pragma unroll
            for (int h = 0; h < Q; ++h) {
                const int wh = Sch<S>::w(h);
                const T fs = V.at(l, h, k);
                T out = fs;
                if (wh != 0) {
                    int m = 0;
#pragma unroll
                    for (int mm = 0; mm < NM; ++mm)
                        if (Sch<S>::mv(mm) == h) m = mm;
                    if (l == J) {
                        out = wh > 0 ? P[(2 * m) * stride + i] : P[(2 * m + 1) * stride + i + 1];
                    } else {
                        const int side = wh > 0 ? 0 : 1;  // eta = -1 (cell e-1) or 0 (cell e)
                        const T a = P[(2 * m + side) * stride + i];
                        const T b = P[(2 * m + side) * stride + i + 1];
                        const T acc = a - b;
                        out = fs + (T)ldexp(wh > 0 ? acc : -acc, -(J - l));
                    }
                }
                Vn.at(l, h, k) = out;
            }
        }
        // E is free again (its last reader was write_list, two barriers ago).
        for (int w = tid; w < nwords(J); w += NT) E[w] = 0ull;
        __syncthreads();
    }
};

template <typename T>
DEV Vals<T> vals_of(const Desc& d, int which) {
    Vals<T> v;
    v.base = reinterpret_cast<T*>(which ? d.vb : d.va);
    v.jmin = d.jmin;
    v.q = d.q;
    return v;
}

// Block prologue shared by the kernels: level word bases, tree bits into LDS, E cleared.
template <typename T, int S, int G>
DEV void load_tree(Block<T, S, G>& B, int* s_wb) {
    if (B.tid <= 24) s_wb[B.tid] = (B.tid >= B.jmin) ? wbase(B.jmin, B.tid) : 0;
    if (B.tid < 8) B.red[B.tid] = 0;
    const int wt = wbase(B.jmin, B.J + 1);
    const int wsplit = wbase(B.jmin, B.J);
    for (int w = B.tid; w < wt; w += B.NT) {
        B.split[w] = w < wsplit ? B.d.split[w] : 0ull;
        B.nsplit[w] = 0ull;
    }
    for (int w = B.tid; w < nwords(B.J); w += B.NT) B.E[w] = 0ull;
    __syncthreads();
}

template <typename T, int S, int G>
DEV void store_tree(Block<T, S, G>& B) {
    const int wsplit = wbase(B.jmin, B.J);
    for (int w = B.tid; w < wsplit; w += B.NT) B.d.split[w] = B.split[w];
}

// nsteps time steps (or adaptations only) of run blockIdx.x.
template <typename T, int S, int G>
__global__ __launch_bounds__(512) void k_steps(const Desc* __restrict__ descs, State* __restrict__ states,
                                                int nsteps, int mode) {
    extern __shared__ uint64_t lds[];
    __shared__ int s_wb[32];
    __shared__ uint32_t s_red[40];
    __shared__ int s_nan;
    const Desc& d = descs[blockIdx.x];
    Block<T, S, G> B(d, s_wb, lds, s_red);
    if (threadIdx.x == 0) s_nan = 0;
    load_tree(B, s_wb);
    int cur = states[blockIdx.x].cur;
    long long upd = 0;
    int last = -1;
    for (int st = 0; st < nsteps; ++st) {
        const Vals<T> V = vals_of<T>(d, cur);
        if (mode & MODE_ADAPT) {
            B.project_up(V);
            B.details(V, &s_nan);
            __syncthreads();
            B.enlarge();
            B.grade();
            B.transfer(V);
        }
        if (mode & MODE_SCHEME) {
            B.leaves_mark(V, true, &s_nan);
            const int n = (int)B.red[0];
            B.scan_edges();
            B.write_list();
            B.project_up(V);
            B.pairs(V, n);
            const Vals<T> Vn = vals_of<T>(d, cur ^ 1);
            B.combine(V, Vn, n);
            if (threadIdx.x == 0) B.red[0] = 0;
            __syncthreads();
            cur ^= 1;
            upd += n;
            last = n;
        }
    }
    store_tree(B);
    if (threadIdx.x == 0) {
        State& s = states[blockIdx.x];
        s.cur = cur;
        if (mode & MODE_SCHEME) {
            s.steps += nsteps;
            s.leaf_updates += upd;
            if (last >= 0) s.n_leaves = last;
        }
        if (s_nan) s.flags |= 1;
    }
}

// Initial state: populations at equilibrium on the finest level, full tree.
template <typename T, int S>
__global__ void k_init(const Desc* __restrict__ descs, State* __restrict__ states, const double* __restrict__ mc,
                       long long mc_stride) {
    const Desc& d = descs[blockIdx.y];
    const int NJ = 1 << d.jmax;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const double* m = mc + blockIdx.y * mc_stride;
    if (k < NJ) {
        double c[MAXQ];
        for (int i = 0; i < d.qc; ++i) c[i] = m[(size_t)i * NJ + k];
        T f[Sch<S>::Q];
        equilibrium<T, S>(d.cf, c, f);
        Vals<T> V = vals_of<T>(d, 0);
        for (int h = 0; h < Sch<S>::Q; ++h) V.at(d.jmax, h, k) = f[h];
    }
    const int wsplit = wbase(d.jmin, d.jmax);
    for (int w = k; w < wsplit; w += gridDim.x * blockDim.x) {
        // full tree: every cell below J split; partial words keep only their valid bits
        int l = d.jmin;
        while (w >= wbase(d.jmin, l + 1)) ++l;
        d.split[w] = lowmask(1 << l);
    }
    if (k == 0) {
        State& s = states[blockIdx.y];
        s.steps = 0;
        s.leaf_updates = 0;
        s.n_leaves = NJ;
        s.cur = 0;
        s.flags = 0;
    }
}

// Queries: leaf list of the current tree, then per leaf (where = 0) its conserved moments
// (what = 0) or populations (what = 1), or (where = 1) the reconstruction on every finest
// cell followed by its conserved moments. Output in d.out, [component][position].
template <typename T, int S, int G>
__global__ __launch_bounds__(512) void k_query(const Desc* __restrict__ descs, State* __restrict__ states,
                                                int where, int what, double* __restrict__ out) {
    extern __shared__ uint64_t lds[];
    __shared__ int s_wb[32];
    __shared__ uint32_t s_red[40];
    __shared__ int s_nan;
    const Desc& d = descs[blockIdx.x];
    Block<T, S, G> B(d, s_wb, lds, s_red);
    load_tree(B, s_wb);
    const int cur = states[blockIdx.x].cur;
    const Vals<T> V = vals_of<T>(d, cur);
    B.leaves_mark(V, false, &s_nan);
    const int n = (int)B.red[0];
    B.scan_edges();
    B.write_list();
    constexpr int Q = Sch<S>::Q;
    if (where == 0) {
        for (int i = B.tid; i < n; i += B.NT) {
            const uint32_t key = d.list[i];
            const int l = key >> 27, k = key & ((1u << 27) - 1u);
            T f[Q];
            for (int h = 0; h < Q; ++h) f[h] = V.at(l, h, k);
            if (what == 0) {
                double mc[MAXQ];
                conserved<T, S>(d.cf, f, mc);
                for (int c = 0; c < d.qc; ++c) out[(size_t)c * n + i] = mc[c];
            } else {
                for (int h = 0; h < Q; ++h) out[(size_t)h * n + i] = (double)f[h];
            }
        }
    } else {
        B.project_up(V);
        const int NJ = 1 << d.jmax;
        for (int m = B.tid; m < NJ; m += B.NT) {
            T a[Q], b[Q];
            pair_chain<T, G, Q, AllPops<S>>(V, B.split, s_wb, B.jmin, B.J, B.bc, B.cc, m + 1, a, b);
            if (what == 0) {
                double mc[MAXQ];
                conserved<T, S>(d.cf, a, mc);
                for (int c = 0; c < d.qc; ++c) out[(size_t)c * NJ + m] = mc[c];
            } else {
                for (int h = 0; h < Q; ++h) out[(size_t)h * NJ + m] = (double)a[h];
            }
        }
    }
    if (threadIdx.x == 0) states[blockIdx.x].n_leaves = n;
}

}  // namespace mrl
