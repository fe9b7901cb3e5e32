// mrlbm_kernels.h -- the per-run workgroup engine: every phase of an MR-LBM time step as a
// block-cooperative function, and the kernels built from them.
//
// One workgroup advances one run (one instance of a batch) through all the steps of a
// launch; phases are separated by workgroup barriers only, so a launch of K steps for B
// runs is a single grid of B workgroups with no inter-workgroup synchronization.
//
// During a launch the run lives on chip: the tree as bit words in LDS, the values of R(Lambda)
// compactly in LDS (slots, see rank_of) as long as the tree fits the LDS capacity chosen by
// the host. A step whose tree does not fit keeps its values in the run's HBM arrays instead
// (same compact layout, generic pointers); the next step moves back on chip when it fits.
// The home copy in HBM is read at launch start and written at launch end.
#pragma once

#include "mlp.h"
#include "mrlbm_device.h"

namespace mrl {

enum : int { MODE_ADAPT = 1, MODE_SCHEME = 2 };

template <typename T> struct LdsT;
template <> struct LdsT<double> { typedef __attribute__((address_space(3))) double type; };
template <> struct LdsT<float> { typedef __attribute__((address_space(3))) float type; };

// Byte offsets of the dynamic LDS of one workgroup.
struct Layout {
    int wt, ws, nwJ, cap, capS;
    unsigned bits, E, VA, VB, PP, rp, scanE, LL, wl, total;
};
__host__ __device__ inline unsigned al16(unsigned x) { return (x + 15u) & ~15u; }
// wlsz: bytes of a word-list entry (a word's index inside its level): 2, or 4 for levels of more
// than 2^16 words
__host__ __device__ inline Layout make_layout(int jmin, int J, int cap, int capS, int q, int nm, int tsz,
                                              bool learned = false, int wlsz = 2) {
    Layout L;
    L.wt = wbase(jmin, J + 1);
    L.ws = wbase(jmin, J);  // levels Jmin..J-1: the split-bit arrays (no split cell at J)
    L.nwJ = nwords(J);
    L.cap = cap;
    L.capS = capS;
    unsigned o = 0;
    L.bits = o;
    o = al16(o + ((learned ? 4u : 2u) * (unsigned)L.ws + 3u * (unsigned)L.wt) * 8u);
    L.E = o;
    o = al16(o + (unsigned)L.nwJ * 8u);
    L.VA = o;
    o = al16(o + (unsigned)q * (unsigned)cap * (unsigned)tsz);
    L.VB = o;
    o = al16(o + (unsigned)q * (unsigned)cap * (unsigned)tsz);
    // interface pairs: without the predictor they reuse the old value array, dead once the
    // transfer has read it; with it the old values must survive the step (a redo restarts
    // from them), so the pairs go to the run's HBM array instead: no LDS region either way
    L.PP = o;
    (void)learned;
    L.rp = o;
    o = al16(o + 2u * (unsigned)(L.wt + 1) * 4u);
    L.scanE = o;
    o = al16(o + (unsigned)L.nwJ * 4u);
    // leaf list: without the predictor it lives in the old value array behind the pairs
    // (written after the transfer, read until the next one)
    L.LL = o;
    if (learned) o = al16(o + (unsigned)capS * 4u);
    L.wl = o;
    o = al16(o + (2u * (unsigned)L.ws + (unsigned)L.wt) * (unsigned)wlsz);  // split words: levels < J
    L.total = o;
    return L;
}

// Per-level word lists: the words of level l that carry set bits are
// list[WB(l) .. WB(l) + count[l]) (any order inside a level).
template <typename W>
struct WordListT {
    W* w;
    int* c;
};

// WIDE: 32-bit word-list entries (levels of more than 2^16 words, J > 22)
template <typename T, int S, int G, bool LRN = false, bool WIDE = false>
struct Block {
    typedef typename std::conditional<WIDE, uint32_t, uint16_t>::type WLT;
    typedef WordListT<WLT> WordList;
    static constexpr int Q = Sch<S>::Q;
    static constexpr int NM = Sch<S>::NM;
    typedef typename LdsT<T>::type LT;

    const Desc& d;
    int tid, NT, lane, wave, nwaves;
    int jmin, J, bc, wt, ws;
    Layout lay;
    uint32_t* red;    // small scratch: [0] leaf count, [1..16] wave partials
    // tree arrays, rotated at the end of each step
    uint64_t* split;  // Lambda^n split bits
    uint64_t* nsplit; // Lambda^{n+1} split bits
    uint64_t* keep;   // T_eps bits; then R bits of Lambda^{n+1}
    uint64_t* ruleb;  // rule (b) bits; then leaf bits of Lambda^{n+1}
    uint64_t* ro;     // R bits of Lambda^n
    uint64_t* forced;   // predictor: rule (b) pairs the judge forces (this step)
    uint64_t* declined; // predictor: pairs the network declined / recorded candidates
    int* any_declined;  // predictor: set when a declined word of this attempt is nonzero
    uint32_t* rpo;    // slot prefix of Lambda^n
    uint32_t* rpn;    // slot prefix of Lambda^{n+1}
    WordList swl, nswl, lwl;  // split words of Lambda^n, of Lambda^{n+1}; leaf words of Lambda^{n+1}
    uint64_t* E;      // finest-level leaf left edges
    uint32_t* scanE;  // exclusive prefix of popcount(E)
    LT* ldsA;         // on-chip value arrays (capacity lay.cap slots each)
    LT* ldsB;
    uint32_t* ldsL;   // on-chip leaf list
    typedef __attribute__((address_space(3))) uint32_t LU;
    LU* tab;          // split cells of the current tree: (own slot << 16) | slot of the even child
    LU* tabp;         // and their keys (level << 27) | p (same order)
    LU* toff;         // tab offsets per level: level l occupies [toff[l - jmin], toff[l - jmin + 1])
    static constexpr int NOFF = 24;  // offset entries in front of the table (levels + 1 <= 17)
    T cc[3];

    // tb: base of the tree arrays (the workgroup's LDS, or the run's device-memory copy for
    // runs too large for LDS); lds: base of the on-chip value arrays
    DEV Block(const Desc& dd, const Layout& L, uint8_t* tb, uint8_t* lds, uint32_t* red_, int* cnts)
        : d(dd), lay(L), red(red_) {
        tid = threadIdx.x;
        NT = blockDim.x;
        lane = tid & 63;
        wave = tid >> 6;
        nwaves = NT >> 6;
        jmin = d.jmin;
        J = d.jmax;
        bc = d.bc;
        wt = L.wt;
        ws = L.ws;
        uint64_t* bits = reinterpret_cast<uint64_t*>(tb + L.bits);
        split = bits;
        nsplit = bits + ws;
        keep = bits + 2 * ws;
        ruleb = keep + wt;
        ro = ruleb + wt;
        forced = LRN ? ro + wt : nullptr;
        declined = LRN ? ro + wt + ws : nullptr;
        E = reinterpret_cast<uint64_t*>(tb + L.E);
        uint32_t* rp = reinterpret_cast<uint32_t*>(tb + L.rp);
        rpo = rp;
        rpn = rp + wt + 1;
        scanE = reinterpret_cast<uint32_t*>(tb + L.scanE);
        WLT* wl = reinterpret_cast<WLT*>(tb + L.wl);
        swl = {wl, cnts};
        nswl = {wl + ws, cnts + 32};
        lwl = {wl + 2 * ws, cnts + 64};
        ldsA = (LT*)(T*)(lds + L.VA);
        ldsB = (LT*)(T*)(lds + L.VB);
        ldsL = LRN ? reinterpret_cast<uint32_t*>(lds + L.LL) : nullptr;  // plain: set per step
        tab = nullptr;
        tabp = nullptr;
        toff = nullptr;
        for (int a = 0; a < 3; ++a) cc[a] = (T)d.c[a];
        any_declined = nullptr;
    }

    DEV int WB(int l) const { return wbase(jmin, l); }

    // The words of a per-level word list as one sequence of tasks, levels in order: returns
    // the number of tasks; lane i keeps the first task of level jmin + i in *first.
    DEV int list_tasks(WordList wl, int* first) const {
        const int nlev = J - jmin + 1;
        const int c = lane < nlev ? wl.c[jmin + lane] : 0;
        const int x = (int)wave_scan((uint32_t)c);
        *first = x - c;
        return __builtin_amdgcn_readlane(x, nlev - 1);
    }
    // Level of task k (wave-uniform) and its position t inside the level's list.
    DEV int task_level(int k, int first, int* t) const {
        const int nlev = J - jmin + 1;
        const uint64_t m = __ballot(lane < nlev && first <= k);
        const int i = __popcll(m) - 1;
        *t = k - __builtin_amdgcn_readlane(first, i);
        return jmin + i;
    }

    // ----------------------------------------------------------- block scan
    // Exclusive prefix of per-thread values; returns this thread's base, total in *tot.
    DEV uint32_t block_scan(uint32_t s, uint32_t* tot) {
        const uint32_t x = wave_scan(s);
        if (lane == 63) red[1 + wave] = x;
        __syncthreads();
        if (wave == 0) {  // exclusive scan of the wave totals, one lane per wave
            const uint32_t v = lane < nwaves ? red[1 + lane] : 0u;
            const uint32_t y = wave_scan(v);
            if (lane < nwaves) red[1 + lane] = y - v;
            if (lane == nwaves - 1) red[20] = y;
        }
        __syncthreads();
        *tot = red[20];
        return red[1 + wave] + x - s;
    }

    // ----------------------------------------------------------- tree structures
    // From split bits sp: R bits (R), slot prefix (RP, RP[wt] = #R), the list of nonzero
    // split words (sl) and, when LW is given, leaf bits LW = R & ~split, their word list and
    // the leaf count in red[0]. Ends with a barrier. cleared: the caller has zeroed the word
    // counts of sl and ll and red[0] before a barrier of its own.
    DEV void build_tree(const uint64_t* sp, uint64_t* R, uint32_t* RP, WordList sl, uint64_t* LW, WordList ll,
                        bool cleared = false) {
        if (!cleared) {
            if (tid < 32) {
                sl.c[tid] = 0;
                if (LW) ll.c[tid] = 0;
            }
            if (tid == 0 && LW) red[0] = 0;
            __syncthreads();
        }
        const int per = (wt + NT - 1) / NT;
        const int w0 = tid * per;
        uint32_t s = 0;
        uint32_t nleaf = 0;
        for (int i = 0; i < per; ++i) {
            const int w = w0 + i;
            if (w >= wt) break;
            int lw;
            const int l = level_of_word(jmin, w, &lw);
            const uint64_t r = r_word(sp, jmin, l, lw);
            R[w] = r;
            s += (uint32_t)__popcll(r);
            const uint64_t spw = (l < J) ? sp[w] : 0ull;
            if (spw) {
                const int pos = atomicAdd(&sl.c[l], 1);
                sl.w[WB(l) + pos] = (WLT)lw;
            }
            if (LW) {
                const uint64_t lf = r & ~spw;
                LW[w] = lf;
                if (lf) {
                    nleaf += (uint32_t)__popcll(lf);
                    const int pos = atomicAdd(&ll.c[l], 1);
                    ll.w[WB(l) + pos] = (WLT)lw;
                }
            }
        }
        if (LW && nleaf) atomicAdd(&red[0], nleaf);
        uint32_t tot;
        uint32_t base = block_scan(s, &tot);
        for (int i = 0; i < per; ++i) {
            const int w = w0 + i;
            if (w >= wt) break;
            RP[w] = base;
            base += (uint32_t)__popcll(R[w]);
        }
        if (tid == 0) RP[wt] = tot;
        __syncthreads();
    }

    // ----------------------------------------------------------- A1 / B2: projection
    // Every split cell takes half the sum of its two children (adjacent slots), finest
    // level first (Sec. 3.1, Definition Projection operator).
    // PM / NP: the populations projected (all of them by default).
    template <class PM = AllPops<S>, int NP = Q, class V>
    DEV bool project_up(const V& Vx, const uint64_t* sp, const uint64_t* R, const uint32_t* RP, WordList sl) {
        // Two levels per barrier: the thread of a split cell (l-1, p) first takes the average
        // of each split child (l, 2p + c) from its own children, stores it, then stores its own
        // average of the two children. Every split cell of level l has a split parent, so the
        // pass over level l-1 covers level l; each value is still half the sum of its two
        // children, children first.
        bool synced = false;  // whether the last thing done was a barrier
        int l = J - 1;
        for (; l - 1 >= jmin; l -= 2) {
            const int lp = l - 1;
            const int n = sl.c[lp];
            if (n == 0) continue;  // no split cell at lp, hence none at l
            for (int t = wave; t < n; t += nwaves) {
                const int w = sl.w[WB(lp) + t];
                const uint64_t b = sp[WB(lp) + w];
                if ((b >> lane) & 1ull) {
                    const int p = (w << 6) + lane;
                    T cv[2][NP];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const int k = 2 * p + c;
                        const int sk = rank_of(R, RP, jmin, l, k);
                        if (getbit(sp, WB(l), k)) {
                            const int sg = rank_of(R, RP, jmin, l + 1, 2 * k);
                            // every load before the stores: they cannot alias, but the
                            // compiler would otherwise wait for each store before the next load
                            T g0[NP], g1[NP];
#pragma unroll
                            for (int h = 0; h < NP; ++h) {
                                g0[h] = Vx.ld(PM::h(h), sg);
                                g1[h] = Vx.ld(PM::h(h), sg + 1);
                            }
#pragma unroll
                            for (int h = 0; h < NP; ++h) {
                                cv[c][h] = (T)0.5 * (g0[h] + g1[h]);
                                Vx.st(PM::h(h), sk, cv[c][h]);
                            }
                        } else {
#pragma unroll
                            for (int h = 0; h < NP; ++h) cv[c][h] = Vx.ld(PM::h(h), sk);
                        }
                    }
                    const int so = rank_of(R, RP, jmin, lp, p);
#pragma unroll
                    for (int h = 0; h < NP; ++h) Vx.st(PM::h(h), so, (T)0.5 * (cv[0][h] + cv[1][h]));
                }
            }
            __syncthreads();
            synced = true;
        }
        if (l == jmin) {  // one level left
            const int n = sl.c[l];
            for (int t = wave; t < n; t += nwaves) {
                const int w = sl.w[WB(l) + t];
                const uint64_t b = sp[WB(l) + w];
                if ((b >> lane) & 1ull) {
                    const int p = (w << 6) + lane;
                    const int sc = rank_of(R, RP, jmin, l + 1, 2 * p);
                    const int sp_ = rank_lane(R, RP, jmin, l, w);
                    T g0[NP], g1[NP];
#pragma unroll
                    for (int h = 0; h < NP; ++h) {
                        g0[h] = Vx.ld(PM::h(h), sc);
                        g1[h] = Vx.ld(PM::h(h), sc + 1);
                    }
#pragma unroll
                    for (int h = 0; h < NP; ++h) Vx.st(PM::h(h), sp_, (T)0.5 * (g0[h] + g1[h]));
                }
            }
            if (n) {
                __syncthreads();
                synced = true;
            }
        }
        return synced;
    }

    // Slot table of a tree (split bits sp, R bits, slot prefix RP, split-word list wl) written
    // to dst (room for maxe words, in a dead part of the LDS value arrays): NOFF words of
    // per-level offsets (toff), then the split cells in level order, each as (own slot << 16) |
    // slot of its even child, then their keys (level << 27) | p in the same order. Slots are
    // ranks in R(Lambda), the same whether the values sit on chip or in HBM; they must fit 16
    // bits (#R <= 2^16). The cells of R above level jmin come in sibling pairs, in the order of
    // their parents, so a split cell's place in the table is (slot of its even child - #R at
    // level jmin) / 2 and the level offsets follow from the slot prefix: no scan. Returns false
    // when the slots do not fit or the table outgrows maxe (no table); when it returns true it
    // ends with a barrier, unless sync is false (the caller's next barrier orders the writes).
    DEV bool build_table(const uint64_t* sp, const uint64_t* R, const uint32_t* RP, WordList wl, LU* dst,
                         int maxe, bool sync = true) {
        if ((int)RP[wt] > 65536 || lay.cap > 65535) return false;
        const int nlev = J - jmin + 1;
        const uint32_t base = RP[WB(jmin + 1)];  // the cells of level jmin
        const uint32_t tot = (RP[wt] - base) >> 1;
        if (2 * tot + NOFF > (uint32_t)maxe) return false;  // uniform
        toff = dst;
        tab = dst + NOFF;
        tabp = tab + tot;
        // level jmin + i starts after the split cells of the levels below it, i.e. after half
        // the cells of R at levels jmin + 1 .. jmin + i; lane nlev holds the total
        if (wave == 0 && lane <= nlev) toff[lane] = lane < nlev ? (RP[WB(jmin + lane + 1)] - base) >> 1 : tot;
        int first;
        const int ntask = list_tasks(wl, &first);
        for (int task = wave; task < ntask; task += nwaves) {
            int t;
            const int l = task_level(task, first, &t);
            const int w = wl.w[WB(l) + t];
            const uint64_t b = sp[WB(l) + w];
            if ((b >> lane) & 1ull) {
                const int p = (w << 6) + lane;
                const uint32_t so = (uint32_t)rank_lane(R, RP, jmin, l, w);
                const uint32_t sc = (uint32_t)rank_of(R, RP, jmin, l + 1, 2 * p);
                const uint32_t e = (sc - base) >> 1;
                tab[e] = (so << 16) | sc;
                tabp[e] = ((uint32_t)l << 27) | (uint32_t)p;
            }
        }
        if (sync) __syncthreads();
        return true;
    }

    // Projection through the slot table (same arithmetic as project_up, one level per pass).
    // PM / NP: the populations projected (all of them by default).
    template <class PM = AllPops<S>, int NP = Q, class V>
    DEV bool project_table(const V& Vx) {
        const int nlev = J - jmin + 1;
        const int myoff = lane <= nlev ? (int)toff[lane] : 0;  // every wave keeps the offsets
        bool synced = false;
        for (int i = nlev - 2; i >= 0; --i) {            // levels J-1 .. jmin
            const int a = __builtin_amdgcn_readlane(myoff, i);
            const int b = __builtin_amdgcn_readlane(myoff, i + 1);
            if (a == b) continue;
            synced = true;
            for (int e = a + tid; e < b; e += NT) {
                const uint32_t en = tab[e];
                const int so = (int)(en >> 16), sc = (int)(en & 0xFFFFu);
                T g0[NP], g1[NP];
#pragma unroll
                for (int h = 0; h < NP; ++h) {
                    g0[h] = Vx.ld(PM::h(h), sc);
                    g1[h] = Vx.ld(PM::h(h), sc + 1);
                }
#pragma unroll
                for (int h = 0; h < NP; ++h) Vx.st(PM::h(h), so, (T)0.5 * (g0[h] + g1[h]));
            }
            __syncthreads();
        }
        return synced;
    }

    // ----------------------------------------------------------- A2-A4(b): details
    // For every split cell (l, p): d^h = f_{l+1,2p} - (f_{l,p} + sum_a c_a (f_{l,p+a} - f_{l,p-a}))
    // in double (Sec. 3.1-3.2), D = max_h |d^h|; keep iff D >= eps_{l+1} (Sec. 3.4, T_eps);
    // rule (b) iff kept, l+1 < J and D >= 2^(mu+1) eps_{l+1} (Sec. 4.2). One wave per split
    // word; __ballot turns the 64 lane decisions into the keep / ruleb words. keep and ruleb
    // must be zero beforehand (only words with split cells are written).
    // Features of a candidate pair (l, p) from the values of Lambda^n: for the split cells
    // p-2..p+2 and every population, d / (|d| + eps_{l+1}) (0 for cells that are not split),
    // then (l + 1) / J. Same detail arithmetic as details().
    template <class V>
    DEV void features(const V& Vx, int l, int p, float* x) {
        const int N = 1 << l;
        const double el = ldexp(d.eps, l + 1 - J);
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) x[i] = 0.f;
#pragma unroll
        for (int di = 0; di < 5; ++di) {
            const int c = bcx(p + di - 2, N, bc);
            if (getbit(split, WB(l), c)) {
                const int sc = rank_of(ro, rpo, jmin, l + 1, 2 * c);
                const int s0 = rank_of(ro, rpo, jmin, l, c);
                int sp_[G], sm_[G];
#pragma unroll
                for (int a = 1; a <= G; ++a) {
                    sp_[a - 1] = rank_of(ro, rpo, jmin, l, bcx(c + a, N, bc));
                    sm_[a - 1] = rank_of(ro, rpo, jmin, l, bcx(c - a, N, bc));
                }
#pragma unroll
                for (int h = 0; h < Q; ++h) {
                    const double f0 = (double)Vx.ld(h, s0);
                    double acc = 0.0;
#pragma unroll
                    for (int a = 1; a <= G; ++a) {
                        const double tt = d.c[a - 1] * ((double)Vx.ld(h, sp_[a - 1]) - (double)Vx.ld(h, sm_[a - 1]));
                        acc = (a == 1) ? tt : acc + tt;
                    }
                    const double dd = (double)Vx.ld(h, sc) - (f0 + acc);
                    x[di * Q + h] = (float)(dd / (fabs(dd) + el));
                }
            }
        }
        x[5 * Q] = (float)((double)(l + 1) / (double)J);
    }

    // Max over populations of |d| for the split cell (l, p) of a tree (R bits, slot prefix).
    template <class V>
    DEV double max_detail(const V& Vx, const uint64_t* R, const uint32_t* RP, int l, int p) {
        const int N = 1 << l;
        const int sc = rank_of(R, RP, jmin, l + 1, 2 * p);
        const int s0 = rank_of(R, RP, jmin, l, p);
        int sp_[G], sm_[G];
#pragma unroll
        for (int a = 1; a <= G; ++a) {
            sp_[a - 1] = rank_of(R, RP, jmin, l, bcx(p + a, N, bc));
            sm_[a - 1] = rank_of(R, RP, jmin, l, bcx(p - a, N, bc));
        }
        double D = 0.0;
#pragma unroll
        for (int h = 0; h < Q; ++h) {
            const double f0 = (double)Vx.ld(h, s0);
            double acc = 0.0;
#pragma unroll
            for (int a = 1; a <= G; ++a) {
                const double tt = d.c[a - 1] * ((double)Vx.ld(h, sp_[a - 1]) - (double)Vx.ld(h, sm_[a - 1]));
                acc = (a == 1) ? tt : acc + tt;
            }
            const double ad = fabs((double)Vx.ld(h, sc) - (f0 + acc));
            D = ad > D ? ad : D;
        }
        return D;
    }

    template <class V>
    DEV void details(const V& Vx, int* nanflag) {
        int first;
        const int ntask = list_tasks(swl, &first);
        for (int task = wave; task < ntask; task += nwaves) {
            {
                int t;
                const int l = task_level(task, first, &t);
                const int N = 1 << l;
                const double thr = ldexp(d.eps, l + 1 - J);
                const double thrb = ldexp(d.eps, d.mu_bar + 1 + l + 1 - J);
                const bool rb_level = (l + 1 < J);
                const int w = swl.w[WB(l) + t];
                const uint64_t b = split[WB(l) + w];
                bool kb = false, rbb = false, rbu = false, cand = false;
                if ((b >> lane) & 1ull) {
                    const int p = (w << 6) + lane;
                    const int sc = rank_of(ro, rpo, jmin, l + 1, 2 * p);
                    const int s0 = rank_lane(ro, rpo, jmin, l, w);
                    int sp_[G], sm_[G];
#pragma unroll
                    for (int a = 1; a <= G; ++a) {
                        sp_[a - 1] = rank_of(ro, rpo, jmin, l, bcx(p + a, N, bc));
                        sm_[a - 1] = rank_of(ro, rpo, jmin, l, bcx(p - a, N, bc));
                    }
                    double D = 0.0;
                    bool bad = false;
#pragma unroll
                    for (int h = 0; h < Q; ++h) {
                        const double f0 = (double)Vx.ld(h, s0);
                        double acc = 0.0;
#pragma unroll
                        for (int a = 1; a <= G; ++a) {
                            const double tt = d.c[a - 1] * ((double)Vx.ld(h, sp_[a - 1]) - (double)Vx.ld(h, sm_[a - 1]));
                            acc = (a == 1) ? tt : acc + tt;
                        }
                        const double pred = f0 + acc;
                        const double dd = (double)Vx.ld(h, sc) - pred;
                        const double ad = fabs(dd);
                        bad = bad || (ad != ad);
                        D = ad > D ? ad : D;
                    }
                    if (bad) *nanflag = 1;
                    kb = bad || (D >= thr);
                    rbb = kb && rb_level && (bad || D >= thrb);
                    rbu = rbb;
                    if constexpr (LRN)
                        cand = d.pmode == 1 && d.mlp && rbb && !getbit(forced, WB(l), p) && D < d.gate * thrb;
                }
                if constexpr (LRN) {
                    // the network decides the candidates of this word one at a time, each
                    // evaluated by the whole wave (lane = hidden unit)
                    uint64_t cm = __ballot(cand);
                    if (cm) {
                        float x[MLP_IN];
#pragma unroll
                        for (int i = 0; i < MLP_IN; ++i) x[i] = 0.f;
                        if (cand) features(Vx, l, (w << 6) + lane, x);
                        uint64_t accept = 0ull;
                        while (cm) {
                            const int c = __builtin_ctzll(cm);
                            cm &= cm - 1ull;
                            if (mlp_logit_wave(d.mlp, x, c, lane) >= 0.f) accept |= 1ull << c;
                        }
                        if (cand) rbu = ((accept >> lane) & 1ull) != 0ull;
                    }
                }
                const uint64_t kw = __ballot(kb);
                const uint64_t rw = __ballot(rbb);
                const uint64_t uw = __ballot(rbu);
                if (lane == 0) {
                    keep[WB(l) + w] = kw;
                    ruleb[WB(l) + w] = uw;
                    if constexpr (LRN) {
                        const uint64_t dw = d.pmode == 1 ? (rw & ~uw) : (d.pmode == 2 ? rw : 0ull);
                        declined[WB(l) + w] = dw;
                        if (dw) *any_declined = 1;
                    }
                }
                (void)rw;
            }
        }
    }

    // Details and decisions of the current tree from its slot table: one thread per split
    // cell (all levels at once), the same arithmetic as details(); the keep and rule-(b)
    // bits are set with LDS atomics (the words start cleared). Plain kernels only.
    template <class V>
    DEV void details_table(const V& Vx, int* nanflag) {
        const int nlev = J - jmin + 1;
        const int myoff = lane <= nlev ? (int)toff[lane] : 0;
        const int total = __builtin_amdgcn_readlane(myoff, nlev - 1);  // start of level J
        for (int e = tid; e < total; e += NT) {
            const uint32_t key = tabp[e];
            const int l = (int)(key >> 27), p = (int)(key & ((1u << 27) - 1u));
            const int N = 1 << l;
            const uint32_t en = tab[e];
            const int s0 = (int)(en >> 16), sc = (int)(en & 0xFFFFu);
            // the tree is graded: the cells within gamma of a split cell at its level are in R,
            // so their slots follow from its own (R is ranked by index within a level); across
            // the periodic seam from the level's first or last slot, under clamp the edge cell
            int sp_[G], sm_[G];
#pragma unroll
            for (int a = 1; a <= G; ++a) {
                const int qp = p + a, qm = p - a;
                if (bc == PERIODIC) {
                    sp_[a - 1] = qp < N ? s0 + a : (int)rpo[WB(l)] + (qp - N);
                    sm_[a - 1] = qm >= 0 ? s0 - a : (int)rpo[WB(l + 1)] + qm;
                } else {
                    sp_[a - 1] = s0 + ((qp < N ? qp : N - 1) - p);
                    sm_[a - 1] = s0 + ((qm >= 0 ? qm : 0) - p);
                }
            }
            double D = 0.0;
            bool bad = false;
#pragma unroll
            for (int h = 0; h < Q; ++h) {
                const double f0 = (double)Vx.ld(h, s0);
                double acc = 0.0;
#pragma unroll
                for (int a = 1; a <= G; ++a) {
                    const double tt = d.c[a - 1] * ((double)Vx.ld(h, sp_[a - 1]) - (double)Vx.ld(h, sm_[a - 1]));
                    acc = (a == 1) ? tt : acc + tt;
                }
                const double pred = f0 + acc;
                const double dd = (double)Vx.ld(h, sc) - pred;
                const double ad = fabs(dd);
                bad = bad || (ad != ad);
                D = ad > D ? ad : D;
            }
            if (bad) *nanflag = 1;
            const double thr = ldexp(d.eps, l + 1 - J);
            const double thrb = ldexp(d.eps, d.mu_bar + 1 + l + 1 - J);
            const bool kb = bad || (D >= thr);
            const bool rbb = kb && (l + 1 < J) && (bad || D >= thrb);
            const int wi = WB(l) + (p >> 6);
            const unsigned long long bit = 1ull << (p & 63);
            if (kb) atomicOr((unsigned long long*)&keep[wi], bit);
            if (rbb) atomicOr((unsigned long long*)&ruleb[wi], bit);
        }
    }

    // ----------------------------------------------------------- A4: enlargement
    // Rule (a): every cell of R(T_eps) at level l+1 puts its neighbours within sigma into R,
    // i.e. their parents split: a dilation of keep[l] by ceil(sigma/2) at level l. Rule (b):
    // both children of a flagged cell are split. Writes every word of nsplit.
    DEV void enlarge() {
        // the children 2p, 2p + 1 of a kept cell put the cells 2p - sigma .. 2p + 1 + sigma into R:
        // the parents p - ceil(sigma / 2) .. p + floor((sigma + 1) / 2), i.e. p -+ 1 for sigma = 1, 2
        static_assert(Sch<S>::SIG <= 2, "rule (a) is written for sigma <= 2");
        const int ra = 1;
        for (int w = tid; w < ws; w += NT) {
            int t;
            const int l = level_of_word(jmin, w, &t);
            uint64_t v = 0;
            if (l < J) {
                v = dilate_word(keep, w - t, l, t, ra, bc);
                if (l > jmin) {
                    const uint64_t pb = ruleb[WB(l - 1) + (t >> 1)] >> ((t & 1) * 32);
                    v |= spread32(pb);
                }
            }
            nsplit[w] = v;
        }
        __syncthreads();
    }

    // ----------------------------------------------------------- A5: grading
    // Smallest graded tree (Sec. 3.3): a split cell (a, p), a > Jmin, needs (a, p + delta),
    // |delta| <= gamma, in R, so the parents of those cells are split. One sweep from the
    // finest level; delta = 0 also restores the tree property.
    DEV void grade() {
        // one parent word per thread and a barrier per level while a level is wider than a
        // wave; the remaining coarse levels in wave 0 alone (LDS order within a wave)
        int a = J - 1;
        for (; a > jmin && nwords(a - 1) > 64; --a) {
            grade_level(a, tid, NT);
            __syncthreads();
        }
        if (wave == 0 && a > jmin) {
            // the rest of the run waits at the barrier for this wave: issue it first on its SIMD
            __builtin_amdgcn_s_setprio(3);
            grade_wave(a);
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
    }

    // Levels a .. jmin + 1 of the grading in one wave, the words in registers: at level a
    // (at most 128 words) lane i holds words 2i and 2i + 1, takes its outer neighbours from
    // lanes i - 1 and i + 1 and owns parent word i; parent words are stored as they come and
    // regrouped in pairs for the next level by lane exchange.
    DEV void grade_wave(int a) {
        // the words of the single-word levels below min(a, 6) (level l < 6 is word l - jmin)
        const int ncoarse = (a < 6 ? a : 6) - jmin;
        const uint64_t cw = lane < ncoarse ? nsplit[lane] : 0ull;
        // a level of 128 words (two per lane): its parents, one per lane
        if (a > jmin && nwords(a) > 64) {
            const int h = nwords(a) >> 1;  // 64
            const uint64_t x0 = nsplit[WB(a) + 2 * lane], x1 = nsplit[WB(a) + 2 * lane + 1];
            const uint64_t old = nsplit[WB(a - 1) + lane];
            const uint64_t pl = shfl64(x1, (lane - 1) & (h - 1));
            const uint64_t nx = shfl64(x0, (lane + 1) & (h - 1));
            const uint64_t xl = (bc == PERIODIC || lane > 0) ? pl : 0ull;
            const uint64_t xr = (bc == PERIODIC || lane < h - 1) ? nx : 0ull;
            const uint64_t pw = old | compress64(dilate_val(x0, xl, x1, a, G, bc)) |
                                (compress64(dilate_val(x1, x0, xr, a, G, bc)) << 32);
            nsplit[WB(a - 1) + lane] = pw;
            --a;
        }
        // levels of 2..64 words: word i of the level in lane i
        uint64_t x = lane < nwords(a) ? nsplit[WB(a) + lane] : 0ull;
        uint64_t old = lane < nwords(a - 1) ? nsplit[WB(a - 1) + lane] : 0ull;
        for (; a > jmin && nwords(a) >= 2; --a) {
            const int cnw = nwords(a);
            const int pnw = cnw >> 1;
            const uint64_t onext = (a - 2 >= jmin && lane < nwords(a - 2)) ? nsplit[WB(a - 2) + lane] : 0ull;
            // neighbour words from the adjacent lanes; the ends wrap within the cnw lanes
            // (periodic) or read zero (clamp)
            const uint64_t wl = bc == PERIODIC ? readlane64(x, cnw - 1) : 0ull;
            const uint64_t wr = bc == PERIODIC ? readlane64(x, 0) : 0ull;
            const uint64_t pv = from_prev_lane(x), nv = from_next_lane(x);
            const uint64_t xl = lane == 0 ? wl : pv;
            const uint64_t xr = lane == cnw - 1 ? wr : nv;
            // half of parent word i >> 1 (low half from the even word)
            const uint32_t c = (uint32_t)compress64(dilate_val(x, xl, xr, a, G, bc));
            const uint32_t o = from_pair_lane(c);
            const uint64_t pe = (uint64_t)c | ((uint64_t)o << 32);  // parent word lane / 2, even lanes
            x = shfl64(pe, 2 * lane) | old;                          // parent word j in lane j
            if (lane < pnw) nsplit[WB(a - 1) + lane] = x;
            old = onext;
        }
        // single-word levels (at most 64 cells): the word is uniform, so the chain runs on
        // the scalar unit; a level of 64 cells wraps onto itself (or reads zero when clamped)
        uint64_t xs = readlane64(x, 0);
        for (; a > jmin; --a) {
            const uint64_t e = bc == PERIODIC ? xs : 0ull;
            xs = compress64(dilate_val(xs, e, e, a, G, bc)) | readlane64(cw, a - 1 - jmin);
            if (lane == 0) nsplit[a - 1 - jmin] = xs;
        }
    }

    DEV void grade_level(int a, int t0, int stride) {
        const int pnw = nwords(a - 1);
        const int cnw = nwords(a);
        for (int pw = t0; pw < pnw; pw += stride) {
            const int c0 = 2 * pw, c1 = 2 * pw + 1;
            uint64_t v = 0;
            if (c0 < cnw) v |= compress64(dilate_word(nsplit, WB(a), a, c0, G, bc));
            if (c1 < cnw) v |= compress64(dilate_word(nsplit, WB(a), a, c1, G, bc)) << 32;
            nsplit[WB(a - 1) + pw] |= v;
        }
    }

    // ----------------------------------------------------------- A7 (+ B1): data transfer
    // Every complete leaf of Lambda^{n+1} gets its value at t^n: the stored value when the
    // cell is in R(Lambda^n) (a leaf, or the projection of a coarsened subtree), otherwise the
    // reconstruction from Lambda^n, i.e. level-by-level prediction (Sec. 4.1.1). With collide
    // set the leaf is collided right away (Sec. 4.5) and its left edge is marked in E.
    template <class VO_, class VN_>
    DEV void transfer(const VO_& VO, const VN_& VN, bool collide_leaf, bool mark, int* nanflag) {
        int first;
        const int ntask = list_tasks(lwl, &first);
        for (int task = wave; task < ntask; task += nwaves) {
            {
                int t;
                const int l = task_level(task, first, &t);
                const int w = lwl.w[WB(l) + t];
                const uint64_t b = ruleb[WB(l) + w];
                if ((b >> lane) & 1ull) {
                    const int k = (w << 6) + lane;
                    T f[Q];
                    if (rbit(ro, jmin, l, k)) {
                        const int so = rank_lane(ro, rpo, jmin, l, w);
#pragma unroll
                        for (int h = 0; h < Q; ++h) f[h] = VO.ld(h, so);
                    } else {
                        chain<T, G, Q, AllPops<S>, 1>(VO, ro, rpo, jmin, l, bc, cc, k, k, f, l);
                    }
                    if (mark) {
                        if (collide_leaf) {
                            collide<T, S>(d.cf, f);
                            bool bad = false;
#pragma unroll
                            for (int h = 0; h < Q; ++h) bad = bad || (f[h] != f[h]);
                            if (bad) *nanflag = 1;
                        }
                        const int e = k << (J - l);
                        atomicOr((unsigned long long*)&E[e >> 6], 1ull << (e & 63));
                    }
                    const int sn = rank_lane(keep, rpn, jmin, l, w);
#pragma unroll
                    for (int h = 0; h < Q; ++h) VN.st(h, sn, f[h]);
                }
            }
        }
        __syncthreads();
    }

    // ----------------------------------------------------------- A6: leaf list
    DEV void scan_edges() {
        const int nwJ = lay.nwJ;
        const int per = (nwJ + NT - 1) / NT;
        const int w0 = tid * per;
        uint32_t s = 0;
        for (int i = 0; i < per; ++i) {
            const int w = w0 + i;
            if (w < nwJ) s += (uint32_t)__popcll(E[w]);
        }
        uint32_t tot;
        uint32_t base = block_scan(s, &tot);
        for (int i = 0; i < per; ++i) {
            const int w = w0 + i;
            if (w < nwJ) {
                scanE[w] = base;
                base += (uint32_t)__popcll(E[w]);
            }
        }
        __syncthreads();
    }

    // Spatial rank of a leaf = number of leaf left edges before its own.
    template <class LP>
    DEV void write_list(LP* list, bool sync = true) {
        int first;
        const int ntask = list_tasks(lwl, &first);
        for (int task = wave; task < ntask; task += nwaves) {
            {
                int t;
                const int l = task_level(task, first, &t);
                const int w = lwl.w[WB(l) + t];
                const uint64_t b = ruleb[WB(l) + w];
                if ((b >> lane) & 1ull) {
                    const int k = (w << 6) + lane;
                    const int e = k << (J - l);
                    const uint64_t below = E[e >> 6] & ((1ull << (e & 63)) - 1ull);
                    const uint32_t rank = scanE[e >> 6] + (uint32_t)__popcll(below);
                    list[rank] = ((uint32_t)l << 27) | (uint32_t)k;
                }
            }
        }
        if (sync) __syncthreads();
    }

    // ----------------------------------------------------------- B1': reconstructed collision
    // Reconstructed collision (Sec. 4.3.1, eq. reconstructedCollision). The values of
    // R(Lambda^{n+1}) hold f^n projected up the tree. First one thread per pair of finest
    // cells m: the leaf holding m (the last leaf edge at or before m, from the edge bits and their
    // prefix), the reconstruction of m from that leaf's level, and the equilibria of its
    // conserved moments, written to eqs (NE planes of 2^J values). Then one thread per leaf
    // of the spatial list: the sum of its cells' equilibria in cell order, scaled by
    // 2^-(J-l) (exact), and the relaxation of the leaf towards that mean, in place (no
    // thread reads another leaf's values any more).
    template <class V, class LP>
    DEV void recon_collide(const V& Vx, const LP* list, T* eqs, int n, int* nanflag) {
        constexpr int NE = NEq<S>::N;
        const int NJ = 1 << J;
        // cells 2t and 2t+1 (J >= 1) share one chain (its window covers both), started at the
        // coarser of their leaves' levels
        auto leaf_level = [&](int m) {
            const uint64_t upto = E[m >> 6] & ((2ull << (m & 63)) - 1ull);  // edges at or before m
            const int i = (int)(scanE[m >> 6] + (uint32_t)__popcll(upto)) - 1;
            return (int)(list[i] >> 27);
        };
        for (int t = tid; t < (NJ >> 1); t += NT) {
            const int ma = 2 * t, mb = 2 * t + 1;
            const int la = leaf_level(ma), lb = leaf_level(mb);
            T ab[2 * Q];
            chain<T, G, Q, AllPops<S>, 2>(Vx, keep, rpn, jmin, J, bc, cc, ma, mb, ab, la < lb ? la : lb);
            T a[Q], b[Q];
#pragma unroll
            for (int h = 0; h < Q; ++h) {
                a[h] = ab[2 * h];
                b[h] = ab[2 * h + 1];
            }
            T e[NE];
            eq_moments<T, S>(d.cf, a, e);
#pragma unroll
            for (int x = 0; x < NE; ++x) eqs[x * NJ + ma] = e[x];
            eq_moments<T, S>(d.cf, b, e);
#pragma unroll
            for (int x = 0; x < NE; ++x) eqs[x * NJ + mb] = e[x];
        }
        __syncthreads();
        for (int i = tid; i < n; i += NT) {
            const uint32_t key = list[i];
            const int l = key >> 27, k = key & ((1u << 27) - 1u);
            const int dl = J - l;
            const int m0 = k << dl;
            T acc[NE];
#pragma unroll
            for (int x = 0; x < NE; ++x) acc[x] = eqs[x * NJ + m0];
            for (int dd = 1; dd < (1 << dl); ++dd)
#pragma unroll
                for (int x = 0; x < NE; ++x) acc[x] = acc[x] + eqs[x * NJ + m0 + dd];
            const T sc = (T)ldexp(1.0, -dl);
#pragma unroll
            for (int x = 0; x < NE; ++x) acc[x] = acc[x] * sc;
            const int s = rank_of(keep, rpn, jmin, l, k);
            T f[Q];
#pragma unroll
            for (int h = 0; h < Q; ++h) f[h] = Vx.ld(h, s);
            relax_to<T, S>(d.cf, f, acc);
            bool bad = false;
#pragma unroll
            for (int h = 0; h < Q; ++h) {
                bad = bad || (f[h] != f[h]);
                Vx.st(h, s, f[h]);
            }
            if (bad) *nanflag = 1;
        }
        __syncthreads();
    }

    // ----------------------------------------------------------- B3: stream
    // Interface i is the left edge e of leaf i (i = n: the right end of the domain). The
    // stream of the leaves on both of its sides reads the reconstructed finest values at
    // e + eta(h, delta), eta in -SIG..SIG-1 (eq. AdaptiveStreamPhase); one reconstruction
    // chain per interface covers the cells e - SIG .. e + SIG - 1, and only the values some
    // population reads are kept (Planes<S>: sum over moving populations of |w| planes).
    template <class V, class LP, class PP>
    DEV void pairs(const V& Vx, const LP* list, PP* P, int n) {
        constexpr int SG = Sch<S>::SIG;
        constexpr int NO = 2 * SG;
        typedef Planes<S> PLN;
        const int NJ = 1 << J;
        const int stride = n + 1;
        for (int i = tid; i <= n; i += NT) {
            int e = NJ;
            // levels of the leaves left (la) and right (lb) of the interface; the finest
            // cells e - 1 and e lie in them, so no window above min(la, lb) is inside R. With
            // SIG = 2 the cells e - 2 and e + 1 may lie in the next leaves out, at most one
            // level coarser (adjacent leaves differ by at most one level in a graded tree)
            int la, lb;
            if (i < n) {
                const uint32_t key = list[i];
                const int l = key >> 27, k = key & ((1u << 27) - 1u);
                e = k << (J - l);
                lb = l;
                la = i > 0 ? (int)(list[i - 1] >> 27) : (bc == CLAMP ? l : (int)(list[n - 1] >> 27));
            } else {
                la = (int)(list[n - 1] >> 27);
                lb = bc == CLAMP ? la : (int)(list[0] >> 27);
            }
            int ls = la < lb ? la : lb;
            if (SG > 1) ls = ls - 1 > jmin ? ls - 1 : jmin;
            int tA = e - SG, tB = e + SG - 1;
            if (bc == CLAMP) {
                tA = tA < 0 ? 0 : (tA > NJ - 1 ? NJ - 1 : tA);
                tB = tB < 0 ? 0 : (tB > NJ - 1 ? NJ - 1 : tB);
            }
            T win[Sch<S>::NM * NO];
            chain<T, G, Sch<S>::NM, MovingPops<S>, NO>(Vx, keep, rpn, jmin, J, bc, cc, tA, tB, win, ls);
#pragma unroll
            for (int m = 0; m < Sch<S>::NM; ++m) {
#pragma unroll
                for (int dl = 1; dl <= PLN::aw(m); ++dl) {
                    const int eta = PLN::eta(m, dl);
                    // the cell's position in the window: SG + eta, or under clamp the
                    // position of the clamped cell
                    T v = win[m * NO + SG + eta];
                    if (bc == CLAMP) {
                        int x = e + eta;
                        x = x < 0 ? 0 : (x > NJ - 1 ? NJ - 1 : x);
                        const int pos = x - tA;
#pragma unroll
                        for (int j = 0; j < NO; ++j) v = (pos == j) ? win[m * NO + j] : v;
                    }
                    P[(PLN::base(m) + dl - 1) * stride + i] = v;
                }
            }
        }
        __syncthreads();
    }

    // f^{n+1} of every leaf from its collided value and the interface values, in place
    // (eq. AdaptiveStreamPhase: the terms delta = 1..|w| summed in order; leaves at level J take
    // the reconstructed finest value at k - w, which the interface planes hold too).
    template <class V, class LP, class PP>
    DEV void combine(const V& Vx, const LP* list, const PP* P, int n) {
        typedef Planes<S> PLN;
        const int stride = n + 1;
        for (int i = tid; i < n; i += NT) {
            const uint32_t key = list[i];
            const int l = key >> 27, k = key & ((1u << 27) - 1u);
            const int s = rank_of(keep, rpn, jmin, l, k);
            // all loads first, then the stores (they never alias; the compiler cannot tell)
            T out[Q];
#pragma unroll
            for (int m = 0; m < Sch<S>::NM; ++m) {
                const int h = Sch<S>::mv(m);
                const int wh = Sch<S>::w(h);
                const int aw = PLN::aw(m);
                if (l == J) {
                    // k - w = e + eta(|w|) on the left interface (w > 0) or the right one (w < 0)
                    const int pl = PLN::base(m) + aw - 1;
                    out[h] = wh > 0 ? (T)P[pl * stride + i] : (T)P[pl * stride + i + 1];
                } else {
                    T acc = (T)0;
#pragma unroll
                    for (int dl = 1; dl <= aw; ++dl) {
                        const int pl = PLN::base(m) + dl - 1;
                        const T t = (T)P[pl * stride + i] - (T)P[pl * stride + i + 1];
                        acc = dl == 1 ? t : acc + t;
                    }
                    out[h] = Vx.ld(h, s) + (T)ldexp(wh > 0 ? acc : -acc, -(J - l));
                }
            }
#pragma unroll
            for (int m = 0; m < Sch<S>::NM; ++m) Vx.st(Sch<S>::mv(m), s, out[Sch<S>::mv(m)]);
        }
        for (int w = tid; w < lay.nwJ; w += NT) E[w] = 0ull;
        __syncthreads();
    }

    // ----------------------------------------------------------- predictor: judge / record
    // After the step (VN holds f^{n+1} on Lambda^{n+1}, its split cells projected). Learned
    // mode: a declined pair whose new detail still reaches the rule-(b) threshold is a miss;
    // it is forced for the redo; returns the number of misses. Record mode: every rule-(b)
    // pair becomes a sample, features from t^n, label 1 when declining it would have been
    // a miss.
    template <class VO_, class VN_>
    DEV void judge_or_record(const VO_& VO, const VN_& VN, int* s_miss) {
        int t = wave;
        for (int l = jmin; l < J; ++l) {
            const int n = nswl.c[l];
            const double thrb = ldexp(d.eps, d.mu_bar + 1 + l + 1 - J);
            for (; t < n; t += nwaves) {
                const int w = nswl.w[WB(l) + t];
                const uint64_t dec = declined[WB(l) + w];
                if (!dec) continue;
                bool miss = false;
                if ((dec >> lane) & 1ull) {
                    const int p = (w << 6) + lane;
                    const bool over = max_detail(VN, keep, rpn, l, p) >= thrb;
                    if (d.pmode == 1) {
                        miss = over;
                    } else {
                        const unsigned slot = atomicAdd(d.nsamples, 1u);
                        if (slot < (unsigned)d.sample_cap) {
                            float x[MLP_IN];
                            features(VO, l, p, x);
                            float* o = d.samples + (size_t)slot * (MLP_IN + 1);
#pragma unroll
                            for (int i = 0; i < MLP_IN; ++i) o[i] = x[i];
                            o[MLP_IN] = over ? 1.f : 0.f;
                        }
                    }
                }
                const uint64_t mw = __ballot(miss);
                if (lane == 0 && mw) {
                    forced[WB(l) + w] |= mw;
                    atomicAdd(s_miss, __popcll(mw));
                }
            }
            t -= n;
        }
        __syncthreads();
    }

    // ----------------------------------------------------------- rotation
    DEV void rotate() {
        uint64_t* t = split;
        split = nsplit;
        nsplit = t;
        t = ro;
        ro = keep;
        keep = t;
        uint32_t* r = rpo;
        rpo = rpn;
        rpn = r;
        WordList w = swl;
        swl = nswl;
        nswl = w;
    }
};

// Where the values of the current tree live during a launch.
enum : int { IN_LDS_A = 0, IN_LDS_B = 1, IN_HBM_0 = 2, IN_HBM_1 = 3 };

template <typename T>
DEV T* hbm_vals(const Desc& d, int which) { return reinterpret_cast<T*>(which ? d.vb : d.va); }

// nsteps time steps (or adaptations only) of run sched[blockIdx.x]. cap / capS: on-chip capacity in
// R(Lambda) cells and in leaves (0 = always use the HBM arrays). LRN: the variant that can run
// the refinement predictor (d.pmode != 0). RC: the variant that can run the reconstructed
// collision (runs with d.recon set; the others in the same launch use the leaves collision).
// BIG: the variant for runs whose tree arrays exceed LDS (J > 16): the tree arrays live in the
// run's device-memory copy d.gtree, the values in HBM, and no slot table is built.
template <typename T, int S, int G, bool LRN = false, bool RC = false, bool BIG = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu((G == 1 && !LRN && !RC && S <= 1) ? 4 : 1))) void k_steps(const Desc* __restrict__ descs, State* __restrict__ states,
                                               const int* __restrict__ sched, int nsteps, int mode, int cap, int capS) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_red[24];
    __shared__ int s_cnt[96];
    __shared__ int s_nan;
    __shared__ int s_miss;
    __shared__ int s_dec;
    typedef Block<T, S, G, LRN, BIG> B_t;
    typedef typename B_t::LT LT;
    constexpr int Q = B_t::Q;
    // the run of this workgroup: the launch schedule maps workgroups to runs (identity when null)
    const int run = sched ? sched[blockIdx.x] : (int)blockIdx.x;
    const Desc& d = descs[run];
    if constexpr (BIG) {
        cap = 0;
        capS = 0;
    }
    const Layout lay = make_layout(d.jmin, d.jmax, cap, capS, d.q, d.nm, (int)sizeof(T), LRN, BIG ? 4 : 2);
    B_t B(d, lay, BIG ? d.gtree : lds, lds, s_red, s_cnt);
    B.any_declined = &s_dec;
    const int Cg = (1 << (d.jmax + 1)) - (1 << d.jmin);  // slots of an HBM array
    if (threadIdx.x == 0) {
        s_nan = 0;
        s_miss = 0;
    }
    if (threadIdx.x < 24) s_red[threadIdx.x] = 0;
    const int wsplit = wbase(d.jmin, d.jmax);
    for (int w = threadIdx.x; w < lay.ws; w += blockDim.x) B.split[w] = d.split[w];
    for (int w = threadIdx.x; w < lay.nwJ; w += blockDim.x) B.E[w] = 0ull;
    __syncthreads();
    B.build_tree(B.split, B.ro, B.rpo, B.swl, nullptr, B.lwl);
    State& st = states[run];
    int where = st.cur ? IN_HBM_1 : IN_HBM_0;
    {
        const int nR = (int)B.rpo[lay.wt];
        if (nR <= cap) {
            const T* src = hbm_vals<T>(d, st.cur);
            for (int i = threadIdx.x; i < Q * nR; i += blockDim.x) {
                const int h = i / nR, s = i - h * nR;
                B.ldsA[h * cap + s] = src[(size_t)h * Cg + s];
            }
            where = IN_LDS_A;
            __syncthreads();
        }
    }
    // slot table of the current tree (plain kernels, trees on chip): projections without
    // per-cell slot lookups
    // (the table sits in the free array B)
    bool tvalid = false;
    const unsigned arrb = (unsigned)Q * (unsigned)cap * (unsigned)sizeof(T);  // one LDS value array
    if constexpr (!LRN) {
        if (where == IN_LDS_A)
            tvalid = B.build_table(B.split, B.ro, B.rpo, B.swl, (typename B_t::LU*)(lds + lay.VB), (int)(arrb / 4u));
        else if (cap > 0)  // values in HBM: both value arrays are free
            tvalid = B.build_table(B.split, B.ro, B.rpo, B.swl, (typename B_t::LU*)(lds + lay.VA),
                                   (int)((lay.VB + arrb - lay.VA) / 4u));
    }
    const bool scheme = (mode & MODE_SCHEME) != 0;
    // reconstructed collision: only the RC instances carry its code (it would raise the
    // register count of every other kernel)
    const bool recon = RC && !LRN && d.recon != 0;
    const bool judge = LRN && scheme && (d.pmode == 2 || (d.pmode == 1 && d.mlp != nullptr));
    long long upd = 0, misses = 0, redos = 0;
    int last = -1, lastn = -1;  // leaves of the last step's tree (scheme steps / any step)
    bool last_lds_list = false;  // the last scheme step's leaf list is in LDS (B.ldsL)
    // the adaptation's decision bits, the new tree's word counts and leaf count start cleared
    // (all of them dead since the last step's lists were used)
    auto clear_decisions = [&]() {
        for (int w = threadIdx.x; w < lay.wt; w += blockDim.x) {
            B.keep[w] = 0ull;
            B.ruleb[w] = 0ull;
            if constexpr (LRN)
                if (w < lay.ws) B.declined[w] = 0ull;
        }
        if (threadIdx.x == 0) s_dec = 0;
        if (threadIdx.x < 32) {
            B.nswl.c[threadIdx.x] = 0;
            B.lwl.c[threadIdx.x] = 0;
        }
        if (threadIdx.x == 0) B.red[0] = 0;
    };
    for (int stp = 0; stp < nsteps; ++stp) {
        // ---- projection of f^n up the old tree (once per step, kept through redos); the
        // clearing touches none of its data, and its barriers order the clearing before the
        // details
        if constexpr (LRN)
            for (int w = threadIdx.x; w < lay.ws; w += blockDim.x) B.forced[w] = 0ull;
        clear_decisions();
        bool psync;
        if (where <= IN_LDS_B) {
            VP<T, LT> VO{where == IN_LDS_A ? B.ldsA : B.ldsB, cap};
            psync = tvalid ? B.project_table(VO) : B.project_up(VO, B.split, B.ro, B.rpo, B.swl);
        } else {
            VP<T, T> VO{hbm_vals<T>(d, where - IN_HBM_0), Cg};
            psync = tvalid ? B.project_table(VO) : B.project_up(VO, B.split, B.ro, B.rpo, B.swl);
        }
        if (!psync) __syncthreads();
        int nwhere = where, n = 0;
        bool fast = false;
        int attempt = 0;
        for (;;) {
            // ---- adaptation on the old tree (a redo starts from cleared decisions again)
            if (attempt > 0) {
                clear_decisions();
                __syncthreads();
            }
            if (where <= IN_LDS_B) {
                VP<T, LT> VO{where == IN_LDS_A ? B.ldsA : B.ldsB, cap};
                if (!LRN && tvalid) B.details_table(VO, &s_nan);
                else B.details(VO, &s_nan);
            } else {
                VP<T, T> VO{hbm_vals<T>(d, where - IN_HBM_0), Cg};
                if (!LRN && tvalid) B.details_table(VO, &s_nan);
                else B.details(VO, &s_nan);
            }
            __syncthreads();
            B.enlarge();
            B.grade();
            B.build_tree(B.nsplit, B.keep, B.rpn, B.nswl, B.ruleb, B.lwl, true);
            const int nR = (int)B.rpn[lay.wt];
            n = (int)B.red[0];
            // ---- new values: on chip when the new tree fits
            if (where <= IN_LDS_B) nwhere = (nR <= cap) ? (IN_LDS_B - where) : IN_HBM_0;
            else nwhere = (nR <= cap) ? IN_LDS_A : (where == IN_HBM_0 ? IN_HBM_1 : IN_HBM_0);
            fast = (where <= IN_LDS_B) && (nwhere <= IN_LDS_B) && (n <= capS) &&
                   (LRN || (unsigned)(Planes<S>::PL * (n + 1)) * sizeof(T) + 4u * (unsigned)n <=
                               (unsigned)(Q * cap) * sizeof(T));
            if (threadIdx.x == 0) s_miss = 0;
            if constexpr (!LRN) tvalid = false;
            if (fast) {
                VP<T, LT> VO{where == IN_LDS_A ? B.ldsA : B.ldsB, cap};
                VP<T, LT> VN{nwhere == IN_LDS_A ? B.ldsA : B.ldsB, cap};
                B.transfer(VO, VN, scheme && !recon, scheme, &s_nan);
                if constexpr (!LRN) {
                    // the old array, dead until the next transfer, holds the interface pairs,
                    // then this step's leaf list, then the new tree's table (read by the next
                    // step's projection and details)
                    const int pe = Planes<S>::PL * (n + 1);
                    const unsigned loff = (where == IN_LDS_A ? lay.VA : lay.VB) + (unsigned)pe * sizeof(T);
                    B.ldsL = reinterpret_cast<uint32_t*>(lds + loff);
                    const unsigned toff_ = loff + 4u * (unsigned)n;
                    // a scheme step's edge scan follows: its barriers order the table writes
                    tvalid = B.build_table(B.nsplit, B.keep, B.rpn, B.nswl, (typename B_t::LU*)(lds + toff_),
                                           (int)(((unsigned)(Q * cap - pe) * sizeof(T) - 4u * (unsigned)n) / 4u),
                                           !scheme);
                }
                if (scheme) {
                    B.scan_edges();
                    // the list and the projection touch different arrays: the projection's
                    // barriers (or one here, when it has none) order both before the pairs
                    B.write_list(B.ldsL, false);
                    if constexpr (RC && !LRN) {
                        if (recon) {
                            // f^n up the new tree, then the leaves collide on its reconstruction
                            // (the finest cells' equilibria go to the run's HBM pairs array, free
                            // until the stream: 2 nm (2^J + 1) values, at least NE 2^J)
                            const bool sy = tvalid ? B.project_table(VN)
                                                   : B.project_up(VN, B.nsplit, B.keep, B.rpn, B.nswl);
                            if (!sy) __syncthreads();
                            B.recon_collide(VN, B.ldsL, reinterpret_cast<T*>(d.pairs), n, &s_nan);
                        }
                    }
                    // the stream reads only the moving populations above the leaves, and the
                    // next step projects every population again from the leaves
                    const bool synced =
                        tvalid ? B.template project_table<MovingPops<S>, B_t::NM>(VN)
                               : B.template project_up<MovingPops<S>, B_t::NM>(VN, B.nsplit, B.keep, B.rpn, B.nswl);
                    if (!synced) __syncthreads();
                    if constexpr (LRN) {
                        T* PH = reinterpret_cast<T*>(d.pairs);
                        B.pairs(VN, B.ldsL, PH, n);
                        B.combine(VN, B.ldsL, PH, n);
                    } else {
                        LT* PB = where == IN_LDS_A ? B.ldsA : B.ldsB;
                        B.pairs(VN, B.ldsL, PB, n);
                        B.combine(VN, B.ldsL, PB, n);
                    }
                }
                if constexpr (LRN) {
                    if (judge && (d.pmode == 2 || s_dec)) {
                        B.project_up(VN, B.nsplit, B.keep, B.rpn, B.nswl);
                        B.judge_or_record(VO, VN, &s_miss);
                    }
                }
            } else {
                T* po = where <= IN_LDS_B ? (T*)(where == IN_LDS_A ? B.ldsA : B.ldsB) : hbm_vals<T>(d, where - IN_HBM_0);
                const int so = where <= IN_LDS_B ? cap : Cg;
                T* pn = nwhere <= IN_LDS_B ? (T*)(nwhere == IN_LDS_A ? B.ldsA : B.ldsB) : hbm_vals<T>(d, nwhere - IN_HBM_0);
                const int sn = nwhere <= IN_LDS_B ? cap : Cg;
                VP<T, T> VO{po, so};
                VP<T, T> VN{pn, sn};
                B.transfer(VO, VN, scheme && !recon, scheme, &s_nan);
                // From here to the next transfer the LDS value arrays that do not hold the new
                // values are free (the old array too, once the transfer has read it): the
                // interface planes and the leaf list go there when they fit, as on chip, then
                // the new tree's slot table; otherwise planes and list go to the run's HBM arrays
                bool lds_lists = false;
                if constexpr (!LRN) {
                    unsigned f0 = 0, f1 = 0;
                    if (cap > 0) {
                        if (nwhere == IN_LDS_A) {
                            f0 = lay.VB;
                            f1 = lay.VB + arrb;
                        } else if (nwhere == IN_LDS_B) {
                            f0 = lay.VA;
                            f1 = lay.VA + arrb;
                        } else {
                            f0 = lay.VA;
                            f1 = lay.VB + arrb;
                        }
                    }
                    const unsigned pe = (unsigned)(Planes<S>::PL * (n + 1)) * (unsigned)sizeof(T);
                    unsigned toff_ = f0;
                    if (scheme && f0 + pe + 4u * (unsigned)n <= f1) {
                        lds_lists = true;
                        B.ldsL = reinterpret_cast<uint32_t*>(lds + f0 + pe);
                        toff_ = f0 + pe + 4u * (unsigned)n;
                    }
                    if (f1 > toff_)
                        tvalid = B.build_table(B.nsplit, B.keep, B.rpn, B.nswl, (typename B_t::LU*)(lds + toff_),
                                               (int)((f1 - toff_) / 4u), !scheme);
                    if (scheme && lds_lists) {
                        B.scan_edges();
                        B.write_list(B.ldsL, false);
                        if constexpr (RC) {
                            if (recon) {
                                const bool sy = tvalid ? B.project_table(VN)
                                                       : B.project_up(VN, B.nsplit, B.keep, B.rpn, B.nswl);
                                if (!sy) __syncthreads();
                                B.recon_collide(VN, B.ldsL, reinterpret_cast<T*>(d.pairs), n, &s_nan);
                            }
                        }
                        const bool synced =
                            tvalid ? B.template project_table<MovingPops<S>, B_t::NM>(VN)
                                   : B.template project_up<MovingPops<S>, B_t::NM>(VN, B.nsplit, B.keep, B.rpn, B.nswl);
                        if (!synced) __syncthreads();
                        LT* PB = (LT*)(T*)(lds + f0);
                        B.pairs(VN, B.ldsL, PB, n);
                        B.combine(VN, B.ldsL, PB, n);
                    }
                }
                if (scheme && !lds_lists) {
                    B.scan_edges();
                    B.write_list(d.list);
                    T* P = reinterpret_cast<T*>(d.pairs);
                    if constexpr (RC && !LRN) {
                        if (recon) {
                            const bool sy = tvalid ? B.project_table(VN)
                                                   : B.project_up(VN, B.nsplit, B.keep, B.rpn, B.nswl);
                            if (!sy) __syncthreads();
                            B.recon_collide(VN, d.list, P, n, &s_nan);
                        }
                    }
                    const bool synced =
                        tvalid ? B.template project_table<MovingPops<S>, B_t::NM>(VN)
                               : B.template project_up<MovingPops<S>, B_t::NM>(VN, B.nsplit, B.keep, B.rpn, B.nswl);
                    if (!synced) __syncthreads();
                    B.pairs(VN, d.list, P, n);
                    B.combine(VN, d.list, P, n);
                }
                last_lds_list = lds_lists;
                if constexpr (LRN) {
                    if (judge && (d.pmode == 2 || s_dec)) {
                        B.project_up(VN, B.nsplit, B.keep, B.rpn, B.nswl);
                        B.judge_or_record(VO, VN, &s_miss);
                    }
                }
            }
            if (!judge || d.pmode != 1) break;
            const int nm = s_miss;  // written before the barrier that ends judge_or_record
            if (nm == 0) break;
            misses += nm;
            ++redos;
            ++attempt;
            __syncthreads();
            if constexpr (LRN) {
                // after a few redos every rule-(b) pair is forced: the plain rule, no misses
                if (attempt >= 8)
                    for (int w = threadIdx.x; w < lay.ws; w += blockDim.x) B.forced[w] = ~0ull;
            }
        }
        B.rotate();
        where = nwhere;
        lastn = n;
        if (scheme) {
            upd += n;
            last = n;
            if (fast) last_lds_list = true;
        }
        // no barrier here: every path above ends with one, and nothing until the next step's
        // first barrier writes what another wave may still read
    }
    // ---- epilogue: home copy, tree, leaf list of the last step, statistics
    const int nR = (int)B.rpo[lay.wt];
    int home;
    if (where <= IN_LDS_B) {
        home = st.cur;  // the array the launch started from is free to overwrite
        T* dst = hbm_vals<T>(d, home);
        const LT* src = where == IN_LDS_A ? B.ldsA : B.ldsB;
        for (int i = threadIdx.x; i < Q * nR; i += blockDim.x) {
            const int h = i / nR, s = i - h * nR;
            dst[(size_t)h * Cg + s] = src[h * cap + s];
        }
    } else {
        home = where - IN_HBM_0;
    }
    if (last >= 0 && last_lds_list)
        for (int i = threadIdx.x; i < last; i += blockDim.x) d.list[i] = B.ldsL[i];
    for (int w = threadIdx.x; w < wsplit; w += blockDim.x) d.split[w] = B.split[w];
    if (threadIdx.x == 0) {
        st.cur = home;
        if (mode & MODE_SCHEME) {
            st.steps += nsteps;
            st.leaf_updates += upd;
        }
        if (lastn >= 0) st.n_leaves = lastn;
        st.n_r = nR;
        st.misses += misses;
        st.redos += redos;
        if (s_nan) st.flags |= 1;
    }
}

// Initial state: populations at equilibrium on the finest level of the full tree.
template <typename T, int S>
__global__ void k_init(const Desc* __restrict__ descs, State* __restrict__ states, const double* __restrict__ mc,
                       long long mc_stride) {
    const Desc& d = descs[blockIdx.y];
    const int NJ = 1 << d.jmax;
    const int Cg = (1 << (d.jmax + 1)) - (1 << d.jmin);
    const int base = (1 << d.jmax) - (1 << d.jmin);  // slot of (J, 0) in the full tree
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const double* m = mc + blockIdx.y * mc_stride;
    if (k < NJ) {
        double c[MAXQ];
        for (int i = 0; i < d.qc; ++i) c[i] = m[(size_t)i * NJ + k];
        T f[Sch<S>::Q];
        equilibrium<T, S>(d.cf, c, f);
        T* v = reinterpret_cast<T*>(d.va);
        for (int h = 0; h < Sch<S>::Q; ++h) v[(size_t)h * Cg + base + k] = f[h];
    }
    const int wsplit = wbase(d.jmin, d.jmax);
    for (int w = k; w < wsplit; w += gridDim.x * blockDim.x) {
        int l = d.jmin;
        while (w >= wbase(d.jmin, l + 1)) ++l;
        d.split[w] = lowmask(1 << l);
    }
    if (k == 0) {
        State& s = states[blockIdx.y];
        s.steps = 0;
        s.leaf_updates = 0;
        s.n_leaves = NJ;
        s.n_r = Cg;
        s.cur = 0;
        s.flags = 0;
        s.misses = 0;
        s.redos = 0;
    }
}

// Queries on the home copy: leaf list of the current tree, then per leaf (where = 0) its
// conserved moments (what = 0) or populations (what = 1), or (where = 1) the reconstruction on
// every finest cell followed by its conserved moments or populations. Output [component][position].
template <typename T, int S, int G, bool BIG = false>
__global__ __launch_bounds__(512) void k_query(const Desc* __restrict__ descs, State* __restrict__ states,
                                               int where, int what, double* __restrict__ out) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_red[24];
    __shared__ int s_cnt[96];
    typedef Block<T, S, G, false, BIG> B_t;
    constexpr int Q = B_t::Q;
    const Desc& d = descs[blockIdx.x];
    const Layout lay = make_layout(d.jmin, d.jmax, 0, 0, d.q, d.nm, (int)sizeof(T), false, BIG ? 4 : 2);
    B_t B(d, lay, BIG ? d.gtree : lds, lds, s_red, s_cnt);
    const int Cg = (1 << (d.jmax + 1)) - (1 << d.jmin);
    if (threadIdx.x < 24) s_red[threadIdx.x] = 0;
    for (int w = threadIdx.x; w < lay.ws; w += blockDim.x) B.split[w] = d.split[w];
    for (int w = threadIdx.x; w < lay.nwJ; w += blockDim.x) B.E[w] = 0ull;
    __syncthreads();
    // The current tree plays the role of the "new" tree of a step (keep = R bits, ruleb = leaf bits).
    for (int w = threadIdx.x; w < lay.ws; w += blockDim.x) B.nsplit[w] = B.split[w];
    __syncthreads();
    B.build_tree(B.nsplit, B.keep, B.rpn, B.nswl, B.ruleb, B.lwl);
    const int n = (int)B.red[0];
    VP<T, T> V{hbm_vals<T>(d, states[blockIdx.x].cur), Cg};
    // mark edges, rank, list
    {
        int t = B.wave;
        for (int l = B.jmin; l <= B.J; ++l) {
            const int nn = B.lwl.c[l];
            for (; t < nn; t += B.nwaves) {
                const int w = B.lwl.w[B.WB(l) + t];
                const uint64_t b = B.ruleb[B.WB(l) + w];
                if ((b >> B.lane) & 1ull) {
                    const int k = (w << 6) + B.lane;
                    const int e = k << (B.J - l);
                    atomicOr((unsigned long long*)&B.E[e >> 6], 1ull << (e & 63));
                }
            }
            t -= nn;
        }
        __syncthreads();
    }
    B.scan_edges();
    B.write_list(d.list);
    if (where == 0) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t key = d.list[i];
            const int l = key >> 27, k = key & ((1u << 27) - 1u);
            const int s = rank_of(B.keep, B.rpn, B.jmin, l, k);
            T f[Q];
            for (int h = 0; h < Q; ++h) f[h] = V.ld(h, s);
            if (what == 0) {
                double mc[MAXQ];
                conserved<T, S>(d.cf, f, mc);
                for (int c = 0; c < d.qc; ++c) out[(size_t)c * n + i] = mc[c];
            } else {
                for (int h = 0; h < Q; ++h) out[(size_t)h * n + i] = (double)f[h];
            }
        }
    } else {
        B.project_up(V, B.nsplit, B.keep, B.rpn, B.nswl);
        const int NJ = 1 << d.jmax;
        for (int m = threadIdx.x; m < NJ; m += blockDim.x) {
            T a[Q];
            chain<T, G, Q, AllPops<S>, 1>(V, B.keep, B.rpn, B.jmin, B.J, B.bc, B.cc, m, m, a, B.J);
            if (what == 0) {
                double mc[MAXQ];
                conserved<T, S>(d.cf, a, mc);
                for (int c = 0; c < d.qc; ++c) out[(size_t)c * NJ + m] = mc[c];
            } else {
                for (int h = 0; h < Q; ++h) out[(size_t)h * NJ + m] = (double)a[h];
            }
        }
    }
    if (threadIdx.x == 0) {
        states[blockIdx.x].n_leaves = n;
        states[blockIdx.x].n_r = (int)B.rpn[lay.wt];
    }
}

}  // namespace mrl
