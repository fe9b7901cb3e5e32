// mrlbm.hip -- host side of the C ABI declared in include/mrlbm.h.
//
// The library validates parameters on the host, allocates one device pool per handle
// (values, tree words, leaf list, interface pairs for every run), starts each run at
// equilibrium on the full tree, and advances runs with the workgroup-per-run kernel of
// mrlbm_kernels.h. Batched steps are captured once per (nsteps, block size) in a HIP graph
// and replayed.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mrlbm.h"
#include "mrlbm_kernels.h"

// The kernels are instantiated in instances.hip (one object per storage type and scheme).
namespace mrl {
#define MRL_EXTERN(T, S)                                                                        \
    extern template __global__ void k_init<T, S>(const Desc*, State*, const double*, long long); \
    extern template __global__ void k_steps<T, S, 1>(const Desc*, State*, const int*, int, int, int, int);   \
    extern template __global__ void k_steps<T, S, 2>(const Desc*, State*, const int*, int, int, int, int);   \
    extern template __global__ void k_steps<T, S, 3>(const Desc*, State*, const int*, int, int, int, int);   \
    extern template __global__ void k_query<T, S, 1>(const Desc*, State*, int, int, double*);    \
    extern template __global__ void k_query<T, S, 2>(const Desc*, State*, int, int, double*);    \
    extern template __global__ void k_query<T, S, 3>(const Desc*, State*, int, int, double*);          \
    extern template __global__ void k_steps<T, S, 1, true>(const Desc*, State*, const int*, int, int, int, int); \
    extern template __global__ void k_steps<T, S, 1, false, false, true>(const Desc*, State*, const int*, int, int, int, int); \
    extern template __global__ void k_steps<T, S, 2, false, false, true>(const Desc*, State*, const int*, int, int, int, int); \
    extern template __global__ void k_steps<T, S, 3, false, false, true>(const Desc*, State*, const int*, int, int, int, int); \
    extern template __global__ void k_query<T, S, 1, true>(const Desc*, State*, int, int, double*);   \
    extern template __global__ void k_query<T, S, 2, true>(const Desc*, State*, int, int, double*);   \
    extern template __global__ void k_query<T, S, 3, true>(const Desc*, State*, int, int, double*);   \
    extern template __global__ void k_steps<T, S, 1, false, true>(const Desc*, State*, const int*, int, int, int, int);
MRL_EXTERN(double, 0)
MRL_EXTERN(double, 1)
MRL_EXTERN(double, 2)
MRL_EXTERN(double, 3)
MRL_EXTERN(double, 4)
#undef MRL_EXTERN
#define MRL_EXTERN32(T, S)                                                                      \
    extern template __global__ void k_init<T, S>(const Desc*, State*, const double*, long long); \
    extern template __global__ void k_steps<T, S, 1>(const Desc*, State*, const int*, int, int, int, int);   \
    extern template __global__ void k_steps<T, S, 2>(const Desc*, State*, const int*, int, int, int, int);   \
    extern template __global__ void k_steps<T, S, 3>(const Desc*, State*, const int*, int, int, int, int);   \
    extern template __global__ void k_query<T, S, 1>(const Desc*, State*, int, int, double*);    \
    extern template __global__ void k_query<T, S, 2>(const Desc*, State*, int, int, double*);    \
    extern template __global__ void k_query<T, S, 3>(const Desc*, State*, int, int, double*);         \
    extern template __global__ void k_steps<T, S, 1, false, false, true>(const Desc*, State*, const int*, int, int, int, int); \
    extern template __global__ void k_steps<T, S, 2, false, false, true>(const Desc*, State*, const int*, int, int, int, int); \
    extern template __global__ void k_steps<T, S, 3, false, false, true>(const Desc*, State*, const int*, int, int, int, int); \
    extern template __global__ void k_query<T, S, 1, true>(const Desc*, State*, int, int, double*);   \
    extern template __global__ void k_query<T, S, 2, true>(const Desc*, State*, int, int, double*);   \
    extern template __global__ void k_query<T, S, 3, true>(const Desc*, State*, int, int, double*);   \
    extern template __global__ void k_steps<T, S, 1, false, true>(const Desc*, State*, const int*, int, int, int, int);
MRL_EXTERN32(float, 0)
MRL_EXTERN32(float, 1)
MRL_EXTERN32(float, 2)
MRL_EXTERN32(float, 3)
MRL_EXTERN32(float, 4)
#undef MRL_EXTERN32
}  // namespace mrl

using namespace mrl;

namespace {

struct Engine {
    int n = 0, prec = 0, scheme = 0, gamma = 1;
    std::vector<mrlbm_params> P;
    std::vector<Desc> hd;
    std::vector<size_t> voff;
    Desc* dd = nullptr;
    State* ds = nullptr;
    int* d_sched = nullptr;       // workgroup -> run (null: identity)
    int launch_max = 0;           // steps per launch (0: all steps of a call in one launch)
    int sched_stride = 0;         // 0: identity; else heavy/light pairs (b, b + stride)
    char* pool = nullptr;
    size_t pool_bytes = 0;
    double* stage = nullptr;
    size_t stage_elems = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t lds = 0;        // dynamic LDS of the step kernel (bytes)
    size_t lds_query = 0;  // dynamic LDS of the query kernel
    int cap = 0, capS = 0; // on-chip capacity in R(Lambda) cells and in leaves
    size_t lds_budget = 0; // LDS bytes one workgroup may use
    size_t lds_full = 0;   // the device's budget for one workgroup (lds_budget at create)
    int cap_user = -1;     // user limit on the on-chip capacity (-1: none)
    int maxJ = 0;
    int nt = 0;          // threads per workgroup in use
    int nt_user = 0;     // 0: tuner choice
    bool numeric = false;
    char* ckpt = nullptr;      // checkpoint of the pool (mrlbm_batch_checkpoint)
    State* ckpt_s = nullptr;   // and of the per-run states
    bool ckpt_numeric = false;
    std::string err;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int gsteps = -1, gnt = -1, gcap = -1;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // launch classes (empty: one launch for the whole batch); class c advances the runs
    // d_sched[first, first + count) with its own workgroup size and on-chip capacity
    struct LaunchClass {
        int first = 0, count = 0, jhi = 0, nt = 512, per_cu = 1, cap = 0, capS = 0;
        size_t lds = 0;
    };
    std::vector<LaunchClass> cls;
    int cls_gen = 0, gcls = -1;           // generation of the class set (graph cache key)
    hipStream_t side = nullptr;           // second stream: class launches run side by side
    hipEvent_t evf = nullptr, evj = nullptr;
    // refinement predictor
    bool big = false;             // runs beyond the on-chip J: tree arrays in device memory
    bool lrn = false;             // launch the predictor-capable kernels
    bool any_recon = false;       // some run uses the reconstructed collision
    uint16_t* d_mlp = nullptr;
    float* d_samples = nullptr;
    unsigned int* d_nsamples = nullptr;
    long long sample_cap = 0;    // samples the current record may hold
    long long sample_alloc = 0;  // rows of d_samples
};

thread_local std::string g_create_error;

struct SchemeInfo {
    int q, qc, nm;
};

bool scheme_info(int scheme, int physics, SchemeInfo* si) {
    if (scheme == MRLBM_D1Q2 && (physics == MRLBM_ADVECTION || physics == MRLBM_BURGERS)) {
        *si = {2, 1, 2};
        return true;
    }
    if (scheme == MRLBM_D1Q3 && physics == MRLBM_BURGERS) {
        *si = {3, 1, 2};
        return true;
    }
    if (scheme == MRLBM_D1Q3 && physics == MRLBM_SHALLOW_WATER) {
        *si = {3, 2, 2};
        return true;
    }
    if (scheme == MRLBM_D1Q2x2 && physics == MRLBM_SHALLOW_WATER) {
        *si = {4, 2, 4};
        return true;
    }
    if (scheme == MRLBM_D1Q2x3 && physics == MRLBM_EULER) {
        *si = {6, 3, 6};
        return true;
    }
    if (scheme == MRLBM_D1Q5 && physics == MRLBM_SHALLOW_WATER) {
        *si = {5, 2, 4};
        return true;
    }
    return false;
}

int validate(const mrlbm_params* p, std::string* why) {
    auto bad = [&](const char* m) {
        if (why) *why = m;
        return (int)MRLBM_EINVAL;
    };
    if (!p) return bad("params is NULL");
    if (p->abi_version != MRLBM_ABI_VERSION) return bad("abi_version mismatch");
    SchemeInfo si;
    if (!scheme_info(p->scheme, p->physics, &si)) return bad("unsupported scheme/physics pair");
    if (p->bc != MRLBM_PERIODIC && p->bc != MRLBM_CLAMP) return bad("bc must be PERIODIC or CLAMP");
    if (p->precision != MRLBM_FP64 && p->precision != MRLBM_FP32_STORAGE) return bad("unknown precision");
    if (!(p->lambda > 0.0) || !isfinite(p->lambda)) return bad("lambda must be finite and > 0");
    const int nn = si.q - si.qc;
    if (p->n_s != 1 && p->n_s != nn) return bad("n_s must be 1 or q - q_cons");
    for (int i = 0; i < p->n_s; ++i)
        if (!(p->s[i] > 0.0 && p->s[i] <= 2.0)) return bad("relaxation rates must lie in (0, 2]");
    if (!isfinite(p->x_min) || !isfinite(p->x_max) || !(p->x_max > p->x_min)) return bad("need x_min < x_max");
    if (p->gamma < 1 || p->gamma > 3) return bad("gamma must be 1, 2 or 3");
    if (p->j_min < 0 || p->j_min > p->j_max) return bad("need 0 <= j_min <= j_max");
    if (p->bc == MRLBM_PERIODIC && (1 << p->j_min) < 2 * p->gamma + 1)
        return bad("periodic coarsest level needs 2^j_min >= 2 gamma + 1");
    if (p->mu_bar < 0 || p->mu_bar > 30) return bad("mu_bar must be in 0..30");
    if (!(p->eps >= 0.0) || !isfinite(p->eps)) return bad("eps must be finite and >= 0");
    if ((p->flags & ~(uint32_t)MRLBM_FLAG_RECONSTRUCTED_COLLISION) != 0)
        return bad("flags: only MRLBM_FLAG_RECONSTRUCTED_COLLISION is defined");
    if ((p->flags & MRLBM_FLAG_RECONSTRUCTED_COLLISION) && p->gamma != 1)
        return bad("the reconstructed collision runs with gamma = 1");
    if ((p->flags & MRLBM_FLAG_RECONSTRUCTED_COLLISION) && p->j_max > MRLBM_ONCHIP_MAX_J)
        return bad("the reconstructed collision runs with j_max <= MRLBM_ONCHIP_MAX_J");
    if (p->physics == MRLBM_SHALLOW_WATER && !(p->phys[1] > 0.0)) return bad("gravity must be > 0");
    if (p->physics == MRLBM_EULER && !(p->phys[2] > 1.0)) return bad("gamma_gas must be > 1");
    if (p->scheme == MRLBM_D1Q3 && p->physics == MRLBM_BURGERS && !(p->phys[3] > 0.0))
        return bad("alpha must be > 0");
    for (int i = 0; i < 4; ++i)
        if (!isfinite(p->phys[i])) return bad("physical parameters must be finite");
    if (p->j_max > MRLBM_MAX_J) {
        if (why) *why = "j_max beyond MRLBM_MAX_J";
        return MRLBM_ECAPACITY;
    }
    return MRLBM_OK;
}

Coef make_coef(const mrlbm_params* p, const SchemeInfo& si) {
    Coef c;
    memset(&c, 0, sizeof(c));
    c.lam = p->lambda;
    c.lam2 = p->lambda * p->lambda;
    c.V = p->phys[0];
    c.alam2 = p->phys[3] * c.lam2;
    c.g2 = 0.5 * p->phys[1];
    c.gam = p->phys[2];
    c.k3 = 0.5 * (3.0 - c.gam);
    c.gm1 = c.gam - 1.0;
    c.k5 = 0.5 * (1.0 - c.gam);
    const int nn = si.q - si.qc;
    for (int i = 0; i < nn; ++i) {
        c.s[i] = p->n_s == 1 ? p->s[0] : p->s[i];
        c.oms[i] = 1.0 - c.s[i];
    }
    c.physics = p->physics;
    c.qc = si.qc;
    int ex = 0;
    c.lam_pow2 = std::frexp(p->lambda, &ex) == 0.5 ? 1 : 0;
    c.ilam = 1.0 / c.lam;
    c.ilam2 = 1.0 / c.lam2;
    c.lam3 = c.lam2 * c.lam;
    c.lam4 = c.lam2 * c.lam2;
    c.ilam3 = 1.0 / c.lam3;
    c.ilam4 = 1.0 / c.lam4;
    // D1Q5: alpha lambda^2 (alam2, phys[3]) and beta lambda^2 with beta in phys[0]
    c.blam2 = p->scheme == MRLBM_D1Q5 ? p->phys[0] * c.lam2 : 0.0;
    return c;
}

void pred_coeffs(int gamma, double* c) {
    c[0] = c[1] = c[2] = 0.0;
    if (gamma == 1) {
        c[0] = -1.0 / 8.0;
    } else if (gamma == 2) {
        c[0] = -22.0 / 128.0;
        c[1] = 3.0 / 128.0;
    } else {
        // Sec. 3.1 prints +5/1024 for c_3; exactness on odd degrees requires -5/1024.
        c[0] = -201.0 / 1024.0;
        c[1] = 11.0 / 256.0;
        c[2] = -5.0 / 1024.0;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Largest on-chip capacity (cells of R(Lambda)) whose LDS layout fits the budget for every
// run of the batch; never more than the full tree of the largest run.
void choose_capacity(Engine* e) {
    if (e->big) {  // tree arrays and values in device memory: nothing on chip
        e->cap = e->capS = 0;
        e->lds = e->lds_query = 0;
        return;
    }
    int cg_max = 0;
    for (auto& d : e->hd) cg_max = std::max(cg_max, (1 << (d.jmax + 1)) - (1 << d.jmin));
    const int tsz = e->prec == MRLBM_FP64 ? 8 : 4;
    auto total = [&](int cap) {
        size_t t = 0;
        for (auto& d : e->hd) {
            const int capS = cap > 0 ? cap / 2 + (1 << d.jmin) : 0;
            t = std::max(t, (size_t)make_layout(d.jmin, d.jmax, cap, capS, d.q, d.nm, tsz, e->lrn).total);
        }
        return t;
    };
    int lo = 0, hi = cg_max;
    if (e->cap_user >= 0) hi = std::min(hi, e->cap_user);
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (total(mid) <= e->lds_budget) lo = mid;
        else hi = mid - 1;
    }
    e->cap = lo;
    int jmin_min = 30;
    for (auto& d : e->hd) jmin_min = std::min(jmin_min, d.jmin);
    e->capS = lo > 0 ? lo / 2 + (1 << jmin_min) : 0;
    e->lds = total(lo);
    size_t q = 0;
    for (auto& d : e->hd) q = std::max(q, (size_t)make_layout(d.jmin, d.jmax, 0, 0, d.q, d.nm, tsz).total);
    e->lds_query = q;
}

// ---------------------------------------------------------------- kernel dispatch
typedef void (*StepK)(const Desc*, State*, const int*, int, int, int, int);
typedef void (*QueryK)(const Desc*, State*, int, int, double*);
typedef void (*InitK)(const Desc*, State*, const double*, long long);

template <typename T, int S, int G>
void pick(bool big, StepK* s, QueryK* q) {
    *s = big ? k_steps<T, S, G, false, false, true> : k_steps<T, S, G>;
    *q = big ? k_query<T, S, G, true> : k_query<T, S, G>;
}

StepK lrn_kernel(int scheme) {
    switch (scheme) {
        case 0: return k_steps<double, 0, 1, true>;
        case 1: return k_steps<double, 1, 1, true>;
        case 2: return k_steps<double, 2, 1, true>;
        case 3: return k_steps<double, 3, 1, true>;
        default: return k_steps<double, 4, 1, true>;
    }
}

// Step kernels that can run the reconstructed collision (gamma = 1).
StepK rc_kernel(int prec, int scheme) {
    if (prec == MRLBM_FP64) {
        switch (scheme) {
            case 0: return k_steps<double, 0, 1, false, true>;
            case 1: return k_steps<double, 1, 1, false, true>;
            case 2: return k_steps<double, 2, 1, false, true>;
            case 3: return k_steps<double, 3, 1, false, true>;
            default: return k_steps<double, 4, 1, false, true>;
        }
    }
    switch (scheme) {
        case 0: return k_steps<float, 0, 1, false, true>;
        case 1: return k_steps<float, 1, 1, false, true>;
        case 2: return k_steps<float, 2, 1, false, true>;
        case 3: return k_steps<float, 3, 1, false, true>;
        default: return k_steps<float, 4, 1, false, true>;
    }
}

bool kernels_for(int prec, int scheme, int gamma, bool big, StepK* s, QueryK* q, InitK* in) {
#define MRL_CASE(P, TT, SS)                                               \
    if (prec == P && scheme == SS) {                                      \
        *in = k_init<TT, SS>;                                             \
        if (gamma == 1) { pick<TT, SS, 1>(big, s, q); return true; }      \
        if (gamma == 2) { pick<TT, SS, 2>(big, s, q); return true; }      \
        if (gamma == 3) { pick<TT, SS, 3>(big, s, q); return true; }      \
    }
    MRL_CASE(0, double, 0)
    MRL_CASE(0, double, 1)
    MRL_CASE(0, double, 2)
    MRL_CASE(0, double, 3)
    MRL_CASE(0, double, 4)
    MRL_CASE(1, float, 0)
    MRL_CASE(1, float, 1)
    MRL_CASE(1, float, 2)
    MRL_CASE(1, float, 3)
    MRL_CASE(1, float, 4)
#undef MRL_CASE
    return false;
}

int hip_fail(Engine* e, hipError_t st, const char* what) {
    e->err = std::string(what) + ": " + hipGetErrorString(st);
    return st == hipErrorOutOfMemory ? MRLBM_ENOMEM : MRLBM_EDEVICE;
}

int default_block(int maxJ) {
    if (maxJ <= 9) return 128;
    if (maxJ <= 12) return 256;
    return 512;
}

void engine_free(Engine* e) {
    if (!e) return;
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    if (e->ev0) (void)hipEventDestroy(e->ev0);
    if (e->ev1) (void)hipEventDestroy(e->ev1);
    if (e->evf) (void)hipEventDestroy(e->evf);
    if (e->evj) (void)hipEventDestroy(e->evj);
    if (e->side) (void)hipStreamDestroy(e->side);
    if (e->stage) (void)hipFree(e->stage);
    if (e->d_mlp) (void)hipFree(e->d_mlp);
    if (e->d_samples) (void)hipFree(e->d_samples);
    if (e->d_nsamples) (void)hipFree(e->d_nsamples);
    if (e->pool) (void)hipFree(e->pool);
    if (e->dd) (void)hipFree(e->dd);
    if (e->ds) (void)hipFree(e->ds);
    if (e->d_sched) (void)hipFree(e->d_sched);
    if (e->ckpt) (void)hipFree(e->ckpt);
    if (e->ckpt_s) (void)hipFree(e->ckpt_s);
    if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

int engine_create(const mrlbm_params* ps, int n, const double* const* m0, void* stream, Engine** out) {
    *out = nullptr;
    g_create_error.clear();
    if (n <= 0 || !ps || !m0) {
        g_create_error = "need n > 0, params and initial data";
        return MRLBM_EINVAL;
    }
    for (int i = 0; i < n; ++i) {
        std::string why;
        const int rc = validate(&ps[i], &why);
        if (rc != MRLBM_OK) {
            g_create_error = "instance " + std::to_string(i) + ": " + why;
            return rc;
        }
        if (ps[i].scheme != ps[0].scheme || ps[i].precision != ps[0].precision || ps[i].gamma != ps[0].gamma) {
            g_create_error = "all runs of a batch must share scheme, precision and gamma";
            return MRLBM_EINVAL;
        }
        if (!m0[i]) {
            g_create_error = "initial data pointer is NULL";
            return MRLBM_EINVAL;
        }
        SchemeInfo si;
        scheme_info(ps[i].scheme, ps[i].physics, &si);
        const size_t cnt = (size_t)si.qc << ps[i].j_max;
        for (size_t k = 0; k < cnt; ++k)
            if (!isfinite(m0[i][k])) {
                g_create_error = "initial data must be finite";
                return MRLBM_EINVAL;
            }
    }
    Engine* e = new (std::nothrow) Engine();
    if (!e) return MRLBM_ENOMEM;
    e->n = n;
    e->prec = ps[0].precision;
    e->scheme = ps[0].scheme;
    e->gamma = ps[0].gamma;
    e->P.assign(ps, ps + n);
    for (int i = 0; i < n; ++i) e->big = e->big || ps[i].j_max > MRLBM_ONCHIP_MAX_J;
    StepK sk;
    QueryK qk;
    InitK ik;
    kernels_for(e->prec, e->scheme, e->gamma, e->big, &sk, &qk, &ik);
    int dev_count = 0;
    hipError_t st = hipGetDeviceCount(&dev_count);
    if (st != hipSuccess || dev_count == 0) {
        g_create_error = "no HIP device";
        delete e;
        return MRLBM_EDEVICE;
    }
    const size_t tsz = e->prec == MRLBM_FP64 ? 8 : 4;
    // layout of the pool
    size_t off = 0;
    size_t maxNJ = 0, maxq = 0;
    e->hd.resize(n);
    std::vector<size_t> o_va(n), o_vb(n), o_split(n), o_list(n), o_pairs(n), o_tree(n);
    for (int i = 0; i < n; ++i) {
        const mrlbm_params& p = ps[i];
        SchemeInfo si;
        scheme_info(p.scheme, p.physics, &si);
        const size_t NJ = (size_t)1 << p.j_max;
        const size_t vals = (size_t)si.q * (((size_t)1 << (p.j_max + 1)) - ((size_t)1 << p.j_min));
        o_va[i] = off;
        off = align256(off + vals * tsz);
        o_vb[i] = off;
        off = align256(off + vals * tsz);
        o_split[i] = off;
        off = align256(off + (size_t)std::max(1, wbase(p.j_min, p.j_max)) * 8);
        o_list[i] = off;
        off = align256(off + NJ * 4);
        o_pairs[i] = off;
        off = align256(off + 2 * (size_t)si.nm * (NJ + 1) * tsz);
        // runs too large for LDS: the tree arrays of the step, in device memory
        o_tree[i] = off;
        if (e->big)
            off = align256(off + make_layout(p.j_min, p.j_max, 0, 0, si.q, si.nm, (int)tsz, false, 4).total);
        maxNJ = std::max(maxNJ, NJ);
        maxq = std::max(maxq, (size_t)si.q);
        e->maxJ = std::max(e->maxJ, p.j_max);
        Desc& d = e->hd[i];
        memset(&d, 0, sizeof(d));
        d.jmin = p.j_min;
        d.jmax = p.j_max;
        d.gamma = p.gamma;
        d.mu_bar = p.mu_bar;
        d.bc = p.bc;
        d.q = si.q;
        d.qc = si.qc;
        d.nm = si.nm;
        d.recon = (p.flags & MRLBM_FLAG_RECONSTRUCTED_COLLISION) ? 1 : 0;
        e->any_recon = e->any_recon || d.recon;
        d.eps = p.eps;
        pred_coeffs(p.gamma, d.c);
        d.cf = make_coef(&p, si);
    }
    e->pool_bytes = off;
    auto fail = [&](hipError_t s, const char* what) {
        hip_fail(e, s, what);
        g_create_error = e->err;
        const int rc = s == hipErrorOutOfMemory ? MRLBM_ENOMEM : MRLBM_EDEVICE;
        engine_free(e);
        return rc;
    };
    if ((st = hipMalloc(&e->pool, e->pool_bytes)) != hipSuccess) return fail(st, "hipMalloc(pool)");
    if ((st = hipMalloc(&e->dd, sizeof(Desc) * n)) != hipSuccess) return fail(st, "hipMalloc(desc)");
    if ((st = hipMalloc(&e->ds, sizeof(State) * n)) != hipSuccess) return fail(st, "hipMalloc(state)");
    e->stage_elems = maxNJ * maxq;
    if ((st = hipMalloc(&e->stage, e->stage_elems * sizeof(double))) != hipSuccess) return fail(st, "hipMalloc(stage)");
    if (stream) {
        e->stream = (hipStream_t)stream;
    } else {
        if ((st = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking)) != hipSuccess)
            return fail(st, "hipStreamCreate");
        e->own_stream = true;
    }
    if ((st = hipEventCreate(&e->ev0)) != hipSuccess) return fail(st, "hipEventCreate");
    if ((st = hipEventCreate(&e->ev1)) != hipSuccess) return fail(st, "hipEventCreate");
    if ((st = hipMemsetAsync(e->pool, 0, e->pool_bytes, e->stream)) != hipSuccess) return fail(st, "hipMemset");
    for (int i = 0; i < n; ++i) {
        Desc& d = e->hd[i];
        d.va = e->pool + o_va[i];
        d.vb = e->pool + o_vb[i];
        d.split = reinterpret_cast<uint64_t*>(e->pool + o_split[i]);
        d.list = reinterpret_cast<uint32_t*>(e->pool + o_list[i]);
        d.pairs = e->pool + o_pairs[i];
        d.gtree = e->big ? reinterpret_cast<uint8_t*>(e->pool + o_tree[i]) : nullptr;
    }
    if ((st = hipMemcpyAsync(e->dd, e->hd.data(), sizeof(Desc) * n, hipMemcpyHostToDevice, e->stream)) != hipSuccess)
        return fail(st, "hipMemcpy(desc)");
    // initial conserved averages: staged through one device buffer, one run at a time
    double* dm = nullptr;
    size_t mcap = 0;
    for (int i = 0; i < n; ++i) {
        const size_t cnt = (size_t)e->hd[i].qc << ps[i].j_max;
        mcap = std::max(mcap, cnt);
    }
    if ((st = hipMalloc(&dm, mcap * sizeof(double))) != hipSuccess) return fail(st, "hipMalloc(init)");
    for (int i = 0; i < n; ++i) {
        const size_t cnt = (size_t)e->hd[i].qc << ps[i].j_max;
        st = hipMemcpyAsync(dm, m0[i], cnt * sizeof(double), hipMemcpyHostToDevice, e->stream);
        if (st != hipSuccess) {
            (void)hipFree(dm);
            return fail(st, "hipMemcpy(init)");
        }
        const int NJ = 1 << ps[i].j_max;
        dim3 grid((NJ + 255) / 256, 1);
        hipLaunchKernelGGL(ik, grid, dim3(256), 0, e->stream, e->dd + i, e->ds + i, (const double*)dm, 0LL);
        st = hipGetLastError();
        if (st != hipSuccess) {
            (void)hipFree(dm);
            return fail(st, "init launch");
        }
    }
    st = hipStreamSynchronize(e->stream);
    (void)hipFree(dm);
    if (st != hipSuccess) return fail(st, "init");
    int dev = 0, maxlds = 65536;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    // static LDS of the kernels (word bases, counters) is below 1 KB
    e->lds_budget = (size_t)std::max(0, maxlds - 1024);
    e->lds_full = e->lds_budget;
    choose_capacity(e);
    // the dynamic-LDS limit of a kernel is shared by every handle that launches it, so it is
    // set to the device's whole budget, which no launch (single, class or query) exceeds
    (void)hipFuncSetAttribute((const void*)sk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)e->lds_full);
    if (e->any_recon)
        (void)hipFuncSetAttribute((const void*)rc_kernel(e->prec, e->scheme), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)e->lds_full);
    (void)hipFuncSetAttribute((const void*)qk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)e->lds_full);
    e->nt = default_block(e->maxJ);
    *out = e;
    return MRLBM_OK;
}

int check_numeric(Engine* e) { return e->numeric ? MRLBM_ENUMERIC : MRLBM_OK; }

static int launch_once(Engine* e, int nsteps, int mode, bool use_graph);

// The class launches of one step call: forked from the handle's stream to the side stream and
// joined back, so that classes run side by side (also inside a captured graph).
static int launch_classes(Engine* e, StepK sk, int nsteps, int mode) {
    hipError_t st;
    if ((st = hipEventRecord(e->evf, e->stream)) != hipSuccess) return hip_fail(e, st, "hipEventRecord(fork)");
    if ((st = hipStreamWaitEvent(e->side, e->evf, 0)) != hipSuccess) return hip_fail(e, st, "hipStreamWaitEvent(fork)");
    // heaviest class first (on the handle's stream): its runs hold the most LDS, and the
    // lighter classes fill what is left on each compute unit around them
    int k = 0;
    for (auto it = e->cls.rbegin(); it != e->cls.rend(); ++it) {
        const auto& c = *it;
        if (c.count == 0) continue;
        hipStream_t s = (k++ % 2 == 0) ? e->stream : e->side;
        hipLaunchKernelGGL(sk, dim3(c.count), dim3(c.nt), c.lds, s, (const Desc*)e->dd, e->ds,
                           (const int*)(e->d_sched + c.first), nsteps, mode, c.cap, c.capS);
        if ((st = hipGetLastError()) != hipSuccess) return hip_fail(e, st, "class launch");
    }
    if ((st = hipEventRecord(e->evj, e->side)) != hipSuccess) return hip_fail(e, st, "hipEventRecord(join)");
    if ((st = hipStreamWaitEvent(e->stream, e->evj, 0)) != hipSuccess) return hip_fail(e, st, "hipStreamWaitEvent(join)");
    return MRLBM_OK;
}

// Graph of one launch of nsteps full steps in the current launch shape, captured once and
// kept until the step count, the block size or the capacity changes.
static int prepare_graph(Engine* e, int nsteps) {
    StepK sk;
    QueryK qk;
    InitK ik;
    kernels_for(e->prec, e->scheme, e->gamma, e->big, &sk, &qk, &ik);
    if (e->lrn) sk = lrn_kernel(e->scheme);
    else if (e->any_recon) sk = rc_kernel(e->prec, e->scheme);
    const int nt = e->nt_user ? e->nt_user : e->nt;
    const int gc = e->cls.empty() ? -1 : e->cls_gen;
    if (e->gexec && e->gsteps == nsteps && e->gnt == nt && e->gcap == e->cap && e->gcls == gc) return MRLBM_OK;
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->gexec = nullptr;
    e->graph = nullptr;
    hipError_t st;
    if ((st = hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, st, "hipStreamBeginCapture");
    if (e->cls.empty()) {
        hipLaunchKernelGGL(sk, dim3(e->n), dim3(nt), e->lds, e->stream, (const Desc*)e->dd, e->ds,
                           (const int*)e->d_sched, nsteps, MODE_ADAPT | MODE_SCHEME, e->cap, e->capS);
    } else {
        const int rc = launch_classes(e, sk, nsteps, MODE_ADAPT | MODE_SCHEME);
        if (rc != MRLBM_OK) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(e->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
    }
    st = hipStreamEndCapture(e->stream, &e->graph);
    if (st != hipSuccess) return hip_fail(e, st, "hipStreamEndCapture");
    if ((st = hipGraphInstantiate(&e->gexec, e->graph, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(e, st, "hipGraphInstantiate");
    e->gsteps = nsteps;
    e->gnt = nt;
    e->gcap = e->cap;
    e->gcls = gc;
    return MRLBM_OK;
}

// nsteps steps as launches of at most e->launch_max steps each (0: one launch).
int launch_steps(Engine* e, int nsteps, int mode, bool use_graph) {
    if (nsteps <= 0) return MRLBM_OK;
    const int chunk = e->launch_max > 0 ? e->launch_max : nsteps;
    for (int done = 0; done < nsteps;) {
        const int k = std::min(chunk, nsteps - done);
        // the graph is kept for the full chunk size; a shorter tail is launched directly
        const int rc = launch_once(e, k, mode, use_graph && (k == chunk || done == 0));
        if (rc != MRLBM_OK) return rc;
        done += k;
    }
    return MRLBM_OK;
}

static int launch_once(Engine* e, int nsteps, int mode, bool use_graph) {
    StepK sk;
    QueryK qk;
    InitK ik;
    kernels_for(e->prec, e->scheme, e->gamma, e->big, &sk, &qk, &ik);
    if (e->lrn) sk = lrn_kernel(e->scheme);
    else if (e->any_recon) sk = rc_kernel(e->prec, e->scheme);
    const int nt = e->nt_user ? e->nt_user : e->nt;
    hipError_t st;
    if (use_graph && mode == (MODE_ADAPT | MODE_SCHEME)) {
        const int rc = prepare_graph(e, nsteps);
        if (rc != MRLBM_OK) return rc;
        if ((st = hipGraphLaunch(e->gexec, e->stream)) != hipSuccess) return hip_fail(e, st, "hipGraphLaunch");
        return MRLBM_OK;
    }
    if (!e->cls.empty()) return launch_classes(e, sk, nsteps, mode);
    hipLaunchKernelGGL(sk, dim3(e->n), dim3(nt), e->lds, e->stream, (const Desc*)e->dd, e->ds, (const int*)e->d_sched,
                       nsteps, mode, e->cap,
                       e->capS);
    st = hipGetLastError();
    if (st != hipSuccess) return hip_fail(e, st, "step launch");
    return MRLBM_OK;
}

int read_states(Engine* e, std::vector<State>& hs) {
    hs.resize(e->n);
    hipError_t st = hipMemcpyAsync(hs.data(), e->ds, sizeof(State) * e->n, hipMemcpyDeviceToHost, e->stream);
    if (st == hipSuccess) st = hipStreamSynchronize(e->stream);
    if (st != hipSuccess) return hip_fail(e, st, "state readback");
    for (auto& s : hs)
        if (s.flags & 1) e->numeric = true;
    return MRLBM_OK;
}

int run_query(Engine* e, int inst, int where, int what, int64_t* n_out) {
    StepK sk;
    QueryK qk;
    InitK ik;
    kernels_for(e->prec, e->scheme, e->gamma, e->big, &sk, &qk, &ik);
    const int nt = e->nt_user ? e->nt_user : e->nt;
    hipLaunchKernelGGL(qk, dim3(1), dim3(nt), e->lds_query, e->stream, (const Desc*)(e->dd + inst), e->ds + inst,
                       where, what, e->stage);
    hipError_t st = hipGetLastError();
    if (st != hipSuccess) return hip_fail(e, st, "query launch");
    State s;
    st = hipMemcpyAsync(&s, e->ds + inst, sizeof(State), hipMemcpyDeviceToHost, e->stream);
    if (st == hipSuccess) st = hipStreamSynchronize(e->stream);
    if (st != hipSuccess) return hip_fail(e, st, "query");
    if (s.flags & 1) e->numeric = true;
    *n_out = where == MRLBM_FINEST ? ((int64_t)1 << e->P[inst].j_max) : s.n_leaves;
    return MRLBM_OK;
}

int engine_moments(Engine* e, int inst, int where, int what, double* out, int64_t cap, int64_t* n_out) {
    if (inst < 0 || inst >= e->n || !n_out || (where != MRLBM_LEAVES && where != MRLBM_FINEST)) {
        e->err = "bad query arguments";
        return MRLBM_EINVAL;
    }
    if (e->numeric) return MRLBM_ENUMERIC;
    int64_t n = 0;
    int rc = run_query(e, inst, where, what, &n);
    if (rc != MRLBM_OK) return rc;
    const int comps = what == 0 ? e->hd[inst].qc : e->hd[inst].q;
    *n_out = n;
    if (!out || cap < comps * n) {
        e->err = "output capacity too small";
        return MRLBM_ECAPACITY;
    }
    hipError_t st = hipMemcpy(out, e->stage, sizeof(double) * comps * n, hipMemcpyDeviceToHost);
    if (st != hipSuccess) return hip_fail(e, st, "moments readback");
    return check_numeric(e);
}

int engine_leaves(Engine* e, int inst, int32_t* level, int64_t* index, int64_t cap, int64_t* n_leaves) {
    if (inst < 0 || inst >= e->n || !n_leaves) {
        e->err = "bad query arguments";
        return MRLBM_EINVAL;
    }
    if (e->numeric) return MRLBM_ENUMERIC;
    int64_t n = 0;
    int rc = run_query(e, inst, MRLBM_LEAVES, 0, &n);
    if (rc != MRLBM_OK) return rc;
    *n_leaves = n;
    if (!level || !index || cap < n) {
        e->err = "output capacity too small";
        return MRLBM_ECAPACITY;
    }
    std::vector<uint32_t> keys(n);
    hipError_t st = hipMemcpy(keys.data(), e->hd[inst].list, sizeof(uint32_t) * n, hipMemcpyDeviceToHost);
    if (st != hipSuccess) return hip_fail(e, st, "leaves readback");
    for (int64_t i = 0; i < n; ++i) {
        level[i] = (int32_t)(keys[i] >> 27);
        index[i] = (int64_t)(keys[i] & ((1u << 27) - 1u));
    }
    return MRLBM_OK;
}

int engine_stats(Engine* e, int inst, mrlbm_stats_t* st) {
    if (!st || inst < 0 || inst >= e->n) {
        e->err = "bad stats arguments";
        return MRLBM_EINVAL;
    }
    std::vector<State> hs;
    int rc = read_states(e, hs);
    if (rc != MRLBM_OK) return rc;
    const State& s = hs[inst];
    st->steps = s.steps;
    st->leaves = s.n_leaves;
    st->leaf_updates = s.leaf_updates;
    st->numeric_error = (s.flags & 1) ? 1 : 0;
    st->q = e->hd[inst].q;
    st->q_cons = e->hd[inst].qc;
    st->j_max = e->hd[inst].jmax;
    st->tree_cells = s.n_r;
    st->misses = s.misses;
    st->redos = s.redos;
    return MRLBM_OK;
}

int engine_step_timed(Engine* e, int nsteps, bool graph, double* ms) {
    if (e->numeric) return MRLBM_ENUMERIC;
    if (nsteps < 0 || !ms) {
        e->err = "bad timed-step arguments";
        return MRLBM_EINVAL;
    }
    // the graph of the first launch is made before the timed region starts
    if (graph && nsteps > 0) {
        const int rc0 = prepare_graph(e, e->launch_max > 0 ? std::min(e->launch_max, nsteps) : nsteps);
        if (rc0 != MRLBM_OK) return rc0;
    }
    hipError_t st = hipEventRecord(e->ev0, e->stream);
    if (st != hipSuccess) return hip_fail(e, st, "hipEventRecord");
    int rc = launch_steps(e, nsteps, MODE_ADAPT | MODE_SCHEME, graph);
    if (rc != MRLBM_OK) return rc;
    if ((st = hipEventRecord(e->ev1, e->stream)) != hipSuccess) return hip_fail(e, st, "hipEventRecord");
    if ((st = hipEventSynchronize(e->ev1)) != hipSuccess) return hip_fail(e, st, "hipEventSynchronize");
    float f = 0.f;
    if ((st = hipEventElapsedTime(&f, e->ev0, e->ev1)) != hipSuccess) return hip_fail(e, st, "hipEventElapsedTime");
    *ms = (double)f;
    std::vector<State> hs;
    rc = read_states(e, hs);
    if (rc != MRLBM_OK) return rc;
    return check_numeric(e);
}

// ---------------------------------------------------------------- allocation-free run
// The state of the run of mrlbm_run_noalloc: one file-scope device array per GPU. In host code
// its name is a host-side stand-in; the device address comes from hipGetSymbolAddress, looked
// up once per device and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[MRLBM_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
unsigned char* scratch_ptr[kMaxDevices];

// Device address of this device's scratch array (the device must be current), or null.
unsigned char* scratch_for(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
    }
    return scratch_ptr[dev];
}

// Zero fill of n 16-byte words (a kernel rather than a memset node, so that the call can be
// captured in a graph).
__global__ void k_zero16(uint4* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// The run's descriptor, passed by value, written into the scratch array.
__global__ void k_put_desc(Desc d, Desc* dst) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = d;
}

// On-chip capacity of a single run (the arithmetic of choose_capacity for one run).
void single_capacity(const Desc& d, int tsz, size_t budget, int* cap, int* capS, size_t* lds, size_t* lds_query) {
    const int cg = (1 << (d.jmax + 1)) - (1 << d.jmin);
    auto total = [&](int c) {
        const int cs = c > 0 ? c / 2 + (1 << d.jmin) : 0;
        return (size_t)make_layout(d.jmin, d.jmax, c, cs, d.q, d.nm, tsz, false).total;
    };
    int lo = 0, hi = cg;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (total(mid) <= budget) lo = mid;
        else hi = mid - 1;
    }
    *cap = lo;
    *capS = lo > 0 ? lo / 2 + (1 << d.jmin) : 0;
    *lds = total(lo);
    *lds_query = (size_t)make_layout(d.jmin, d.jmax, 0, 0, d.q, d.nm, tsz).total;
}

int run_noalloc(const mrlbm_params* p, const double* d_m0, int32_t nsteps, double* d_out, void* stream_) {
    if (!p || !d_m0 || !d_out || nsteps < 0) return MRLBM_EINVAL;
    const int vr = validate(p, nullptr);
    if (vr != MRLBM_OK) return vr;
    SchemeInfo si;
    scheme_info(p->scheme, p->physics, &si);
    StepK sk;
    QueryK qk;
    InitK ik;
    if (!kernels_for(p->precision, p->scheme, p->gamma, false, &sk, &qk, &ik)) return MRLBM_EINVAL;
    const bool recon = (p->flags & MRLBM_FLAG_RECONSTRUCTED_COLLISION) != 0;
    if (recon) sk = rc_kernel(p->precision, p->scheme);
    const size_t tsz = p->precision == MRLBM_FP64 ? 8 : 4;
    // layout of the scratch array: descriptor, state, then the pool of one run as in create
    const size_t NJ = (size_t)1 << p->j_max;
    const size_t vals = (size_t)si.q * (((size_t)1 << (p->j_max + 1)) - ((size_t)1 << p->j_min));
    size_t off = 0;
    const size_t o_desc = off;
    off = align256(off + sizeof(Desc));
    const size_t o_state = off;
    off = align256(off + sizeof(State));
    const size_t o_va = off;
    off = align256(off + vals * tsz);
    const size_t o_vb = off;
    off = align256(off + vals * tsz);
    const size_t o_split = off;
    off = align256(off + (size_t)std::max(1, wbase(p->j_min, p->j_max)) * 8);
    const size_t o_list = off;
    off = align256(off + NJ * 4);
    const size_t o_pairs = off;
    off = align256(off + 2 * (size_t)si.nm * (NJ + 1) * tsz);
    if (off > (size_t)MRLBM_NOALLOC_SCRATCH_BYTES) return MRLBM_ECAPACITY;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MRLBM_EDEVICE;
    unsigned char* base = scratch_for(dev);
    if (!base) return MRLBM_EDEVICE;
    Desc d;
    memset(&d, 0, sizeof(d));
    d.jmin = p->j_min;
    d.jmax = p->j_max;
    d.gamma = p->gamma;
    d.mu_bar = p->mu_bar;
    d.bc = p->bc;
    d.q = si.q;
    d.qc = si.qc;
    d.nm = si.nm;
    d.recon = recon ? 1 : 0;
    d.eps = p->eps;
    pred_coeffs(p->gamma, d.c);
    d.cf = make_coef(p, si);
    d.va = base + o_va;
    d.vb = base + o_vb;
    d.split = reinterpret_cast<uint64_t*>(base + o_split);
    d.list = reinterpret_cast<uint32_t*>(base + o_list);
    d.pairs = base + o_pairs;
    Desc* dd = reinterpret_cast<Desc*>(base + o_desc);
    State* ds = reinterpret_cast<State*>(base + o_state);
    int maxlds = 65536;
    (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    int cap = 0, capS = 0;
    size_t lds = 0, lds_query = 0;
    single_capacity(d, (int)tsz, (size_t)std::max(0, maxlds - 1024), &cap, &capS, &lds, &lds_query);
    // the kernels' dynamic-LDS limit is the device's whole budget, as for the handles
    const int lim = std::max(0, maxlds - 1024);
    if (hipFuncSetAttribute((const void*)sk, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess ||
        hipFuncSetAttribute((const void*)qk, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess)
        return MRLBM_EDEVICE;
    hipStream_t stream = (hipStream_t)stream_;
    const int nt = default_block(p->j_max);
    const size_t n16 = off / 16;
    hipLaunchKernelGGL(k_zero16, dim3((unsigned)std::min<size_t>((n16 + 255) / 256, 1024)), dim3(256), 0, stream,
                       reinterpret_cast<uint4*>(base), n16);
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, stream, d, dd);
    hipLaunchKernelGGL(ik, dim3((unsigned)((NJ + 255) / 256)), dim3(256), 0, stream, (const Desc*)dd, ds, d_m0, 0LL);
    if (nsteps > 0)
        hipLaunchKernelGGL(sk, dim3(1), dim3(nt), lds, stream, (const Desc*)dd, ds, (const int*)nullptr, (int)nsteps,
                           (int)(MODE_ADAPT | MODE_SCHEME), cap, capS);
    hipLaunchKernelGGL(qk, dim3(1), dim3(nt), lds_query, stream, (const Desc*)dd, ds, (int)MRLBM_FINEST, 0, d_out);
    return hipGetLastError() == hipSuccess ? MRLBM_OK : MRLBM_EDEVICE;
}

}  // namespace

struct mrlbm_s {
    Engine* e;
};
struct mrlbm_batch_s {
    Engine* e;
};

extern "C" {

int mrlbm_validate(const mrlbm_params* p) { return validate(p, nullptr); }

int mrlbm_create(const mrlbm_params* p, const double* m_cons0, void* hip_stream, mrlbm_t* out) {
    if (!out) return MRLBM_EINVAL;
    *out = nullptr;
    const double* m[1] = {m_cons0};
    Engine* e = nullptr;
    const int rc = engine_create(p, 1, m, hip_stream, &e);
    if (rc != MRLBM_OK) return rc;
    mrlbm_t h = new (std::nothrow) mrlbm_s{e};
    if (!h) {
        engine_free(e);
        return MRLBM_ENOMEM;
    }
    *out = h;
    return MRLBM_OK;
}

int mrlbm_adapt(mrlbm_t h) {
    if (!h) return MRLBM_EINVAL;
    if (h->e->numeric) return MRLBM_ENUMERIC;
    return launch_steps(h->e, 1, MODE_ADAPT, false);
}

int mrlbm_step(mrlbm_t h, int32_t nsteps) {
    if (!h || nsteps < 0) return MRLBM_EINVAL;
    if (h->e->numeric) return MRLBM_ENUMERIC;
    return launch_steps(h->e, nsteps, MODE_ADAPT | MODE_SCHEME, false);
}

int mrlbm_moments(mrlbm_t h, int32_t where, double* out, int64_t cap, int64_t* n_out) {
    if (!h) return MRLBM_EINVAL;
    return engine_moments(h->e, 0, where, 0, out, cap, n_out);
}

int mrlbm_populations(mrlbm_t h, double* out, int64_t cap, int64_t* n_out) {
    if (!h) return MRLBM_EINVAL;
    return engine_moments(h->e, 0, MRLBM_LEAVES, 1, out, cap, n_out);
}

int mrlbm_leaves(mrlbm_t h, int32_t* level, int64_t* index, int64_t cap, int64_t* n_leaves) {
    if (!h) return MRLBM_EINVAL;
    return engine_leaves(h->e, 0, level, index, cap, n_leaves);
}

int mrlbm_stats(mrlbm_t h, mrlbm_stats_t* st) {
    if (!h) return MRLBM_EINVAL;
    return engine_stats(h->e, 0, st);
}

int mrlbm_step_timed(mrlbm_t h, int32_t nsteps, double* elapsed_ms) {
    if (!h) return MRLBM_EINVAL;
    return engine_step_timed(h->e, nsteps, false, elapsed_ms);
}

void mrlbm_destroy(mrlbm_t h) {
    if (!h) return;
    if (h->e && h->e->stream) (void)hipStreamSynchronize(h->e->stream);
    engine_free(h->e);
    delete h;
}

const char* mrlbm_last_error(mrlbm_t h) {
    if (!h) return g_create_error.c_str();
    return h->e->err.c_str();
}

int mrlbm_batch_create(const mrlbm_params* p, int32_t n, const double* const* m_cons0, void* hip_stream,
                       mrlbm_batch_t* out) {
    if (!out) return MRLBM_EINVAL;
    *out = nullptr;
    Engine* e = nullptr;
    const int rc = engine_create(p, n, m_cons0, hip_stream, &e);
    if (rc != MRLBM_OK) return rc;
    mrlbm_batch_t b = new (std::nothrow) mrlbm_batch_s{e};
    if (!b) {
        engine_free(e);
        return MRLBM_ENOMEM;
    }
    *out = b;
    return MRLBM_OK;
}

int mrlbm_batch_step(mrlbm_batch_t b, int32_t nsteps) {
    if (!b || nsteps < 0) return MRLBM_EINVAL;
    if (b->e->numeric) return MRLBM_ENUMERIC;
    return launch_steps(b->e, nsteps, MODE_ADAPT | MODE_SCHEME, true);
}

int mrlbm_batch_step_timed(mrlbm_batch_t b, int32_t nsteps, double* elapsed_ms) {
    if (!b) return MRLBM_EINVAL;
    return engine_step_timed(b->e, nsteps, true, elapsed_ms);
}

int mrlbm_batch_moments(mrlbm_batch_t b, int32_t inst, int32_t where, double* out, int64_t cap, int64_t* n_out) {
    if (!b) return MRLBM_EINVAL;
    return engine_moments(b->e, inst, where, 0, out, cap, n_out);
}

int mrlbm_batch_leaves(mrlbm_batch_t b, int32_t inst, int32_t* level, int64_t* index, int64_t cap,
                       int64_t* n_leaves) {
    if (!b) return MRLBM_EINVAL;
    return engine_leaves(b->e, inst, level, index, cap, n_leaves);
}

int mrlbm_batch_stats(mrlbm_batch_t b, int32_t inst, mrlbm_stats_t* st) {
    if (!b) return MRLBM_EINVAL;
    return engine_stats(b->e, inst, st);
}

int mrlbm_batch_total_updates(mrlbm_batch_t b, int64_t* total) {
    if (!b || !total) return MRLBM_EINVAL;
    std::vector<State> hs;
    const int rc = read_states(b->e, hs);
    if (rc != MRLBM_OK) return rc;
    int64_t t = 0;
    for (auto& s : hs) t += s.leaf_updates;
    *total = t;
    return check_numeric(b->e);
}

int mrlbm_batch_set_block(mrlbm_batch_t b, int32_t threads) {
    if (!b) return MRLBM_EINVAL;
    if (!b->e->cls.empty()) {
        b->e->err = "launch classes are set (each has its own block size): clear them first";
        return MRLBM_ESTATE;
    }
    if (threads != 0 && (threads < 64 || threads > 512 || threads % 64 != 0)) {
        b->e->err = "threads must be 0 or a multiple of 64 in 64..512";
        return MRLBM_EINVAL;
    }
    b->e->nt_user = threads;
    return MRLBM_OK;
}

int mrlbm_batch_set_capacity(mrlbm_batch_t b, int32_t cells) {
    if (!b || cells < -1) return MRLBM_EINVAL;
    if (!b->e->cls.empty()) {
        b->e->err = "launch classes are set (each has its own capacity): clear them first";
        return MRLBM_ESTATE;
    }
    b->e->cap_user = cells;
    choose_capacity(b->e);
    return MRLBM_OK;
}

int mrlbm_batch_get_capacity(mrlbm_batch_t b, int32_t* cells) {
    if (!b || !cells) return MRLBM_EINVAL;
    *cells = b->e->cap;
    return MRLBM_OK;
}

// Workgroup -> run schedule. Runs are sorted by cost (leaf count, heaviest first); the
// positions b with (b / stride) even take the heavy runs in that order and their partners
// b + stride the light runs from the lightest up, so that two workgroups that share a CU
// pair a heavy run with a light one. The kernel's wall time is that of its slowest run.
// stride 0 = identity.
static void make_schedule(int stride, const std::vector<long long>& cost, std::vector<int>& perm) {
    const int n = (int)cost.size();
    perm.resize(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    if (stride <= 0) return;
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    if (stride >= n) {  // heaviest first: later workgroups fill the slots the light runs free
        perm = order;
        return;
    }
    int hi = 0, lo = n - 1;
    for (int b = 0; b < n; ++b) {
        if ((b / stride) % 2) continue;
        perm[b] = order[hi++];
        if (b + stride < n) perm[b + stride] = order[lo--];
    }
}

static int set_schedule(Engine* e, int stride) {
    std::vector<State> hs;
    int rc = read_states(e, hs);
    if (rc != MRLBM_OK) return rc;
    // a-priori cost ranking: finer runs first, then smaller thresholds (more cells kept),
    // then larger current trees; the rank is the cost
    std::vector<int> idx(e->n);
    for (int i = 0; i < e->n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (e->P[a].j_max != e->P[b].j_max) return e->P[a].j_max > e->P[b].j_max;
        if (e->P[a].eps != e->P[b].eps) return e->P[a].eps < e->P[b].eps;
        return hs[a].n_leaves > hs[b].n_leaves;
    });
    std::vector<long long> cost(e->n);
    for (int r = 0; r < e->n; ++r) cost[idx[r]] = e->n - r;
    std::vector<int> perm;
    if (e->cls.empty()) {
        make_schedule(stride, cost, perm);
    } else {
        // each class's segment: its runs, scheduled with the stride among themselves
        std::vector<int> members, sub;
        std::vector<long long> subcost;
        int jlo = -1;
        for (auto& c : e->cls) {
            members.clear();
            subcost.clear();
            for (int i = 0; i < e->n; ++i)
                if (e->P[i].j_max > jlo && e->P[i].j_max <= c.jhi) {
                    members.push_back(i);
                    subcost.push_back(cost[i]);
                }
            c.first = (int)perm.size();
            c.count = (int)members.size();
            make_schedule(stride, subcost, sub);
            for (int v : sub) perm.push_back(members[v]);
            jlo = c.jhi;
        }
        if ((int)perm.size() != e->n) {
            e->err = "launch classes do not cover every run";
            return MRLBM_EINVAL;
        }
    }
    std::vector<char> seen(e->n, 0);  // the kernel indexes runs through it: must be a permutation
    for (int v : perm) {
        if (v < 0 || v >= e->n || seen[v]) {
            e->err = "internal: schedule is not a permutation";
            return MRLBM_EDEVICE;
        }
        seen[v] = 1;
    }
    hipError_t st;
    if (!e->d_sched) {
        if ((st = hipMalloc(&e->d_sched, sizeof(int) * e->n)) != hipSuccess) return hip_fail(e, st, "hipMalloc(schedule)");
        e->gsteps = -1;  // a captured launch still has the null schedule
    }
    if ((st = hipMemcpyAsync(e->d_sched, perm.data(), sizeof(int) * e->n, hipMemcpyHostToDevice, e->stream)) !=
            hipSuccess ||
        (st = hipStreamSynchronize(e->stream)) != hipSuccess)
        return hip_fail(e, st, "schedule upload");
    e->sched_stride = stride;
    return MRLBM_OK;
}

static int set_classes(Engine* e, int n, const int32_t* jup, const int32_t* threads, const int32_t* per_cu);

int mrlbm_batch_tune(mrlbm_batch_t b, int32_t trial_steps, int32_t* threads, int32_t* cells) {
    if (!b || trial_steps <= 0) return MRLBM_EINVAL;
    Engine* e = b->e;
    if (e->numeric) return MRLBM_ENUMERIC;
    if (e->big) {
        e->err = "tune: runs beyond MRLBM_ONCHIP_MAX_J keep nothing on chip; set the block size instead";
        return MRLBM_ESTATE;
    }
    if (!e->cls.empty()) {  // the tuner chooses the shape of a single launch
        e->cls.clear();
        ++e->cls_gen;
        e->gsteps = -1;
    }
    // snapshot of every run (values, trees, lists, statistics), restored after each trial
    char* snap = nullptr;
    State* ssnap = nullptr;
    hipError_t st = hipMalloc(&snap, e->pool_bytes);
    if (st != hipSuccess) return hip_fail(e, st, "hipMalloc(tune snapshot)");
    st = hipMalloc(&ssnap, sizeof(State) * e->n);
    if (st != hipSuccess) {
        (void)hipFree(snap);
        return hip_fail(e, st, "hipMalloc(tune snapshot)");
    }
    auto copy_all = [&](bool save) {
        hipError_t s1 = save ? hipMemcpyAsync(snap, e->pool, e->pool_bytes, hipMemcpyDeviceToDevice, e->stream)
                             : hipMemcpyAsync(e->pool, snap, e->pool_bytes, hipMemcpyDeviceToDevice, e->stream);
        hipError_t s2 = save ? hipMemcpyAsync(ssnap, e->ds, sizeof(State) * e->n, hipMemcpyDeviceToDevice, e->stream)
                             : hipMemcpyAsync(e->ds, ssnap, sizeof(State) * e->n, hipMemcpyDeviceToDevice, e->stream);
        return s1 != hipSuccess ? s1 : s2;
    };
    // leaf-cell updates per ms of trial_steps steps from the snapshot, which is restored after
    auto trial = [&](double* rate) -> int {
        std::vector<State> h0, h1;
        int r = read_states(e, h0);
        if (r != MRLBM_OK) return r;
        if ((st = hipEventRecord(e->ev0, e->stream)) != hipSuccess) return hip_fail(e, st, "tune");
        if ((r = launch_steps(e, trial_steps, MODE_ADAPT | MODE_SCHEME, false)) != MRLBM_OK) return r;
        if ((st = hipEventRecord(e->ev1, e->stream)) != hipSuccess) return hip_fail(e, st, "tune");
        if ((st = hipEventSynchronize(e->ev1)) != hipSuccess) return hip_fail(e, st, "tune");
        float f = 0.f;
        (void)hipEventElapsedTime(&f, e->ev0, e->ev1);
        if ((r = read_states(e, h1)) != MRLBM_OK) return r;
        long long upd = 0;
        for (int i = 0; i < e->n; ++i) upd += h1[i].leaf_updates - h0[i].leaf_updates;
        *rate = f > 0.f ? upd / (double)f : 0.0;
        if ((st = copy_all(false)) != hipSuccess) return hip_fail(e, st, "tune restore");
        return MRLBM_OK;
    };
    const int saved_nt = e->nt_user;
    const size_t full_budget = e->lds_full;  // a tuned handle's budget may be smaller
    const int saved_stride = e->sched_stride;
    int best_nt = 0;
    size_t best_budget = full_budget;
    double best_rate = -1.0;
    int rc = MRLBM_OK;
    if ((st = copy_all(true)) != hipSuccess) rc = hip_fail(e, st, "tune snapshot");
    // launch shape: threads per workgroup x runs per CU (which sets the on-chip capacity)
    const int nts[4] = {128, 256, 384, 512};
    const int pcs[5] = {1, 2, 3, 4, 8};
    for (int ti = 0; ti < 4 && rc == MRLBM_OK; ++ti) {
        for (int pi = 0; pi < 5 && rc == MRLBM_OK; ++pi) {
            const int per_cu = pcs[pi];
            if (per_cu * nts[ti] > 2048) continue;  // beyond 32 waves per CU
            e->nt_user = nts[ti];
            e->lds_budget = (full_budget + 1024) / per_cu - 1024;
            choose_capacity(e);
            if (e->lds > e->lds_budget) continue;  // the tree words alone do not fit
            double rate = 0.0;
            if ((rc = trial(&rate)) != MRLBM_OK) break;
            if (rate > best_rate) {
                best_rate = rate;
                best_nt = nts[ti];
                best_budget = e->lds_budget;
            }
        }
    }
    // schedule: identity, or heavy/light pairs at the stride of one CU slot per CU (the
    // dispatcher fills every CU once before doubling up) or of one XCD round (8 XCDs)
    int best_stride = saved_stride;
    if (rc == MRLBM_OK && best_rate >= 0) {
        e->nt_user = best_nt;
        e->lds_budget = best_budget;
        choose_capacity(e);
        int dev = 0, ncu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        const int strides[4] = {0, ncu, 8, e->n};
        double best_s = -1.0;
        for (int si = 0; si < 4 && rc == MRLBM_OK; ++si) {
            if (si > 0 && si < 3 && (strides[si] <= 0 || strides[si] >= e->n)) continue;
            if ((rc = set_schedule(e, strides[si])) != MRLBM_OK) break;
            double rate = 0.0;
            if ((rc = trial(&rate)) != MRLBM_OK) break;
            if (rate > best_s) {
                best_s = rate;
                best_stride = strides[si];
            }
        }
    }
    // launch classes for a batch of uneven j_max: the runs up to j_max - 2 (or - 1) in small
    // workgroups sized for many per CU, the others in larger ones, against the best single
    // launch on the same steps
    int best_cls = -1;
    if (rc == MRLBM_OK && best_rate >= 0 && !e->lrn) {
        int jlo = 30, jhi = 0;
        for (auto& p : e->P) {
            jlo = std::min(jlo, p.j_max);
            jhi = std::max(jhi, p.j_max);
        }
        if (jhi - jlo >= 2) {
            e->nt_user = best_nt;
            e->lds_budget = best_budget;
            choose_capacity(e);
            double best_single = -1.0;
            if ((rc = set_schedule(e, best_stride)) == MRLBM_OK) rc = trial(&best_single);
            const int32_t cj[3][2] = {{jhi - 2, jhi}, {jhi - 1, jhi}, {jhi - 2, jhi}};
            const int32_t ct[3][2] = {{128, 256}, {128, 256}, {128, 512}};
            const int32_t cp[3][2] = {{8, 4}, {8, 4}, {8, 2}};
            double best_c = best_single;
            for (int c = 0; c < 3 && rc == MRLBM_OK; ++c) {
                if ((rc = set_classes(e, 2, cj[c], ct[c], cp[c])) != MRLBM_OK) break;
                double rate = 0.0;
                if ((rc = trial(&rate)) != MRLBM_OK) break;
                if (rate > best_c) {
                    best_c = rate;
                    best_cls = c;
                }
            }
            if (rc == MRLBM_OK && best_cls >= 0) rc = set_classes(e, 2, cj[best_cls], ct[best_cls], cp[best_cls]);
            else if (rc == MRLBM_OK) rc = set_classes(e, 0, nullptr, nullptr, nullptr);
        }
    }
    if ((st = hipStreamSynchronize(e->stream)) != hipSuccess && rc == MRLBM_OK) rc = hip_fail(e, st, "tune");
    (void)hipFree(snap);
    (void)hipFree(ssnap);
    if (rc != MRLBM_OK && !e->cls.empty()) (void)set_classes(e, 0, nullptr, nullptr, nullptr);
    if (rc == MRLBM_OK && best_cls >= 0) {
        // the classes carry their own shapes; the single-launch settings stay the best ones
        e->nt_user = best_nt;
        e->lds_budget = best_budget;
        choose_capacity(e);
        if (threads) *threads = 0;
        if (cells) *cells = 0;
        return check_numeric(e);
    }
    if (rc != MRLBM_OK || best_rate < 0) {
        e->nt_user = saved_nt;
        e->lds_budget = full_budget;
        choose_capacity(e);
        if (e->d_sched) (void)set_schedule(e, saved_stride);
        return rc;
    }
    e->nt_user = best_nt;
    e->lds_budget = best_budget;
    choose_capacity(e);
    if ((rc = set_schedule(e, best_stride)) != MRLBM_OK) return rc;
    if (threads) *threads = best_nt;
    if (cells) *cells = e->cap;
    return check_numeric(e);
}

int mrlbm_batch_checkpoint(mrlbm_batch_t b) {
    if (!b) return MRLBM_EINVAL;
    Engine* e = b->e;
    hipError_t st;
    if (!e->ckpt) {
        if ((st = hipMalloc(&e->ckpt, e->pool_bytes)) != hipSuccess) {
            e->ckpt = nullptr;
            return hip_fail(e, st, "hipMalloc(checkpoint)");
        }
        if ((st = hipMalloc(&e->ckpt_s, sizeof(State) * e->n)) != hipSuccess) {
            (void)hipFree(e->ckpt);
            e->ckpt = nullptr;
            e->ckpt_s = nullptr;
            return hip_fail(e, st, "hipMalloc(checkpoint)");
        }
    }
    if ((st = hipMemcpyAsync(e->ckpt, e->pool, e->pool_bytes, hipMemcpyDeviceToDevice, e->stream)) != hipSuccess ||
        (st = hipMemcpyAsync(e->ckpt_s, e->ds, sizeof(State) * e->n, hipMemcpyDeviceToDevice, e->stream)) !=
            hipSuccess ||
        (st = hipStreamSynchronize(e->stream)) != hipSuccess)
        return hip_fail(e, st, "checkpoint");
    e->ckpt_numeric = e->numeric;
    return MRLBM_OK;
}

int mrlbm_batch_restore(mrlbm_batch_t b) {
    if (!b) return MRLBM_EINVAL;
    Engine* e = b->e;
    if (!e->ckpt) {
        e->err = "restore: no checkpoint taken";
        return MRLBM_EINVAL;
    }
    hipError_t st;
    if ((st = hipMemcpyAsync(e->pool, e->ckpt, e->pool_bytes, hipMemcpyDeviceToDevice, e->stream)) != hipSuccess ||
        (st = hipMemcpyAsync(e->ds, e->ckpt_s, sizeof(State) * e->n, hipMemcpyDeviceToDevice, e->stream)) !=
            hipSuccess ||
        (st = hipStreamSynchronize(e->stream)) != hipSuccess)
        return hip_fail(e, st, "restore");
    e->numeric = e->ckpt_numeric;
    return MRLBM_OK;
}

int mrlbm_batch_set_launch_steps(mrlbm_batch_t b, int32_t steps) {
    if (!b || steps < 0) return MRLBM_EINVAL;
    b->e->launch_max = steps;
    return MRLBM_OK;
}

int mrlbm_batch_get_schedule(mrlbm_batch_t b, int32_t* stride) {
    if (!b || !stride) return MRLBM_EINVAL;
    *stride = b->e->sched_stride;
    return MRLBM_OK;
}

// Launch classes: see the header. Each class's on-chip capacity is the largest that lets
// runs_per_cu of its workgroups share a compute unit's LDS, for the runs of that class only.
static int set_classes(Engine* e, int n, const int32_t* jup, const int32_t* threads, const int32_t* per_cu) {
    if (n < 0 || n > 4 || (n > 0 && (!jup || !threads || !per_cu))) {
        e->err = "classes: need 0 <= n <= 4 and the three arrays";
        return MRLBM_EINVAL;
    }
    if (e->lrn) {
        e->err = "classes: not with the refinement predictor";
        return MRLBM_EINVAL;
    }
    if (e->big && n > 0) {
        e->err = "classes: runs beyond MRLBM_ONCHIP_MAX_J keep nothing on chip";
        return MRLBM_ESTATE;
    }
    int maxj = 0;
    for (auto& p : e->P) maxj = std::max(maxj, p.j_max);
    for (int c = 0; c < n; ++c) {
        if ((c > 0 && jup[c] <= jup[c - 1]) || threads[c] < 64 || threads[c] > 512 || threads[c] % 64 ||
            per_cu[c] < 1 || per_cu[c] > 16) {
            e->err = "classes: bounds must increase, threads in 64..512 (multiple of 64), runs per CU in 1..16";
            return MRLBM_EINVAL;
        }
    }
    if (n > 0 && jup[n - 1] < maxj) {
        e->err = "classes: the last bound must cover the largest j_max";
        return MRLBM_EINVAL;
    }
    hipError_t st;
    // the side stream and the fork/join events, each created once (a failed call leaves the
    // ones it made, and the next call makes the rest)
    if (n > 0) {
        if (!e->side && (st = hipStreamCreateWithFlags(&e->side, hipStreamNonBlocking)) != hipSuccess) {
            e->side = nullptr;
            return hip_fail(e, st, "hipStreamCreate(side)");
        }
        if (!e->evf && (st = hipEventCreateWithFlags(&e->evf, hipEventDisableTiming)) != hipSuccess) {
            e->evf = nullptr;
            return hip_fail(e, st, "hipEventCreate(classes)");
        }
        if (!e->evj && (st = hipEventCreateWithFlags(&e->evj, hipEventDisableTiming)) != hipSuccess) {
            e->evj = nullptr;
            return hip_fail(e, st, "hipEventCreate(classes)");
        }
    }
    // steps in flight use the old class set
    if ((st = hipStreamSynchronize(e->stream)) != hipSuccess) return hip_fail(e, st, "classes");
    const int tsz = e->prec == MRLBM_FP64 ? 8 : 4;
    e->cls.clear();
    int jlo = -1;

    for (int c = 0; c < n; ++c) {
        Engine::LaunchClass k;
        k.jhi = jup[c];
        k.nt = threads[c];
        k.per_cu = per_cu[c];
        const size_t budget = (e->lds_full + 1024) / (size_t)per_cu[c] - 1024;
        int cg_max = 0, jmin_min = 30;
        bool any = false;
        for (auto& d : e->hd)
            if (d.jmax > jlo && d.jmax <= k.jhi) {
                any = true;
                cg_max = std::max(cg_max, (1 << (d.jmax + 1)) - (1 << d.jmin));
                jmin_min = std::min(jmin_min, d.jmin);
            }
        auto total = [&](int cap) {
            size_t t = 0;
            for (auto& d : e->hd)
                if (d.jmax > jlo && d.jmax <= k.jhi) {
                    const int cs = cap > 0 ? cap / 2 + (1 << d.jmin) : 0;
                    t = std::max(t, (size_t)make_layout(d.jmin, d.jmax, cap, cs, d.q, d.nm, tsz, false).total);
                }
            return t;
        };
        int lo = 0, hi = any ? cg_max : 0;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (total(mid) <= budget) lo = mid;
            else hi = mid - 1;
        }
        k.cap = lo;
        k.capS = lo > 0 ? lo / 2 + (1 << jmin_min) : 0;
        k.lds = any ? total(lo) : 0;
        e->cls.push_back(k);
        jlo = k.jhi;
    }
    // (the step kernel's dynamic-LDS limit, set at create, is the whole budget)
    ++e->cls_gen;
    e->gsteps = -1;
    // the schedule array now holds the class segments (heaviest first within each class)
    return set_schedule(e, e->n);
}

int mrlbm_batch_set_classes(mrlbm_batch_t b, int32_t n, const int32_t* j_upper, const int32_t* threads,
                            const int32_t* runs_per_cu) {
    if (!b) return MRLBM_EINVAL;
    if (b->e->numeric) return MRLBM_ENUMERIC;
    return set_classes(b->e, n, j_upper, threads, runs_per_cu);
}

int mrlbm_batch_get_classes(mrlbm_batch_t b, int32_t cap_n, int32_t* n, int32_t* counts, int32_t* cells) {
    if (!b || !n) return MRLBM_EINVAL;
    const Engine* e = b->e;
    *n = (int32_t)e->cls.size();
    if (cap_n < *n || ((!counts || !cells) && *n > 0)) return *n > 0 ? MRLBM_ECAPACITY : MRLBM_OK;
    for (int c = 0; c < *n; ++c) {
        counts[c] = e->cls[c].count;
        cells[c] = e->cls[c].cap;
    }
    return MRLBM_OK;
}

int mrlbm_batch_set_schedule(mrlbm_batch_t b, int32_t stride) {
    if (!b || stride < 0) return MRLBM_EINVAL;
    if (b->e->numeric) return MRLBM_ENUMERIC;
    return set_schedule(b->e, stride);
}

static int set_predictor(Engine* e, const uint16_t* params, int32_t mode, double gate, int64_t sample_capacity) {
    if (mode < MRLBM_PRED_OFF || mode > MRLBM_PRED_RECORD || (mode == MRLBM_PRED_LEARNED && !params) ||
        !(gate > 0.0) || !std::isfinite(gate) || sample_capacity < 0 || sample_capacity > (1ll << 28)) {
        e->err = "bad predictor arguments";
        return MRLBM_EINVAL;
    }
    if (mode != MRLBM_PRED_OFF && (e->prec != MRLBM_FP64 || e->gamma != 1)) {
        e->err = "the refinement predictor runs with FP64 storage and gamma = 1";
        return MRLBM_EINVAL;
    }
    if (mode != MRLBM_PRED_OFF && e->big) {
        e->err = "the refinement predictor runs with j_max <= MRLBM_ONCHIP_MAX_J";
        return MRLBM_ESTATE;
    }
    if (mode != MRLBM_PRED_OFF && e->any_recon) {
        e->err = "the refinement predictor runs with the leaves collision only";
        return MRLBM_EINVAL;
    }
    if (mode != MRLBM_PRED_OFF && !e->cls.empty()) {
        e->err = "the refinement predictor runs with a single launch (no launch classes)";
        return MRLBM_EINVAL;
    }
    // steps still in flight on the handle's stream read the weights and samples replaced here
    hipError_t st = hipStreamSynchronize(e->stream);
    if (st != hipSuccess) return hip_fail(e, st, "set_predictor");
    if (params) {
        if (!e->d_mlp && (st = hipMalloc(&e->d_mlp, sizeof(uint16_t) * MLP_NPARAM)) != hipSuccess)
            return hip_fail(e, st, "hipMalloc(predictor)");
        if ((st = hipMemcpy(e->d_mlp, params, sizeof(uint16_t) * MLP_NPARAM, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, st, "hipMemcpy(predictor)");
    }
    if (mode == MRLBM_PRED_RECORD && sample_capacity > e->sample_alloc) {
        // the old buffer stays valid (and in use by the descriptors) until the new one exists
        float* nb = nullptr;
        if ((st = hipMalloc(&nb, sizeof(float) * (MLP_IN + 1) * sample_capacity)) != hipSuccess)
            return hip_fail(e, st, "hipMalloc(samples)");
        if (e->d_samples) (void)hipFree(e->d_samples);
        e->d_samples = nb;
        e->sample_alloc = sample_capacity;
    }
    e->sample_cap = mode == MRLBM_PRED_RECORD ? sample_capacity : 0;
    if (mode == MRLBM_PRED_RECORD && !e->d_nsamples) {
        if ((st = hipMalloc(&e->d_nsamples, sizeof(unsigned int))) != hipSuccess) return hip_fail(e, st, "hipMalloc");
    }
    if (e->d_nsamples) (void)hipMemsetAsync(e->d_nsamples, 0, sizeof(unsigned int), e->stream);
    for (auto& d : e->hd) {
        d.mlp = e->d_mlp;
        d.pmode = mode;
        d.gate = gate;
        d.samples = e->d_samples;
        d.nsamples = e->d_nsamples;
        d.sample_cap = (int)e->sample_cap;
    }
    if ((st = hipMemcpyAsync(e->dd, e->hd.data(), sizeof(Desc) * e->n, hipMemcpyHostToDevice, e->stream)) != hipSuccess)
        return hip_fail(e, st, "hipMemcpy(desc)");
    if ((st = hipStreamSynchronize(e->stream)) != hipSuccess) return hip_fail(e, st, "set_predictor");
    e->lrn = mode != MRLBM_PRED_OFF;
    choose_capacity(e);
    if (e->lrn)
        (void)hipFuncSetAttribute((const void*)lrn_kernel(e->scheme), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)e->lds_full);
    e->gsteps = -1;  // the captured graph is stale
    return MRLBM_OK;
}

static int get_samples(Engine* e, float* X, float* y, int64_t cap, int64_t* n) {
    if (!n) return MRLBM_EINVAL;
    unsigned int cnt = 0;
    if (e->d_nsamples) {
        // the steps run on the handle's own stream (non-blocking): read behind them
        hipError_t st = hipMemcpyAsync(&cnt, e->d_nsamples, sizeof(unsigned int), hipMemcpyDeviceToHost, e->stream);
        if (st == hipSuccess) st = hipStreamSynchronize(e->stream);
        if (st != hipSuccess) return hip_fail(e, st, "samples");
    }
    const int64_t have = std::min<int64_t>(cnt, e->sample_cap);
    *n = have;
    if (!X || !y || cap < have) {
        e->err = "output capacity too small";
        return MRLBM_ECAPACITY;
    }
    if (have == 0) return MRLBM_OK;
    std::vector<float> buf((size_t)have * (MLP_IN + 1));
    hipError_t st = hipMemcpyAsync(buf.data(), e->d_samples, sizeof(float) * buf.size(), hipMemcpyDeviceToHost, e->stream);
    if (st == hipSuccess) st = hipStreamSynchronize(e->stream);
    if (st != hipSuccess) return hip_fail(e, st, "samples");
    for (int64_t i = 0; i < have; ++i) {
        for (int k = 0; k < MLP_IN; ++k) X[i * MLP_IN + k] = buf[i * (MLP_IN + 1) + k];
        y[i] = buf[i * (MLP_IN + 1) + MLP_IN];
    }
    return MRLBM_OK;
}

int mrlbm_batch_set_predictor(mrlbm_batch_t b, const uint16_t* bf16_params, int32_t mode, double gate,
                              int64_t sample_capacity) {
    if (!b) return MRLBM_EINVAL;
    return set_predictor(b->e, bf16_params, mode, gate, sample_capacity);
}

int mrlbm_batch_samples(mrlbm_batch_t b, float* X, float* y, int64_t cap, int64_t* n) {
    if (!b) return MRLBM_EINVAL;
    return get_samples(b->e, X, y, cap, n);
}

int mrlbm_set_predictor(mrlbm_t h, const uint16_t* bf16_params, int32_t mode, double gate, int64_t sample_capacity) {
    if (!h) return MRLBM_EINVAL;
    return set_predictor(h->e, bf16_params, mode, gate, sample_capacity);
}

int mrlbm_samples(mrlbm_t h, float* X, float* y, int64_t cap, int64_t* n) {
    if (!h) return MRLBM_EINVAL;
    return get_samples(h->e, X, y, cap, n);
}

int mrlbm_batch_get_block(mrlbm_batch_t b, int32_t* threads) {
    if (!b || !threads) return MRLBM_EINVAL;
    *threads = b->e->nt_user ? b->e->nt_user : b->e->nt;
    return MRLBM_OK;
}

int mrlbm_run_noalloc(const mrlbm_params* p, const double* d_m_cons0, int32_t nsteps, double* d_m_out,
                      void* hip_stream) {
    return run_noalloc(p, d_m_cons0, nsteps, d_m_out, hip_stream);
}

void mrlbm_batch_destroy(mrlbm_batch_t b) {
    if (!b) return;
    if (b->e && b->e->stream) (void)hipStreamSynchronize(b->e->stream);
    engine_free(b->e);
    delete b;
}

const char* mrlbm_batch_last_error(mrlbm_batch_t b) {
    if (!b) return g_create_error.c_str();
    return b->e->err.c_str();
}

}  // extern "C"
