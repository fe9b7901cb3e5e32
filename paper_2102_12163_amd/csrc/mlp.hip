// mlp.hip -- training and evaluation of the refinement predictor's network (C ABI part of
// include/mrlbm.h: mrlbm_mlp_*). Training: weighted binary cross-entropy on the logit,
// minibatches split into chunks of 64 samples (one workgroup each), forward and backward
// products on the matrix cores, gradients summed over chunks with float32 atomics, then
// one Adam update of the float32 master parameters.

#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "mlp.h"
#include "mrlbm.h"

using namespace mrl;

namespace {

typedef short __attribute__((ext_vector_type(4))) bf16x4;
typedef float __attribute__((ext_vector_type(4))) f32x4;

constexpr int CH = 64;  // samples per workgroup

// One 16x16 tile of C = A (MxK) * B (KxN), bfloat16 operands from LDS through the accessors
// A(i, k) and B(k, j), float32 accumulation. Lane l contributes A[l % 16][k0 + 4 (l / 16) + r]
// and B[k0 + 4 (l / 16) + r][l % 16], r = 0..3, and ends holding C[4 (l / 16) + r][l % 16].
template <class FA, class FB>
__device__ f32x4 tile16(FA A, FB B, int K, int lane) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int i = lane & 15, kq = (lane >> 4) * 4;
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a[r] = (short)A(i, k0 + kq + r);
            b[r] = (short)B(k0 + kq + r, i);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

struct TrainArgs {
    const float* X;       // [n][32]
    const float* y;       // [n]
    const int* idx;       // sample order
    int first, count;     // this minibatch: idx[first .. first + count)
    float pos_weight;
    float inv_n;          // 1 / count
    const float* theta;   // float32 master parameters
    float* grad;          // [NPARAM], accumulated
    float* loss;          // accumulated mean loss
};

// Forward and backward of one chunk of 64 samples; 256 threads (4 waves).
__global__ __launch_bounds__(256) void k_mlp_fwd_bwd(TrainArgs a) {
    __shared__ uint16_t Xs[CH][MLP_IN];
    __shared__ uint16_t W1s[MLP_H][MLP_IN];
    __shared__ uint16_t W2s[MLP_H][MLP_H];
    __shared__ float Z1[CH][MLP_H];
    __shared__ uint16_t H1q[CH][MLP_H];
    __shared__ float H2[CH][MLP_H];
    __shared__ uint16_t D2q[CH][MLP_H];
    __shared__ uint16_t D1q[CH][MLP_H];
    __shared__ float dout[CH];
    __shared__ float w3q[MLP_H];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int base = a.first + blockIdx.x * CH;
    const int nvalid = min(CH, a.first + a.count - base);
    const float* th = a.theta;
    for (int t = tid; t < CH * MLP_IN; t += 256) {
        const int s = t / MLP_IN, i = t % MLP_IN;
        float v = 0.f;
        if (s < nvalid) v = a.X[(size_t)a.idx[base + s] * MLP_IN + i];
        Xs[s][i] = f2bf(v);
    }
    for (int t = tid; t < MLP_H * MLP_IN; t += 256) W1s[t / MLP_IN][t % MLP_IN] = f2bf(th[MLP_OFF_W1 + t]);
    for (int t = tid; t < MLP_H * MLP_H; t += 256) W2s[t / MLP_H][t % MLP_H] = f2bf(th[MLP_OFF_W2 + t]);
    if (tid < MLP_H) w3q[tid] = bf2f(f2bf(th[MLP_OFF_W3 + tid]));
    __syncthreads();
    // ---- layer 1: Z1 = X W1^T + b1 (M = samples, N = hidden, K = 32); 16 tiles, 4 per wave
    for (int tt = wave; tt < 16; tt += 4) {
        const int tm = tt >> 2, tn = tt & 3;
        f32x4 c = tile16([&](int i, int k) { return Xs[tm * 16 + i][k]; },
                         [&](int k, int j) { return W1s[tn * 16 + j][k]; }, MLP_IN, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = tm * 16 + (lane >> 4) * 4 + r, j = tn * 16 + (lane & 15);
            const float z = c[r] + th[MLP_OFF_B1 + j];
            Z1[s][j] = z;
            H1q[s][j] = f2bf(z > 0.f ? z : 0.f);
        }
    }
    __syncthreads();
    // ---- layer 2: H2 = relu(H1 W2^T + b2)
    for (int tt = wave; tt < 16; tt += 4) {
        const int tm = tt >> 2, tn = tt & 3;
        f32x4 c = tile16([&](int i, int k) { return H1q[tm * 16 + i][k]; },
                         [&](int k, int j) { return W2s[tn * 16 + j][k]; }, MLP_H, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = tm * 16 + (lane >> 4) * 4 + r, j = tn * 16 + (lane & 15);
            const float z = c[r] + th[MLP_OFF_B2 + j];
            H2[s][j] = z > 0.f ? z : 0.f;
        }
    }
    __syncthreads();
    // ---- output, loss and d loss / d logit
    if (tid < CH) {
        const int s = tid;
        float o = th[MLP_OFF_B3];
        for (int j = 0; j < MLP_H; ++j) o += w3q[j] * H2[s][j];
        float g = 0.f, l = 0.f;
        if (s < nvalid) {
            const float y = a.y[a.idx[base + s]];
            const float sg = 1.f / (1.f + expf(-o));
            const float pw = a.pos_weight;
            // log sigma(o) and log(1 - sigma(o)) in a form that does not overflow
            const float ls = -(fmaxf(-o, 0.f) + log1pf(expf(-fabsf(o))));
            const float l1s = -(fmaxf(o, 0.f) + log1pf(expf(-fabsf(o))));
            l = -(pw * y * ls + (1.f - y) * l1s) * a.inv_n;
            g = (sg * (pw * y + 1.f - y) - pw * y) * a.inv_n;
        }
        dout[s] = g;
        if (l != 0.f) atomicAdd(a.loss, l);
    }
    __syncthreads();
    // ---- w3, b3 gradients; dZ2 = dout w3 * (z2 > 0)
    if (tid < MLP_H) {
        float gw = 0.f;
        for (int s = 0; s < CH; ++s) gw += dout[s] * H2[s][tid];
        atomicAdd(&a.grad[MLP_OFF_W3 + tid], gw);
    }
    if (tid == MLP_H) {
        float gb = 0.f;
        for (int s = 0; s < CH; ++s) gb += dout[s];
        atomicAdd(&a.grad[MLP_OFF_B3], gb);
    }
    for (int t = tid; t < CH * MLP_H; t += 256) {
        const int s = t / MLP_H, j = t % MLP_H;
        D2q[s][j] = f2bf(H2[s][j] > 0.f ? dout[s] * w3q[j] : 0.f);
    }
    __syncthreads();
    // b2 gradient
    if (tid < MLP_H) {
        float gb = 0.f;
        for (int s = 0; s < CH; ++s) gb += (H2[s][tid] > 0.f ? dout[s] * w3q[tid] : 0.f);
        atomicAdd(&a.grad[MLP_OFF_B2 + tid], gb);
    }
    // ---- W2 gradient: gW2[j][i] = sum_s dZ2[s][j] H1[s][i] (M = j, N = i, K = samples)
    for (int tt = wave; tt < 16; tt += 4) {
        const int tm = tt >> 2, tn = tt & 3;
        f32x4 c = tile16([&](int i, int k) { return D2q[k][tm * 16 + i]; },
                         [&](int k, int j) { return H1q[k][tn * 16 + j]; }, CH, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int jj = tm * 16 + (lane >> 4) * 4 + r, ii = tn * 16 + (lane & 15);
            atomicAdd(&a.grad[MLP_OFF_W2 + jj * MLP_H + ii], c[r]);
        }
    }
    // ---- dH1 = dZ2 W2 (M = samples, N = hidden i, K = hidden j); dZ1 = dH1 * (z1 > 0)
    for (int tt = wave; tt < 16; tt += 4) {
        const int tm = tt >> 2, tn = tt & 3;
        f32x4 c = tile16([&](int i, int k) { return D2q[tm * 16 + i][k]; },
                         [&](int k, int j) { return W2s[k][tn * 16 + j]; }, MLP_H, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = tm * 16 + (lane >> 4) * 4 + r, i = tn * 16 + (lane & 15);
            const float dz = Z1[s][i] > 0.f ? c[r] : 0.f;
            D1q[s][i] = f2bf(dz);
            Z1[s][i] = dz;  // keeps the float32 dZ1 for the b1 gradient
        }
    }
    __syncthreads();
    if (tid < MLP_H) {
        float gb = 0.f;
        for (int s = 0; s < CH; ++s) gb += Z1[s][tid];
        atomicAdd(&a.grad[MLP_OFF_B1 + tid], gb);
    }
    // ---- W1 gradient: gW1[j][i] = sum_s dZ1[s][j] X[s][i] (M = 64, N = 32, K = samples)
    for (int tt = wave; tt < 8; tt += 4) {
        const int tm = tt >> 1, tn = tt & 1;
        f32x4 c = tile16([&](int i, int k) { return D1q[k][tm * 16 + i]; },
                         [&](int k, int j) { return Xs[k][tn * 16 + j]; }, CH, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int jj = tm * 16 + (lane >> 4) * 4 + r, ii = tn * 16 + (lane & 15);
            atomicAdd(&a.grad[MLP_OFF_W1 + jj * MLP_IN + ii], c[r]);
        }
    }
}

// Adam on the float32 master parameters; clears the gradient; refreshes the bf16 copy.
__global__ void k_mlp_adam(float* theta, float* grad, float* m, float* v, uint16_t* wbf, float lr, float b1, float b2,
                           float c1, float c2, float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM) return;
    const float g = grad[i];
    grad[i] = 0.f;
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    theta[i] = th;
    wbf[i] = f2bf(th);
}

__global__ void k_mlp_to_bf16(const float* theta, uint16_t* wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_NPARAM) wbf[i] = f2bf(theta[i]);
}

__global__ void k_mlp_zero(float* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// Deployment logits of n feature rows, through the in-step decision path: each wave loads
// 64 rows (one per lane) and evaluates them one after the other with the whole wave.
__global__ __launch_bounds__(256) void k_mlp_logits(const uint16_t* __restrict__ wbf, const float* __restrict__ X, int n,
                                                    float* out) {
    const int lane = threadIdx.x & 63;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    float x[MLP_IN];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) x[i] = s < n ? X[(size_t)s * MLP_IN + i] : 0.f;
    const int cnt = min(64, n - (s - lane));  // rows of this wave (wave-uniform)
    float mine = 0.f;
    for (int c = 0; c < cnt; ++c) {
        const float o = mlp_logit_wave(wbf, x, c, lane);
        if (lane == c) mine = o;
    }
    if (s < n) out[s] = mine;
}

}  // namespace

struct mrlbm_mlp_s {
    float* theta = nullptr;
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* loss = nullptr;
    uint16_t* wbf = nullptr;
    long long t = 0;
    hipStream_t stream = nullptr;
    std::string err;
};

namespace {

int mfail(mrlbm_mlp_t h, hipError_t st, const char* what) {
    if (h) h->err = std::string(what) + ": " + hipGetErrorString(st);
    return st == hipErrorOutOfMemory ? MRLBM_ENOMEM : MRLBM_EDEVICE;
}

thread_local std::string g_mlp_error;

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" {

int mrlbm_mlp_create(const float* theta0, mrlbm_mlp_t* out) {
    if (!out || !theta0) return MRLBM_EINVAL;
    *out = nullptr;
    for (int i = 0; i < MLP_NPARAM; ++i)
        if (!std::isfinite(theta0[i])) {
            g_mlp_error = "parameters must be finite";
            return MRLBM_EINVAL;
        }
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || nd == 0) {
        g_mlp_error = "no HIP device";
        return MRLBM_EDEVICE;
    }
    mrlbm_mlp_t h = new (std::nothrow) mrlbm_mlp_s();
    if (!h) return MRLBM_ENOMEM;
    hipError_t st;
    const size_t pb = sizeof(float) * MLP_NPARAM;
    if ((st = hipMalloc(&h->theta, pb)) != hipSuccess || (st = hipMalloc(&h->grad, pb)) != hipSuccess ||
        (st = hipMalloc(&h->m, pb)) != hipSuccess || (st = hipMalloc(&h->v, pb)) != hipSuccess ||
        (st = hipMalloc(&h->loss, sizeof(float))) != hipSuccess ||
        (st = hipMalloc(&h->wbf, sizeof(uint16_t) * MLP_NPARAM)) != hipSuccess ||
        (st = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking)) != hipSuccess) {
        g_mlp_error = std::string("allocation: ") + hipGetErrorString(st);
        mrlbm_mlp_destroy(h);
        return st == hipErrorOutOfMemory ? MRLBM_ENOMEM : MRLBM_EDEVICE;
    }
    (void)hipMemcpy(h->theta, theta0, pb, hipMemcpyHostToDevice);
    (void)hipMemset(h->grad, 0, pb);
    (void)hipMemset(h->m, 0, pb);
    (void)hipMemset(h->v, 0, pb);
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, h->stream, h->theta, h->wbf);
    if ((st = hipStreamSynchronize(h->stream)) != hipSuccess) {
        g_mlp_error = std::string("init: ") + hipGetErrorString(st);
        mrlbm_mlp_destroy(h);
        return MRLBM_EDEVICE;
    }
    *out = h;
    return MRLBM_OK;
}

// Loss and gradient of the current parameters on n samples (host arrays).
int mrlbm_mlp_loss_grad(mrlbm_mlp_t h, const float* X, const float* y, int64_t n, float pos_weight, float* loss,
                        float* grad) {
    if (!h || !X || !y || n <= 0 || !(pos_weight > 0.f) || !loss || !grad) return MRLBM_EINVAL;
    DevBuf dX, dy, di;
    hipError_t st;
    if ((st = hipMalloc(&dX.p, sizeof(float) * MLP_IN * n)) != hipSuccess) return mfail(h, st, "hipMalloc");
    if ((st = hipMalloc(&dy.p, sizeof(float) * n)) != hipSuccess) return mfail(h, st, "hipMalloc");
    if ((st = hipMalloc(&di.p, sizeof(int) * n)) != hipSuccess) return mfail(h, st, "hipMalloc");
    std::vector<int> idx(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = (int)i;
    (void)hipMemcpyAsync(dX.p, X, sizeof(float) * MLP_IN * n, hipMemcpyHostToDevice, h->stream);
    (void)hipMemcpyAsync(dy.p, y, sizeof(float) * n, hipMemcpyHostToDevice, h->stream);
    (void)hipMemcpyAsync(di.p, idx.data(), sizeof(int) * n, hipMemcpyHostToDevice, h->stream);
    hipLaunchKernelGGL(k_mlp_zero, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, h->stream, h->grad, MLP_NPARAM);
    hipLaunchKernelGGL(k_mlp_zero, dim3(1), dim3(64), 0, h->stream, h->loss, 1);
    TrainArgs a;
    a.X = (const float*)dX.p;
    a.y = (const float*)dy.p;
    a.idx = (const int*)di.p;
    a.first = 0;
    a.count = (int)n;
    a.pos_weight = pos_weight;
    a.inv_n = 1.f / (float)n;
    a.theta = h->theta;
    a.grad = h->grad;
    a.loss = h->loss;
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((unsigned)((n + CH - 1) / CH)), dim3(256), 0, h->stream, a);
    if ((st = hipGetLastError()) != hipSuccess) return mfail(h, st, "launch");
    (void)hipMemcpyAsync(grad, h->grad, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, h->stream);
    (void)hipMemcpyAsync(loss, h->loss, sizeof(float), hipMemcpyDeviceToHost, h->stream);
    hipLaunchKernelGGL(k_mlp_zero, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, h->stream, h->grad, MLP_NPARAM);
    if ((st = hipStreamSynchronize(h->stream)) != hipSuccess) return mfail(h, st, "loss_grad");
    return MRLBM_OK;
}

// Adam training on n samples for the given epochs; minibatches of `batch` samples (a multiple
// of 64), order reshuffled every epoch from `seed`. *last_loss: mean loss of the last epoch.
int mrlbm_mlp_train(mrlbm_mlp_t h, const float* X, const float* y, int64_t n, int32_t epochs, int32_t batch, float lr,
                    float pos_weight, uint64_t seed, float* last_loss) {
    if (!h || !X || !y || n <= 0 || epochs <= 0 || batch <= 0 || batch % CH != 0 || !(lr > 0.f) ||
        !(pos_weight > 0.f))
        return MRLBM_EINVAL;
    DevBuf dX, dy, di;
    hipError_t st;
    if ((st = hipMalloc(&dX.p, sizeof(float) * MLP_IN * n)) != hipSuccess) return mfail(h, st, "hipMalloc");
    if ((st = hipMalloc(&dy.p, sizeof(float) * n)) != hipSuccess) return mfail(h, st, "hipMalloc");
    if ((st = hipMalloc(&di.p, sizeof(int) * n)) != hipSuccess) return mfail(h, st, "hipMalloc");
    (void)hipMemcpyAsync(dX.p, X, sizeof(float) * MLP_IN * n, hipMemcpyHostToDevice, h->stream);
    (void)hipMemcpyAsync(dy.p, y, sizeof(float) * n, hipMemcpyHostToDevice, h->stream);
    std::vector<int> idx(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = (int)i;
    std::mt19937_64 rng(seed);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float epoch_loss = 0.f;
    for (int e = 0; e < epochs; ++e) {
        std::shuffle(idx.begin(), idx.end(), rng);
        (void)hipMemcpyAsync(di.p, idx.data(), sizeof(int) * n, hipMemcpyHostToDevice, h->stream);
        hipLaunchKernelGGL(k_mlp_zero, dim3(1), dim3(64), 0, h->stream, h->loss, 1);
        int nb = 0;
        for (int64_t first = 0; first < n; first += batch) {
            const int count = (int)std::min<int64_t>(batch, n - first);
            TrainArgs a;
            a.X = (const float*)dX.p;
            a.y = (const float*)dy.p;
            a.idx = (const int*)di.p;
            a.first = (int)first;
            a.count = count;
            a.pos_weight = pos_weight;
            a.inv_n = 1.f / (float)count;
            a.theta = h->theta;
            a.grad = h->grad;
            a.loss = h->loss;
            hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((count + CH - 1) / CH), dim3(256), 0, h->stream, a);
            h->t += 1;
            const float c1 = 1.f - powf(b1, (float)h->t), c2 = 1.f - powf(b2, (float)h->t);
            hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, h->stream, h->theta, h->grad,
                               h->m, h->v, h->wbf, lr, b1, b2, c1, c2, eps);
            ++nb;
        }
        float lsum = 0.f;
        (void)hipMemcpyAsync(&lsum, h->loss, sizeof(float), hipMemcpyDeviceToHost, h->stream);
        if ((st = hipStreamSynchronize(h->stream)) != hipSuccess) return mfail(h, st, "train");
        epoch_loss = lsum / (float)nb;
    }
    if ((st = hipGetLastError()) != hipSuccess) return mfail(h, st, "train launch");
    if (last_loss) *last_loss = epoch_loss;
    return std::isfinite(epoch_loss) ? MRLBM_OK : MRLBM_ENUMERIC;
}

int mrlbm_mlp_params(mrlbm_mlp_t h, float* theta, uint16_t* bf16) {
    if (!h) return MRLBM_EINVAL;
    hipError_t st = hipSuccess;
    if (theta) st = hipMemcpy(theta, h->theta, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost);
    if (st == hipSuccess && bf16) st = hipMemcpy(bf16, h->wbf, sizeof(uint16_t) * MLP_NPARAM, hipMemcpyDeviceToHost);
    return st == hipSuccess ? MRLBM_OK : mfail(h, st, "params");
}

int mrlbm_mlp_logits(mrlbm_mlp_t h, const float* X, int64_t n, float* logits) {
    if (!h || !X || n <= 0 || !logits) return MRLBM_EINVAL;
    DevBuf dX, dl;
    hipError_t st;
    if ((st = hipMalloc(&dX.p, sizeof(float) * MLP_IN * n)) != hipSuccess) return mfail(h, st, "hipMalloc");
    if ((st = hipMalloc(&dl.p, sizeof(float) * n)) != hipSuccess) return mfail(h, st, "hipMalloc");
    (void)hipMemcpyAsync(dX.p, X, sizeof(float) * MLP_IN * n, hipMemcpyHostToDevice, h->stream);
    hipLaunchKernelGGL(k_mlp_logits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, (const uint16_t*)h->wbf,
                       (const float*)dX.p, (int)n, (float*)dl.p);
    (void)hipMemcpyAsync(logits, dl.p, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream);
    if ((st = hipStreamSynchronize(h->stream)) != hipSuccess) return mfail(h, st, "logits");
    return MRLBM_OK;
}

void mrlbm_mlp_destroy(mrlbm_mlp_t h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->theta) (void)hipFree(h->theta);
    if (h->grad) (void)hipFree(h->grad);
    if (h->m) (void)hipFree(h->m);
    if (h->v) (void)hipFree(h->v);
    if (h->loss) (void)hipFree(h->loss);
    if (h->wbf) (void)hipFree(h->wbf);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char* mrlbm_mlp_last_error(mrlbm_mlp_t h) { return h ? h->err.c_str() : g_mlp_error.c_str(); }

}  // extern "C"
