// Learned initial iterate: a dense network (a, lambda) -> [xhat; lambda] (FP32), its
// fused inference kernel, and the hand-written training step (forward, mean-squared-error
// gradient by back-propagation, Adam).
//
// Network: inputs (log10 a, lambda) mapped affinely onto [-1, 1] over the parameter box
// a in [1, 1e4], lambda in [5, 20]; dense layers W_k [out][in], b_k [out]; SiLU after every
// layer but the last; outputs standardised per component (the solver receives
// y * std + mean in FP64).  The paper starts its solves from an interpolation of training
// solutions (Section 7.2); this network takes that role and is trained on the method's own
// converged solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

using namespace ddrom;

#define MLPCHECK(x)                                                                         \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) {                                                             \
            set_error(std::string(#x) + ": " + hipGetErrorString(e_));                      \
            return DDROM_EHIP;                                                              \
        }                                                                                   \
    } while (0)

namespace {

constexpr int MLP_MAX_LAYERS = 8;
constexpr int MLP_MAX_HIDDEN = 512;   // hidden widths (held in LDS by the inference kernel)
constexpr int INFER_SPB = 8;          // samples per inference workgroup

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_prime_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s + z * s * (1.0f - s);
}

__device__ __forceinline__ void encode_mu(const double* mu, float& u0, float& u1) {
    u0 = (float)(2.0 * (log10(mu[0]) - 0.0) / 4.0 - 1.0);
    u1 = (float)(2.0 * (mu[1] - 5.0) / 15.0 - 1.0);
}

struct LayerTable {
    int n_layers;
    int maxw;                          // widest layer (input, hidden or output)
    int sizes[MLP_MAX_LAYERS + 1];
    long long w_off[MLP_MAX_LAYERS];   // offsets (floats) of the weights in the parameter buffer
    long long b_off[MLP_MAX_LAYERS];
};

// ---- inference: one workgroup = INFER_SPB samples through every layer, activations in LDS ----
// Weights are read transposed (Wt_k [in][out]) so that the threads of a workgroup, one per
// output unit, read consecutive addresses.
__global__ __launch_bounds__(256) void k_mlp_infer(LayerTable T, const float* __restrict__ wt,
                                                   const float* __restrict__ bias, const double* __restrict__ mean,
                                                   const double* __restrict__ stdv, const double* __restrict__ mu,
                                                   int B, int n_D, double* __restrict__ x0, int x_ld,
                                                   double* __restrict__ l0, int l_ld) {
    __shared__ float act[2][INFER_SPB][MLP_MAX_HIDDEN];
    const int s0 = blockIdx.x * INFER_SPB, tid = threadIdx.x;
    if (tid < INFER_SPB) {
        float u0 = 0.f, u1 = 0.f;
        if (s0 + tid < B) encode_mu(mu + 2 * (size_t)(s0 + tid), u0, u1);
        act[0][tid][0] = u0;
        act[0][tid][1] = u1;
    }
    __syncthreads();
    int cur = 0;
    for (int k = 0; k < T.n_layers; ++k) {
        const int nin = T.sizes[k], nout = T.sizes[k + 1];
        const bool last = k == T.n_layers - 1;
        const float* W = wt + T.w_off[k];
        const float* bk = bias + T.b_off[k];
        for (int o = tid; o < nout; o += blockDim.x) {
            float acc[INFER_SPB];
            const float bo = bk[o];
#pragma unroll
            for (int s = 0; s < INFER_SPB; ++s) acc[s] = bo;
            for (int i = 0; i < nin; ++i) {
                const float w = W[(size_t)i * nout + o];
#pragma unroll
                for (int s = 0; s < INFER_SPB; ++s) acc[s] += w * act[cur][s][i];
            }
            if (!last) {
#pragma unroll
                for (int s = 0; s < INFER_SPB; ++s) act[cur ^ 1][s][o] = silu_f(acc[s]);
            } else {
                const double m = mean[o], sd = stdv[o];
#pragma unroll
                for (int s = 0; s < INFER_SPB; ++s) {
                    const int b = s0 + s;
                    if (b >= B) continue;
                    const double y = (double)acc[s] * sd + m;
                    if (o < n_D) x0[(size_t)b * x_ld + o] = y;
                    else if (l0) l0[(size_t)b * l_ld + (o - n_D)] = y;
                }
            }
        }
        __syncthreads();
        cur ^= 1;
    }
}

// ---- training kernels ----
// C[m][n] = sum_k A(m,k) B(k,n) with A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn];
// epilogue EPI: 0 plain store; 1 + bias[n], store Z and SiLU(Z) (hidden layer); 2 + bias[n],
// store (output layer); 3 times SiLU'(aux[m][n]) (gradient through a hidden activation).
// 64 x 64 tile per 256-thread workgroup, 4 x 4 per thread, K staged through LDS in steps of 16.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, long long sam,
                                              long long sak, const float* __restrict__ Bm, long long sbk,
                                              long long sbn, float* __restrict__ C, long long scm,
                                              const float* __restrict__ bias, float* __restrict__ Z,
                                              const float* __restrict__ aux) {
    __shared__ float As[16][65];
    __shared__ float Bs[16][65];
    const int tid = threadIdx.x, tm = tid / 16, tn = tid % 16;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int e = tid; e < 64 * 16; e += 256) {
            const int mm = e / 16, kk = e % 16;
            const int gm = m0 + mm, gk = k0 + kk;
            As[kk][mm] = (gm < M && gk < K) ? A[(long long)gm * sam + (long long)gk * sak] : 0.f;
            const int nn = e % 64, kb = e / 64;
            const int gn = n0 + nn, gk2 = k0 + kb;
            Bs[kb][nn] = (gn < N && gk2 < K) ? Bm[(long long)gk2 * sbk + (long long)gn * sbn] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tm * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gm = m0 + tm * 4 + i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tn * 4 + j;
            if (gn >= N) continue;
            float v = acc[i][j];
            const long long ci = (long long)gm * scm + gn;
            if (EPI == 1) {
                v += bias[gn];
                Z[ci] = v;
                v = silu_f(v);
            } else if (EPI == 2) {
                v += bias[gn];
            } else if (EPI == 3) {
                v *= silu_prime_f(aux[ci]);
            }
            C[ci] = v;
        }
    }
}

// network inputs of the minibatch rows
__global__ void k_mlp_gather(const double* __restrict__ mu, const int* __restrict__ rows, int B,
                             float* __restrict__ X0) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float u0, u1;
    encode_mu(mu + 2 * (size_t)rows[b], u0, u1);
    X0[2 * (size_t)b] = u0;
    X0[2 * (size_t)b + 1] = u1;
}

// dY = 2 (Y - T) / (B n) and per-block partial sums of (Y - T)^2 (fixed order)
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ Tgt,
                                             const int* __restrict__ rows, int B, int n, float* __restrict__ dY,
                                             double* __restrict__ part) {
    __shared__ double red[256];
    const long long tot = (long long)B * n;
    double s = 0.0;
    const float sc = 2.0f / (float)tot;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
        const int b = (int)(e / n), o = (int)(e % n);
        const float r = Y[e] - Tgt[(size_t)rows[b] * n + o];
        dY[e] = sc * r;
        s += (double)r * r;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mse_final(const double* __restrict__ part, int nb, long long tot, float* __restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += part[i];
    loss[0] = (float)(s / (double)tot);
}

// db[o] = sum_b dZ[b][o] (fixed order over b)
__global__ void k_colsum(const float* __restrict__ dZ, int B, int n, float* __restrict__ db) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dZ[(size_t)b * n + o];
    db[o] = s;
}

__global__ void k_adam_tick(int* t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t[0] += 1;
}

__global__ void k_adam(long long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, const int* __restrict__ t, float lr, float b1, float b2, float eps) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int step = t[0];
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_transpose_f(const float* __restrict__ W, int rows, int cols, float* __restrict__ Wt) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    Wt[(size_t)c * rows + r] = W[e];
}

int make_table(int n_layers, const int* sizes, LayerTable& T, long long& n_params) {
    if (n_layers < 1 || n_layers > MLP_MAX_LAYERS || !sizes || sizes[0] != 2) {
        set_error("network must have 1..8 layers and 2 inputs");
        return DDROM_EINVAL;
    }
    T.n_layers = n_layers;
    T.maxw = 0;
    long long off = 0;
    for (int k = 0; k <= n_layers; ++k) {
        const bool hidden = k > 0 && k < n_layers;
        if (sizes[k] < 1 || (hidden && sizes[k] > MLP_MAX_HIDDEN) || sizes[k] > (1 << 16)) {
            set_error("hidden widths must be in 1..512");
            return DDROM_EINVAL;
        }
        T.sizes[k] = sizes[k];
        T.maxw = std::max(T.maxw, sizes[k]);
    }
    for (int k = 0; k < n_layers; ++k) {
        T.w_off[k] = off;
        off += (long long)sizes[k + 1] * sizes[k];
        T.b_off[k] = off;
        off += sizes[k + 1];
    }
    n_params = off;
    return 0;
}

}  // namespace

struct ddrom_mlp {
    LayerTable T{};
    long long n_params = 0;
    int n_out = 0, n_D = 0;
    float* wt = nullptr;       // weights transposed per layer (same offsets as the parameter buffer)
    float* params = nullptr;   // parameters in [out][in] layout (biases read from here)
    double* mean = nullptr;
    double* stdv = nullptr;
};

struct ddrom_mlp_trainer {
    LayerTable T{};
    long long n_params = 0;
    int max_B = 0, n_out = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float* act = nullptr;      // [n_layers + 1][max_B][maxw] layer inputs / outputs ([B][width] each)
    float* zbuf = nullptr;     // [n_layers][max_B][maxw] pre-activations
    float* d0 = nullptr;       // [max_B][maxw] gradient buffers
    float* d1 = nullptr;
    double* part = nullptr;    // loss partial sums
    int* t = nullptr;          // Adam step counter (device)
};

static constexpr int MSE_BLOCKS = 64;

extern "C" {

int ddrom_mlp_create(const ddrom_mlp_desc* d, ddrom_mlp** out) {
    if (!d || !out || !d->params || !d->out_mean || !d->out_std) {
        set_error("bad arguments to ddrom_mlp_create");
        return DDROM_EINVAL;
    }
    *out = nullptr;
    std::unique_ptr<ddrom_mlp> m(new ddrom_mlp());
    int rc = make_table(d->n_layers, d->sizes, m->T, m->n_params);
    if (rc) return rc;
    m->n_out = d->sizes[d->n_layers];
    m->n_D = d->n_D;
    if (m->n_D < 0 || m->n_D > m->n_out) {
        set_error("n_D exceeds the network output width");
        return DDROM_EINVAL;
    }
    const size_t pb = (size_t)m->n_params * sizeof(float), ob = (size_t)m->n_out * sizeof(double);
    if (hipMalloc((void**)&m->wt, pb) != hipSuccess || hipMalloc((void**)&m->params, pb) != hipSuccess ||
        hipMalloc((void**)&m->mean, ob) != hipSuccess || hipMalloc((void**)&m->stdv, ob) != hipSuccess) {
        set_error("device allocation failed");
        ddrom_mlp_destroy(m.release());
        return DDROM_ENOMEM;
    }
    if (hipMemcpy(m->params, d->params, pb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->mean, d->out_mean, ob, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->stdv, d->out_std, ob, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("copy to device failed");
        ddrom_mlp_destroy(m.release());
        return DDROM_EHIP;
    }
    for (int k = 0; k < m->T.n_layers; ++k) {
        const int r = m->T.sizes[k + 1], c = m->T.sizes[k];
        const long long n = (long long)r * c;
        hipLaunchKernelGGL(k_transpose_f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, m->params + m->T.w_off[k],
                           r, c, m->wt + m->T.w_off[k]);
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        set_error("weight transpose failed");
        ddrom_mlp_destroy(m.release());
        return DDROM_EHIP;
    }
    *out = m.release();
    return 0;
}

void ddrom_mlp_destroy(ddrom_mlp* m) {
    if (!m) return;
    if (m->wt) (void)hipFree(m->wt);
    if (m->params) (void)hipFree(m->params);
    if (m->mean) (void)hipFree(m->mean);
    if (m->stdv) (void)hipFree(m->stdv);
    delete m;
}

long long ddrom_mlp_size(const ddrom_mlp* m, int q) {
    if (!m) return -1;
    if (q == 0) return m->n_params;
    if (q == 1) return m->n_out;
    if (q == 2) return m->n_D;
    return -1;
}

int mlp_proposal(const ddrom_mlp* m, const double* mu_d, int B, double* xhat0_d, double* lam0_d, hipStream_t s) {
    if (!m || (B > 0 && (!mu_d || !xhat0_d)) || B < 0) {
        set_error("bad arguments to mlp_proposal");
        return DDROM_EINVAL;
    }
    if (B == 0) return 0;
    hipLaunchKernelGGL(k_mlp_infer, dim3((B + INFER_SPB - 1) / INFER_SPB), dim3(256), 0, s, m->T, m->wt, m->params,
                       m->mean, m->stdv, mu_d, B, m->n_D, xhat0_d, m->n_D, lam0_d, std::max(1, m->n_out - m->n_D));
    MLPCHECK(hipGetLastError());
    return 0;
}

int ddrom_mlp_trainer_create(const ddrom_mlp_desc* d, int max_batch, ddrom_mlp_trainer** out) {
    if (!d || !out || !d->params || max_batch <= 0) {
        set_error("bad arguments to ddrom_mlp_trainer_create");
        return DDROM_EINVAL;
    }
    *out = nullptr;
    std::unique_ptr<ddrom_mlp_trainer> t(new ddrom_mlp_trainer());
    int rc = make_table(d->n_layers, d->sizes, t->T, t->n_params);
    if (rc) return rc;
    t->max_B = max_batch;
    t->n_out = d->sizes[d->n_layers];
    const size_t pb = (size_t)t->n_params * sizeof(float);
    const size_t ab = (size_t)max_batch * t->T.maxw * sizeof(float);
    struct A { void** p; size_t bytes; } allocs[] = {
        {(void**)&t->p, pb}, {(void**)&t->g, pb}, {(void**)&t->m, pb}, {(void**)&t->v, pb},
        {(void**)&t->act, ab * (t->T.n_layers + 1)}, {(void**)&t->zbuf, ab * t->T.n_layers},
        {(void**)&t->d0, ab}, {(void**)&t->d1, ab}, {(void**)&t->part, MSE_BLOCKS * sizeof(double)},
        {(void**)&t->t, sizeof(int)},
    };
    for (auto& a : allocs)
        if (hipMalloc(a.p, a.bytes) != hipSuccess) {
            set_error("trainer allocation failed");
            ddrom_mlp_trainer_destroy(t.release());
            return DDROM_ENOMEM;
        }
    if (hipMemcpy(t->p, d->params, pb, hipMemcpyHostToDevice) != hipSuccess || hipMemset(t->m, 0, pb) != hipSuccess ||
        hipMemset(t->v, 0, pb) != hipSuccess || hipMemset(t->g, 0, pb) != hipSuccess ||
        hipMemset(t->t, 0, sizeof(int)) != hipSuccess) {
        set_error("trainer initialisation failed");
        ddrom_mlp_trainer_destroy(t.release());
        return DDROM_EHIP;
    }
    *out = t.release();
    return 0;
}

void ddrom_mlp_trainer_destroy(ddrom_mlp_trainer* t) {
    if (!t) return;
    void* ptrs[] = {t->p, t->g, t->m, t->v, t->act, t->zbuf, t->d0, t->d1, t->part, t->t};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete t;
}

int mlp_train_step(ddrom_mlp_trainer* t, const double* mu_d, const float* target_d, const int* rows_d, int B,
                   float lr, int update, float* loss_d, float* grad_d, hipStream_t s) {
    if (!t || !mu_d || !target_d || !rows_d || B <= 0 || B > t->max_B) {
        set_error("bad arguments to mlp_train_step (batch must be 1..max_batch)");
        return DDROM_EINVAL;
    }
    const LayerTable& T = t->T;
    const int L = T.n_layers;
    const size_t ab = (size_t)t->max_B * T.maxw;
    auto act = [&](int k) { return t->act + (size_t)k * ab; };
    auto zb = [&](int k) { return t->zbuf + (size_t)k * ab; };
    hipLaunchKernelGGL(k_mlp_gather, dim3((B + 255) / 256), dim3(256), 0, s, mu_d, rows_d, B, act(0));
    // forward: act(k+1) = sigma(act(k) W_k^T + b_k), rows of width sizes[k]
    for (int k = 0; k < L; ++k) {
        const int nin = T.sizes[k], nout = T.sizes[k + 1];
        dim3 grid((nout + 63) / 64, (B + 63) / 64);
        const float* W = t->p + T.w_off[k];
        const float* bk = t->p + T.b_off[k];
        if (k < L - 1)
            hipLaunchKernelGGL(k_gemm<1>, grid, dim3(256), 0, s, B, nout, nin, act(k), (long long)nin, 1LL, W, 1LL,
                               (long long)nin, act(k + 1), (long long)nout, bk, zb(k), (const float*)nullptr);
        else
            hipLaunchKernelGGL(k_gemm<2>, grid, dim3(256), 0, s, B, nout, nin, act(k), (long long)nin, 1LL, W, 1LL,
                               (long long)nin, act(k + 1), (long long)nout, bk, (float*)nullptr, (const float*)nullptr);
    }
    const int n = t->n_out;
    hipLaunchKernelGGL(k_mse, dim3(MSE_BLOCKS), dim3(256), 0, s, act(L), target_d, rows_d, B, n, t->d0, t->part);
    if (loss_d) hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(1), 0, s, t->part, MSE_BLOCKS, (long long)B * n, loss_d);
    // backward: d0 holds dZ_k (rows of width sizes[k+1])
    float* dcur = t->d0;
    float* dnext = t->d1;
    for (int k = L - 1; k >= 0; --k) {
        const int nin = T.sizes[k], nout = T.sizes[k + 1];
        // dW_k[o][i] = sum_b dZ[b][o] act(k)[b][i]
        hipLaunchKernelGGL(k_gemm<0>, dim3((nin + 63) / 64, (nout + 63) / 64), dim3(256), 0, s, nout, nin, B, dcur,
                           1LL, (long long)nout, act(k), (long long)nin, 1LL, t->g + T.w_off[k], (long long)nin,
                           (const float*)nullptr, (float*)nullptr, (const float*)nullptr);
        hipLaunchKernelGGL(k_colsum, dim3((nout + 255) / 256), dim3(256), 0, s, dcur, B, nout, t->g + T.b_off[k]);
        if (k > 0) {
            // dZ_{k-1}[b][i] = (sum_o dZ_k[b][o] W_k[o][i]) * SiLU'(Z_{k-1}[b][i])
            hipLaunchKernelGGL(k_gemm<3>, dim3((nin + 63) / 64, (B + 63) / 64), dim3(256), 0, s, B, nin, nout, dcur,
                               (long long)nout, 1LL, t->p + T.w_off[k], (long long)nin, 1LL, dnext, (long long)nin,
                               (const float*)nullptr, (float*)nullptr, (const float*)zb(k - 1));
            std::swap(dcur, dnext);
        }
    }
    if (grad_d) MLPCHECK(hipMemcpyAsync(grad_d, t->g, (size_t)t->n_params * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (update) {
        hipLaunchKernelGGL(k_adam_tick, dim3(1), dim3(1), 0, s, t->t);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((t->n_params + 255) / 256)), dim3(256), 0, s, t->n_params, t->p, t->g,
                           t->m, t->v, t->t, lr, 0.9f, 0.999f, 1e-8f);
    }
    MLPCHECK(hipGetLastError());
    return 0;
}

int ddrom_mlp_trainer_params(const ddrom_mlp_trainer* t, float* params_d, hipStream_t s) {
    if (!t || !params_d) {
        set_error("bad arguments to ddrom_mlp_trainer_params");
        return DDROM_EINVAL;
    }
    MLPCHECK(hipMemcpyAsync(params_d, t->p, (size_t)t->n_params * sizeof(float), hipMemcpyDeviceToDevice, s));
    return 0;
}

long long ddrom_mlp_trainer_size(const ddrom_mlp_trainer* t, int q) {
    if (!t) return -1;
    if (q == 0) return t->n_params;
    if (q == 1) return t->n_out;
    return -1;
}

}  // extern "C"
