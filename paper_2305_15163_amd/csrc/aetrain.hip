// Training of the shallow band-masked autoencoders (Sections 3.4 and 7.3) on the GPU:
// BF16 matrix-core (MFMA) products with FP32 accumulation, FP32 master weights, Adam.
//
// Network (eq. autoencoder_architecture), on normalised snapshots x~ (columns of a
// minibatch, feature-major layouts [features][B]):
//   encoder  ze = E1 x~ + b1e,  ae = sigma(ze),  xh = W2e ae          (E1: w x N, masked)
//   decoder  zd = W1d xh + b1d, ad = sigma(zd),  y  = D2 ad           (D2: N x w, masked)
//   loss     (1/B) sum_b sum_r (scale_r (y - x~)_rb)^2                 (raw-space MSE)
// D2 carries the three-band mask (row r: columns r s + k b s + t, k in {-1,0,1}, t < b) and E1
// its transpose.  Both masked weights are stored by band slot, W[r][k][t] (the slot of mask
// entry (r, c = r s + k b s + t)); slots whose column falls outside [0, w) hold zeros.
//
// Masked products run on dense 16 x 16 tiles: a 16-row tile of a band touches a window of
// 15 s + b columns per band, so the tile is expanded (zeros outside the band) into BF16 MFMA
// operands; the weight gradients are sampled dense products over the minibatch, kept only at
// band slots.  The dense latent layers (w <-> n) are skinny GEMMs (split over K where K = w).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

using namespace ddrom;

#define AECHECK(x)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) {                                                             \
            set_error(std::string(#x) + ": " + hipGetErrorString(e_));                      \
            return DDROM_EHIP;                                                              \
        }                                                                                   \
    } while (0)

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ short to_bf16(float f) {
    const unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (short)((u >> 16) | 0x40u);
    return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_to_f(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }

// 16 x 16 x 16 BF16 product, FP32 accumulate.  Lane l supplies A[l % 16][4 (l / 16) + i] and
// B[4 (l / 16) + i][l % 16] (i < 4) and holds D[4 (l / 16) + i][l % 16].  With x3 != 0 each
// operand is split into a BF16 head and a BF16 tail (a = a_h + a_l) and the product is
// a_h b_h + a_h b_l + a_l b_h: three matrix-core products, about 16 significant bits.
__device__ __forceinline__ f32x4 mma16(const float a[4], const float b[4], f32x4 c, int x3) {
    bf16x4 ah, bh;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        ah[i] = to_bf16(a[i]);
        bh[i] = to_bf16(b[i]);
    }
    if (x3) {
        bf16x4 al, bl;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            al[i] = to_bf16(a[i] - bf16_to_f(ah[i]));
            bl[i] = to_bf16(b[i] - bf16_to_f(bh[i]));
        }
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
}

__device__ __forceinline__ void act_fwd(float z, int act, float& a, float& d) {
    if (act == DDROM_ACT_IDENTITY) {
        a = z;
        d = 1.f;
        return;
    }
    const float sg = 1.f / (1.f + __expf(-z));
    if (act == DDROM_ACT_SIGMOID) {
        a = sg;
        d = sg * (1.f - sg);
    } else {
        a = z * sg;
        d = sg + z * sg * (1.f - sg);
    }
}

__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// LDS staging of minibatch-major rows: BG_K columns at a time, rows padded to BG_LD floats so
// that 16-byte operand reads of 16 consecutive rows fall in distinct banks.
constexpr int BG_K = 64, BG_LD = BG_K + 4;

// Four consecutive floats of a row with `avail` valid entries (16-byte load when aligned).
__device__ __forceinline__ float4 load_row4(const float* __restrict__ src, int avail, bool vec) {
    if (vec && avail >= 4) return *reinterpret_cast<const float4*>(src);
    float4 v = {0.f, 0.f, 0.f, 0.f};
    if (avail > 0) v.x = src[0];
    if (avail > 1) v.y = src[1];
    if (avail > 2) v.z = src[2];
    if (avail > 3) v.w = src[3];
    return v;
}

// ---- dense products:  C[m][n] = sum_k A(m, k) B(k, n),  A(m, k) = A[m sam + k sak] ----
// One wave per 16 x 16 output tile, four waves per workgroup (2 x 2 tiles, or 1 x 4 with wn).
// With split > 1 the K range is cut in `split` parts written to C + z M ldc (summed by
// k_split_sum).
// EPI 0: store; 1: + bias[m], Z = pre-activation, C = sigma; 2: times sigma'(aux[m][n]).
template <int EPI>
__global__ __launch_bounds__(256) void k_dense(int M, int N, int K, const float* __restrict__ A, long long sam,
                                               long long sak, const float* __restrict__ Bm, long long sbk,
                                               long long sbn, float* __restrict__ C, int ldc, int split,
                                               const float* __restrict__ bias, float* __restrict__ Z,
                                               const float* __restrict__ aux, int act, int x3, int wn,
                                               float* __restrict__ bsum = nullptr) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // wn = 0: the four waves take 2 x 2 tiles (32 x 32 per workgroup); wn = 1: four tiles along N
    // (16 x 64 per workgroup), for products with at most 16 rows
    const int m0 = wn ? blockIdx.y * 16 : (blockIdx.y * 2 + (wave >> 1)) * 16;
    const int n0 = wn ? (blockIdx.x * 4 + wave) * 16 : (blockIdx.x * 2 + (wave & 1)) * 16;
    const int z = blockIdx.z;
    const int kc = (K + split - 1) / split;
    const int kb = z * kc, ke = min(K, kb + kc);
    const int am = m0 + (lane & 15), bn = n0 + (lane & 15), kq = 4 * (lane >> 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if (m0 < M && n0 < N) {
        for (int k0 = kb; k0 < ke; k0 += 16) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k0 + kq + i;
                a[i] = (am < M && k < ke) ? A[(long long)am * sam + (long long)k * sak] : 0.f;
                b[i] = (bn < N && k < ke) ? Bm[(long long)k * sbk + (long long)bn * sbn] : 0.f;
            }
            acc = mma16(a, b, acc, x3);
        }
    }
    float* Cz = C + (size_t)z * M * ldc;
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + kq + i, n = n0 + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[i];
        const size_t ci = (size_t)m * ldc + n;
        if (EPI == 1) {
            v += bias[m];
            Z[ci] = v;
            float a, d;
            act_fwd(v, act, a, d);
            v = a;
        } else if (EPI == 2) {
            float a, d;
            act_fwd(aux[ci], act, a, d);
            v *= d;
        }
        Cz[ci] = v;
        part[i] = v;
    }
    if (bsum) {
        // wn = 1 with one workgroup column (N <= 64): the row sums over the N columns (the bias
        // gradient of the layer), lanes then waves in a fixed order
        __shared__ float red[4][16];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) part[i] += __shfl_xor(part[i], o, 64);
        if ((lane & 15) == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[wave][kq + i] = part[i];
        __syncthreads();
        if (threadIdx.x < 16 && m0 + (int)threadIdx.x < M)
            bsum[m0 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    }
}

// C[e] = sum_z P[z][e]: one workgroup per output, thread t sums z = t, t + 256, ..., then a
// fixed-order tree in LDS (the same order whatever the data).
__global__ __launch_bounds__(256) void k_split_sum(const float* __restrict__ P, int split, long long n,
                                                   float* __restrict__ C) {
    __shared__ float red[256];
    const long long e = blockIdx.x;
    float s = 0.f;
    for (int z = threadIdx.x; z < split; z += 256) s += P[(size_t)z * n + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) C[e] = red[0];
}

// ---- transposed band product:  Z[c][b] = sum_{r,k,t : c = r s + k b s + t} W[r][k][t] A[r][b] ----
// One wave per 16 (c) x 16 (b) tile, four waves per workgroup along b.  For band k the rows
// touching columns [c0, c0 + 16) form a run of at most (15 + b) / s + 1 rows, taken 16 at a
// time.  EPI 1: + bias[c], Z = pre-activation, out = sigma; 2: out = sum times sigma'(aux).
template <int EPI>
__global__ __launch_bounds__(256) void k_band_t(int N, int w, int bw, int sw, int B, const float* __restrict__ W,
                                                const float* __restrict__ Ain, float* __restrict__ out,
                                                const float* __restrict__ bias, float* __restrict__ Z,
                                                const float* __restrict__ aux, int act, int x3,
                                                float* __restrict__ bsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = blockIdx.x * 16, n0 = (blockIdx.y * 4 + wave) * 16;
    const int cm = c0 + (lane & 15), kq = 4 * (lane >> 4), bn = n0 + (lane & 15);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kb = -1; kb <= 1 && n0 < B; ++kb) {
        const int off = kb * bw * sw;
        const int r_lo = max(0, floor_div(c0 - (bw - 1) - off + sw - 1, sw));
        const int r_hi = min(N - 1, floor_div(c0 + 15 - off, sw));
        for (int rr = r_lo; rr <= r_hi; rr += 16) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = rr + kq + i;
                const int t = cm - r * sw - off;
                const bool in = r <= r_hi && t >= 0 && t < bw && cm < w;
                a[i] = in ? W[((size_t)r * 3 + (kb + 1)) * bw + t] : 0.f;
                b[i] = (r <= r_hi && bn < B) ? Ain[(size_t)r * B + bn] : 0.f;
            }
            acc = mma16(a, b, acc, x3);
        }
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = c0 + kq + i, n = n0 + (lane & 15);
        if (c >= w || n >= B) continue;
        const size_t ci = (size_t)c * B + n;
        float v = acc[i];
        if (EPI == 1) {
            v += bias[c];
            Z[ci] = v;
            float a, d;
            act_fwd(v, act, a, d);
            v = a;
        } else {
            float a, d;
            act_fwd(aux[ci], act, a, d);
            v *= d;
        }
        out[ci] = v;
        part[i] = v;
    }
    if (bsum) {
        // one workgroup row (B <= 64): the sums over the minibatch of the output (the bias
        // gradient of the layer below), lanes then waves in a fixed order
        __shared__ float red[4][16];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) part[i] += __shfl_xor(part[i], o, 64);
        if ((lane & 15) == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[wave][kq + i] = part[i];
        __syncthreads();
        if (threadIdx.x < 16 && c0 + (int)threadIdx.x < w)
            bsum[c0 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    }
}

// ---- band product with the loss:  y[r][b] = sum_{k,t} W[r][k][t] A[r s + k b s + t][b] ----
// diff = scale_r (y - x~), dY = (2 / B) scale_r diff, per-workgroup partial sums of diff^2.
__global__ __launch_bounds__(256) void k_band_loss(int N, int w, int bw, int sw, int B, const float* __restrict__ W,
                                                   const float* __restrict__ Ain, const float* __restrict__ Xb,
                                                   const float* __restrict__ scale, float* __restrict__ dY,
                                                   double* __restrict__ part, int x3) {
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = blockIdx.x * 16, n0 = (blockIdx.y * 4 + wave) * 16;
    const int rm = r0 + (lane & 15), kq = 4 * (lane >> 4), bn = n0 + (lane & 15);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if (n0 < B) {
        for (int kb = -1; kb <= 1; ++kb) {
            const int off = kb * bw * sw;
            const int cb = max(0, r0 * sw + off), ce = min(w, (r0 + 15) * sw + off + bw);
            for (int cc = cb; cc < ce; cc += 16) {
                float a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int c = cc + kq + i;
                    const int t = c - rm * sw - off;
                    const bool in = rm < N && c < ce && t >= 0 && t < bw;
                    a[i] = in ? W[((size_t)rm * 3 + (kb + 1)) * bw + t] : 0.f;
                    b[i] = (c < ce && bn < B) ? Ain[(size_t)c * B + bn] : 0.f;
                }
                acc = mma16(a, b, acc, x3);
            }
        }
    }
    double sq = 0.0;
    if (n0 < B) {
        const float sc2 = 2.f / (float)B;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + kq + i, n = n0 + (lane & 15);
            if (r >= N || n >= B) continue;
            const size_t ci = (size_t)r * B + n;
            const float d = scale[r] * (acc[i] - Xb[ci]);
            dY[ci] = sc2 * scale[r] * d;
            sq += (double)d * d;
        }
    }
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if (lane == 0) red[wave] = sq;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// ---- band-slot gradient:  G[r][k][t] = sum_b P[r][b] Q[r s + k b s + t][b] ----
// Per 16-row tile, each band's column window is cut in 16-column tiles; a wave forms the dense
// 16 x 16 product over the minibatch and keeps the band slots (all of them: no separate
// clearing pass).
__global__ __launch_bounds__(256) void k_band_grad(int N, int w, int bw, int sw, int B, const float* __restrict__ P,
                                                   const float* __restrict__ Q, float* __restrict__ G, int x3) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = blockIdx.x * 16;
    const int ntile = (15 * sw + bw + 15) / 16;      // column tiles per band window
    const int rm = r0 + (lane & 15), kq = 4 * (lane >> 4);
    // the rows' operand fragments are the same for every column tile: the first KC minibatch
    // chunks of 16 stay in registers
    constexpr int KC = 4;
    float pa[KC][4];
#pragma unroll
    for (int it = 0; it < KC; ++it)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int smp = it * 16 + kq + i;
            pa[it][i] = (rm < N && smp < B) ? P[(size_t)rm * B + smp] : 0.f;
        }
    for (int tt = wave; tt < 3 * ntile; tt += 4) {
        const int kb = tt / ntile - 1, ci = tt % ntile;
        const int off = kb * bw * sw;
        const int cc = r0 * sw + off + 16 * ci;
        const int cn = cc + (lane & 15);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int it = 0; it < KC; ++it) {
            if (it * 16 >= B) break;
            float b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int smp = it * 16 + kq + i;
                b[i] = (cn >= 0 && cn < w && smp < B) ? Q[(size_t)cn * B + smp] : 0.f;
            }
            acc = mma16(pa[it], b, acc, x3);
        }
        for (int s0 = KC * 16; s0 < B; s0 += 16) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int smp = s0 + kq + i;
                a[i] = (rm < N && smp < B) ? P[(size_t)rm * B + smp] : 0.f;
                b[i] = (cn >= 0 && cn < w && smp < B) ? Q[(size_t)cn * B + smp] : 0.f;
            }
            acc = mma16(a, b, acc, x3);
        }
        // the tiles of a band cover every slot of the 16 rows once; slots whose column falls
        // outside [0, w) summed zero operands and store 0
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + kq + i;
            const int t = cn - r * sw - off;
            if (r < N && t >= 0 && t < bw) G[((size_t)r * 3 + (kb + 1)) * bw + t] = acc[i];
        }
    }
}

// The same band-slot gradient with LDS staging: per 64 minibatch columns, the 16 rows of P and
// the union of their three band windows of Q (columns [r0 s - b s, r0 s + b s + 16 ntile)) are
// loaded with coalesced 16-byte loads into padded LDS rows; each wave keeps the accumulators of
// up to 4 column tiles (3 ntile <= 16, i.e. 15 s + b <= 80).

__global__ __launch_bounds__(256) void k_band_grad_lds(int N, int w, int bw, int sw, int B,
                                                       const float* __restrict__ P, const float* __restrict__ Q,
                                                       float* __restrict__ G, int x3) {
    extern __shared__ __align__(16) float sm[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = blockIdx.x * 16;
    const int ntile = (15 * sw + bw + 15) / 16, ntt = 3 * ntile;
    const int c_lo = r0 * sw - bw * sw, nc = 2 * bw * sw + 16 * ntile;
    float* Ps = sm;                       // [16][BG_LD]
    float* Qs = sm + 16 * BG_LD;          // [nc][BG_LD]
    const int rl = lane & 15, kq = 4 * (lane >> 4);
    const bool vec = (B & 3) == 0;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int s0 = 0; s0 < B; s0 += BG_K) {
        const int kn = min(BG_K, B - s0);
        for (int e = tid; e < (16 + nc) * (BG_K / 4); e += 256) {
            const int row = e / (BG_K / 4), q4 = (e % (BG_K / 4)) * 4;
            float4 v = {0.f, 0.f, 0.f, 0.f};
            if (row < 16) {
                const int r = r0 + row;
                if (r < N) v = load_row4(P + (size_t)r * B + s0 + q4, kn - q4, vec);
            } else {
                const int c = c_lo + row - 16;
                if (c >= 0 && c < w) v = load_row4(Q + (size_t)c * B + s0 + q4, kn - q4, vec);
            }
            *reinterpret_cast<float4*>(sm + (size_t)row * BG_LD + q4) = v;
        }
        __syncthreads();
        for (int it = 0; it < BG_K / 16 && s0 + it * 16 < B; ++it) {
            const float4 av = *reinterpret_cast<const float4*>(Ps + rl * BG_LD + it * 16 + kq);
            const float a[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int tt = wave + 4 * t;
                if (tt >= ntt) break;
                const int kb = tt / ntile - 1, ci = tt % ntile;
                const int cl = bw * sw + kb * bw * sw + 16 * ci + rl;
                const float4 bv = *reinterpret_cast<const float4*>(Qs + (size_t)cl * BG_LD + it * 16 + kq);
                const float b[4] = {bv.x, bv.y, bv.z, bv.w};
                acc[t] = mma16(a, b, acc[t], x3);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int tt = wave + 4 * t;
        if (tt >= ntt) break;
        const int kb = tt / ntile - 1, ci = tt % ntile;
        const int off = kb * bw * sw;
        const int cn = r0 * sw + off + 16 * ci + rl;
        // every slot of the 16 rows lies in exactly one tile; slots whose column falls outside
        // [0, w) summed zero operands and store 0
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + kq + i;
            const int tq = cn - r * sw - off;
            if (r < N && tq >= 0 && tq < bw) G[((size_t)r * 3 + (kb + 1)) * bw + tq] = acc[t][i];
        }
    }
}

// minibatch of normalised snapshots, feature-major: Xb[r][b] = X[rows[b]][r]
__global__ void k_ae_gather(const float* __restrict__ X, int N, const int* __restrict__ rows, int B,
                            float* __restrict__ Xb) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)N * B) return;
    const int r = (int)(e / B), b = (int)(e % B);
    Xb[e] = X[(size_t)rows[b] * N + r];
}

// out[m] = sum_b D[m][b]: one wave per row, lanes along the minibatch (coalesced loads), then
// a butterfly sum (every lane ends with the same value).
__global__ __launch_bounds__(256) void k_rowsum(const float* __restrict__ D, int M, int B, float* __restrict__ out) {
    const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (m >= M) return;
    float s = 0.f;
    for (int b = lane; b < B; b += 64) s += D[(size_t)m * B + b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[m] = s;
}

__global__ void k_loss_final(const double* __restrict__ part, int n, int B, float* __restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    loss[0] = (float)(s / B);
}

// Adam (Section 7.3), step number `step` (1, 2, ...) counted on the host.
__global__ void k_ae_adam(long long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, int step, float lr) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi, vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

struct ddrom_ae_trainer {
    int N = 0, n = 0, bw = 0, sw = 0, w = 0, act = 0, max_B = 0;
    long long n_band = 0, n_params = 0;
    long long o_w1e = 0, o_b1e = 0, o_w2e = 0, o_w1d = 0, o_b1d = 0, o_w2d = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *Xb = nullptr, *ze = nullptr, *ae = nullptr, *zd = nullptr, *ad = nullptr, *dY = nullptr, *dzd = nullptr;
    float *dze = nullptr, *xh = nullptr, *dxh = nullptr, *kpart = nullptr;
    double* lpart = nullptr;
    int step = 0;              // Adam steps taken
    int split = 1;
    int x3 = 0;                // 1: split-BF16 (three products) for FP32-class operands
};

// Transposed band product (encoder forward: EPI 1; decoder backward: EPI 2), with the bias
// gradient sum when one workgroup row covers the minibatch.  Returns whether bsum was formed.
template <int EPI>
static bool band_t(const ddrom_ae_trainer* t, int B, const float* W, const float* Ain, float* out, const float* bias,
                   float* Z, const float* aux, float* bsum, hipStream_t s) {
    const dim3 grid(cdiv(t->w, 16), cdiv(B, 64));
    float* bs = grid.y == 1 ? bsum : nullptr;
    hipLaunchKernelGGL(k_band_t<EPI>, grid, dim3(256), 0, s, t->N, t->w, t->bw, t->sw, B, W, Ain, out, bias, Z, aux,
                       t->act, t->x3, bs);
    return bs != nullptr;
}

// Band-slot gradient G = sampled P Q^T: the LDS-staged kernel where its window fits, else the
// plain one.
static void band_grad(const ddrom_ae_trainer* t, int B, const float* P, const float* Q, float* G, hipStream_t s) {
    const int ntile = (15 * t->sw + t->bw + 15) / 16;
    const size_t lds = (size_t)(16 + 2 * t->bw * t->sw + 16 * ntile) * BG_LD * sizeof(float);
    if (3 * ntile <= 16 && lds <= 65536)
        hipLaunchKernelGGL(k_band_grad_lds, dim3(cdiv(t->N, 16)), dim3(256), lds, s, t->N, t->w, t->bw, t->sw, B, P,
                           Q, G, t->x3);
    else
        hipLaunchKernelGGL(k_band_grad, dim3(cdiv(t->N, 16)), dim3(256), 0, s, t->N, t->w, t->bw, t->sw, B, P, Q, G,
                           t->x3);
}

extern "C" {

int ddrom_ae_trainer_create(int N, int n, int b, int s, int activation, int max_batch, int precision,
                            const float* params_h, ddrom_ae_trainer** out) {
    if (!out || !params_h || N <= 0 || n <= 0 || n > 64 || b <= 0 || s <= 0 || max_batch <= 0 || activation < 0 ||
        activation > 2 || (precision != 0 && precision != 1)) {
        set_error("bad arguments to ddrom_ae_trainer_create");
        return DDROM_EINVAL;
    }
    *out = nullptr;
    std::unique_ptr<ddrom_ae_trainer> t(new ddrom_ae_trainer());
    t->N = N; t->n = n; t->bw = b; t->sw = s; t->w = N * s; t->act = activation; t->max_B = max_batch;
    t->x3 = precision;
    const long long w = t->w;
    t->n_band = 3LL * N * b;
    t->o_w1e = 0;
    t->o_b1e = t->o_w1e + t->n_band;
    t->o_w2e = t->o_b1e + w;
    t->o_w1d = t->o_w2e + (long long)n * w;
    t->o_b1d = t->o_w1d + w * n;
    t->o_w2d = t->o_b1d + w;
    t->n_params = t->o_w2d + t->n_band;
    // about 64 K entries per split part of the skinny products with K = w (enough workgroups to
    // fill the device), at most 256 parts
    t->split = (int)std::max<long long>(1, std::min<long long>(256, w / 64));
    const size_t pb = (size_t)t->n_params * sizeof(float);
    const size_t Bm = (size_t)max_batch;
    struct A { void** p; size_t bytes; } allocs[] = {
        {(void**)&t->p, pb}, {(void**)&t->g, pb}, {(void**)&t->m, pb}, {(void**)&t->v, pb},
        {(void**)&t->Xb, N * Bm * 4}, {(void**)&t->ze, w * Bm * 4}, {(void**)&t->ae, w * Bm * 4},
        {(void**)&t->zd, w * Bm * 4}, {(void**)&t->ad, w * Bm * 4}, {(void**)&t->dY, N * Bm * 4},
        {(void**)&t->dzd, w * Bm * 4}, {(void**)&t->dze, w * Bm * 4}, {(void**)&t->xh, n * Bm * 4},
        {(void**)&t->dxh, n * Bm * 4}, {(void**)&t->kpart, (size_t)t->split * n * Bm * 4},
        {(void**)&t->lpart, (size_t)cdiv(N, 16) * cdiv(max_batch, 64) * 8},
    };
    for (auto& a : allocs)
        if (hipMalloc(a.p, a.bytes) != hipSuccess) {
            set_error("trainer allocation failed");
            ddrom_ae_trainer_destroy(t.release());
            return DDROM_ENOMEM;
        }
    if (hipMemcpy(t->p, params_h, pb, hipMemcpyHostToDevice) != hipSuccess || hipMemset(t->m, 0, pb) != hipSuccess ||
        hipMemset(t->v, 0, pb) != hipSuccess) {
        set_error("trainer initialisation failed");
        ddrom_ae_trainer_destroy(t.release());
        return DDROM_EHIP;
    }
    *out = t.release();
    return 0;
}

void ddrom_ae_trainer_destroy(ddrom_ae_trainer* t) {
    if (!t) return;
    void* ptrs[] = {t->p, t->g, t->m, t->v, t->Xb, t->ze, t->ae, t->zd, t->ad, t->dY, t->dzd, t->dze, t->xh, t->dxh,
                    t->kpart, t->lpart};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete t;
}

long long ddrom_ae_trainer_size(const ddrom_ae_trainer* t, int q) {
    if (!t) return -1;
    switch (q) {
        case 0: return t->n_params;
        case 1: return t->w;
        case 2: return t->n_band;
        default: return -1;
    }
}

int ddrom_ae_trainer_params(const ddrom_ae_trainer* t, float* params_d, hipStream_t s) {
    if (!t || !params_d) {
        set_error("bad arguments to ddrom_ae_trainer_params");
        return DDROM_EINVAL;
    }
    AECHECK(hipMemcpyAsync(params_d, t->p, (size_t)t->n_params * sizeof(float), hipMemcpyDeviceToDevice, s));
    return 0;
}

int ae_train_step(ddrom_ae_trainer* t, const float* X_d, const int* rows_d, int B, const float* scale_d, float lr,
                  int update, float* loss_d, float* grad_d, hipStream_t s) {
    if (!t || !X_d || !rows_d || !scale_d || B <= 0 || B > t->max_B) {
        set_error("bad arguments to ae_train_step (batch must be 1..max_batch)");
        return DDROM_EINVAL;
    }
    const int N = t->N, n = t->n, w = t->w, bw = t->bw, sw = t->sw, act = t->act;
    float* P = t->p;
    float* G = t->g;
    const dim3 blk(256);
    hipLaunchKernelGGL(k_ae_gather, dim3(cdiv((long long)N * B, 256)), blk, 0, s, X_d, N, rows_d, B, t->Xb);
    // encoder: ze = E1 x~ + b1e, ae = sigma(ze)
    band_t<1>(t, B, P + t->o_w1e, t->Xb, t->ae, P + t->o_b1e, t->ze, nullptr, nullptr, s);
    // xh = W2e ae (K = w, split)
    const int wn = n <= 16;
    const dim3 sgrid = wn ? dim3(cdiv(B, 64), cdiv(n, 16), t->split) : dim3(cdiv(B, 32), cdiv(n, 32), t->split);
    hipLaunchKernelGGL(k_dense<0>, sgrid, blk, 0, s, n, B, w, P + t->o_w2e, (long long)w, 1LL, t->ae, (long long)B,
                       1LL, t->kpart, B, t->split, (const float*)nullptr, (float*)nullptr, (const float*)nullptr, act,
                       t->x3, wn);
    hipLaunchKernelGGL(k_split_sum, dim3((unsigned)((long long)n * B)), blk, 0, s, t->kpart, t->split,
                       (long long)n * B, t->xh);
    // decoder: zd = W1d xh + b1d, ad = sigma(zd)
    hipLaunchKernelGGL(k_dense<1>, dim3(cdiv(B, 32), cdiv(w, 32), 1), blk, 0, s, w, B, n, P + t->o_w1d, (long long)n,
                       1LL, t->xh, (long long)B, 1LL, t->ad, B, 1, P + t->o_b1d, t->zd, (const float*)nullptr, act,
                       t->x3, 0);
    // y = D2 ad, loss and dY
    const dim3 lgrid(cdiv(N, 16), cdiv(B, 64));
    hipLaunchKernelGGL(k_band_loss, lgrid, blk, 0, s, N, w, bw, sw, B, P + t->o_w2d, t->ad, t->Xb, scale_d, t->dY,
                       t->lpart, t->x3);
    if (loss_d) hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1), 0, s, t->lpart, (int)(lgrid.x * lgrid.y), B, loss_d);
    // gradients
    band_grad(t, B, t->dY, t->ad, G + t->o_w2d, s);
    // dzd = (D2^T dY) o sigma'(zd)
    // (with B <= 64 the bias gradient gb1d = sum_b dzd comes from the same kernel)
    const bool fused_b1d = band_t<2>(t, B, P + t->o_w2d, t->dY, t->dzd, nullptr, nullptr, t->zd,
                                     B <= 64 ? G + t->o_b1d : nullptr, s);
    // gW1d = dzd xh^T, gb1d = sum_b dzd
    hipLaunchKernelGGL(k_dense<0>, dim3(cdiv(n, 32), cdiv(w, 32), 1), blk, 0, s, w, n, B, t->dzd, (long long)B, 1LL,
                       t->xh, 1LL, (long long)B, G + t->o_w1d, n, 1, (const float*)nullptr, (float*)nullptr,
                       (const float*)nullptr, act, t->x3, 0);
    if (!fused_b1d) hipLaunchKernelGGL(k_rowsum, dim3(cdiv(w, 4)), blk, 0, s, t->dzd, w, B, G + t->o_b1d);
    // dxh = W1d^T dzd (K = w, split)
    hipLaunchKernelGGL(k_dense<0>, sgrid, blk, 0, s, n, B, w, P + t->o_w1d, 1LL, (long long)n, t->dzd, (long long)B,
                       1LL, t->kpart, B, t->split, (const float*)nullptr, (float*)nullptr, (const float*)nullptr, act,
                       t->x3, wn);
    hipLaunchKernelGGL(k_split_sum, dim3((unsigned)((long long)n * B)), blk, 0, s, t->kpart, t->split,
                       (long long)n * B, t->dxh);
    // gW2e = dxh ae^T
    hipLaunchKernelGGL(k_dense<0>, dim3(cdiv(w, 32), cdiv(n, 32), 1), blk, 0, s, n, w, B, t->dxh, (long long)B, 1LL,
                       t->ae, 1LL, (long long)B, G + t->o_w2e, w, 1, (const float*)nullptr, (float*)nullptr,
                       (const float*)nullptr, act, t->x3, 0);
    // dze = (W2e^T dxh) o sigma'(ze)
    // (with B <= 64, one workgroup column of 16 x 64 tiles, which also sums gb1e = sum_b dze)
    const bool fused_b1e = B <= 64;
    if (fused_b1e)
        hipLaunchKernelGGL(k_dense<2>, dim3(1, cdiv(w, 16), 1), blk, 0, s, w, B, n, P + t->o_w2e, 1LL, (long long)w,
                           t->dxh, (long long)B, 1LL, t->dze, B, 1, (const float*)nullptr, (float*)nullptr, t->ze, act,
                           t->x3, 1, G + t->o_b1e);
    else
        hipLaunchKernelGGL(k_dense<2>, dim3(cdiv(B, 32), cdiv(w, 32), 1), blk, 0, s, w, B, n, P + t->o_w2e, 1LL,
                           (long long)w, t->dxh, (long long)B, 1LL, t->dze, B, 1, (const float*)nullptr,
                           (float*)nullptr, t->ze, act, t->x3, 0, (float*)nullptr);
    // gW1e[r][k][t] = sum_b x~[r][b] dze[c][b], gb1e = sum_b dze
    band_grad(t, B, t->Xb, t->dze, G + t->o_w1e, s);
    if (!fused_b1e) hipLaunchKernelGGL(k_rowsum, dim3(cdiv(w, 4)), blk, 0, s, t->dze, w, B, G + t->o_b1e);
    if (grad_d) AECHECK(hipMemcpyAsync(grad_d, G, (size_t)t->n_params * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (update) {
        t->step += 1;
        hipLaunchKernelGGL(k_ae_adam, dim3(cdiv(t->n_params, 256)), blk, 0, s, t->n_params, P, G, t->m, t->v,
                           t->step, lr);
    }
    AECHECK(hipGetLastError());
    return 0;
}

}  // extern "C"
