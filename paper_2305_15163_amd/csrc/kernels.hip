// HIP kernels for gfx950 and the C ABI of the HR DD NM-ROM online solve.
//
// Batch layout: one solve per wavefront lane.  Every per-solve buffer that a
// batch-as-lanes kernel touches is stored [...][Bp] (solve index fastest, Bp = B rounded up
// to 64), so a wave's 64 lanes read and write 64 consecutive elements, while the weights
// of a decoder, the gather tables and C A_i are indexed only by wave-uniform values and are
// fetched through the scalar cache, shared by the 64 solves of the wave.
//
// One solver round (one evaluation of every active solve at its trial point) is
//   k_decode   interior subnets (eq. subnet) and full interface decoders, value + Jacobian
//   k_res_gn   HR Burgers residual at the sampled nodes, Z R_i by the chain rule, and the
//              Gauss-Newton blocks H_i = (Z R_i)^T Z R_i, g_i = (Z R_i)^T Z r_i (partial sums)
//   k_con      weak constraint sum_i C A_i g_i^Gamma and E_i^Gamma = C A_i dg_i^Gamma/dxhat
//   k_reduce   sums the partial slots of each solve into one contiguous record
//   k_update   one workgroup per solve: merit, Armijo test, KKT solve by Schur complement on
//              the block-arrow system (eq. sqp_system), next trial point
//   k_compact  list of the solves still running; the next round's kernels run over it only
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>

#include "internal.h"

using namespace ddrom;

namespace ddrom {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace ddrom

#define HIPCHECK(x)                                                                         \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) {                                                             \
            set_error(std::string(#x) + ": " + hipGetErrorString(e_));                      \
            return DDROM_EHIP;                                                              \
        }                                                                                   \
    } while (0)

static constexpr int RING = 64;
static constexpr int PH_INIT = 0, PH_TRIAL = 1, PH_DONE = 2, PH_ZERO = 3;
static constexpr int KKT_NN = 20;     // max n_i^Omega + n_i^Gamma
static constexpr int KKT_MG = 12;     // max n_i^Gamma
static constexpr int KKT_NC = 64;     // n_C < KKT_NC

// ------------------------------------------------------------------------------------
// Activations
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void act_eval(float z, int act, float& s, float& d) {
    if (act == DDROM_ACT_IDENTITY) {
        s = z;
        d = 1.0f;
        return;
    }
    float e = __expf(-z);
    float sg = __builtin_amdgcn_rcpf(1.0f + e);
    if (act == DDROM_ACT_SIGMOID) {
        s = sg;
        d = sg * (1.0f - sg);
    } else {
        s = z * sg;
        d = sg + z * sg * (1.0f - sg);
    }
}

__device__ __forceinline__ void act_eval(double z, int act, double& s, double& d) {
    if (act == DDROM_ACT_IDENTITY) {
        s = z;
        d = 1.0;
        return;
    }
    double sg = 1.0 / (1.0 + exp(-z));
    if (act == DDROM_ACT_SIGMOID) {
        s = sg;
        d = sg * (1.0 - sg);
    } else {
        s = z * sg;
        d = sg + z * sg * (1.0 - sg);
    }
}

// Solve slots.  Batch kernels run over slots j = 0, 1, ...: during a solve, slot j holds the
// j-th still-running solve (live[j], ascending) and only the first *n_live slots are in use,
// so a round costs in proportion to the running solves; per-round buffers (decoder output,
// partial sums, reduced blocks) are indexed by slot, per-solve state by the solve index.
// Without a live list (live == nullptr) slot j is solve j and all B slots are in use.
__device__ __forceinline__ int live_count(const int* n_live, int B) { return n_live ? *n_live : B; }
__device__ __forceinline__ int slot_solve(const int* live, int j, int nl) {
    return j < nl ? (live ? live[j] : j) : 0;
}

// ------------------------------------------------------------------------------------
// Decoder: value and Jacobian rows of g(xhat) = x_ref + W2~ sigma(W1~ xhat + b1~)
// ------------------------------------------------------------------------------------
// A workgroup of WAVES waves takes one work item (a run of consecutive kept rows of one
// decoder) for WAVES x 64 solves, one solve per lane.  The weights the rows read (W1~ rows
// and biases of their hidden units, W2~ band values, x_ref, band descriptors) are staged
// once in LDS with coalesced loads and read back as wave-wide broadcasts.  Rows are visited
// in ascending order; each row's three bands lie in a window of at most RING consecutive
// compressed hidden units, so every hidden activation is computed once per lane into a
// per-lane ring in LDS and consumed by the rows that need it.  For the sigmoid the ring
// holds s = sigma(z) and sigma' = s - s^2 is formed on use; the swish keeps (value, sigma').

template <typename T, int ACT>
struct RingSlots { static constexpr int K = (ACT == DDROM_ACT_SWISH) ? 2 : 1; };

template <typename T>
__device__ __forceinline__ T sig_fast(T z);
template <>
__device__ __forceinline__ float sig_fast<float>(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
template <>
__device__ __forceinline__ double sig_fast<double>(double z) { return 1.0 / (1.0 + exp(-z)); }

// TAG only renames the instantiation (0: solver rounds, 1: standalone timing launches) so that
// profiler summaries separate the two; the code is identical.  VO = 1 evaluates values only
// (decoded states after a solve): row r goes to Bp-row out + r.
template <typename T, int NL, int ACT, int WAVES, int TAG, int VO = 0, int RING = DEC_RING>
__global__ __launch_bounds__(64 * WAVES) void k_decode(const DecChunk* __restrict__ chunks, int chunk_base,
                                                       const DecSeg* __restrict__ segs, const T* __restrict__ W1,
                                                       const T* __restrict__ B1, const int2* __restrict__ bands,
                                                       const T* __restrict__ W2, const T* __restrict__ XR,
                                                       const double* __restrict__ xhat, int xstride, int xoff_override,
                                                       const int* __restrict__ live, const int* __restrict__ n_live,
                                                       int B, T* __restrict__ out, int Bp, long long oshift) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int RK = RingSlots<T, ACT>::K;
    const DecChunk ch = chunks[chunk_base + blockIdx.x];
    const DecSeg sg = segs[ch.seg];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nl = live_count(n_live, B);
    // Slot groups of 64 running solves -> waves.  While there are more running groups than
    // workgroup rows (gridDim.y), workgroup row y takes groups 4y .. 4y + 3; when only one or
    // two of them run (the last rounds of a batch), the idle waves take a share of the rows
    // instead: G slot groups x R row parts.  Once the running groups fit in the workgroup rows,
    // each workgroup row takes one group and all its waves split the rows (R = WAVES).  Each
    // wave keeps its own activation ring.
    const int groups_live = (nl + 63) / 64;
    int R, G, group_abs;
    if (groups_live <= (int)gridDim.y) {
        if ((int)blockIdx.y >= groups_live) return;
        R = WAVES;
        G = 1;
        group_abs = blockIdx.y;
    } else {
        const int j0 = (int)blockIdx.y * WAVES * 64;
        if (j0 >= nl) return;     // every slot of this workgroup is idle
        const int live_groups = min(WAVES, (nl - j0 + 63) / 64);
        R = live_groups == 1 ? WAVES : ((live_groups == 2 && WAVES % 2 == 0) ? WAVES / 2 : 1);
        G = WAVES / R;
        group_abs = blockIdx.y * WAVES + wave % G;
    }
    const int part = wave / G;
    const int j = group_abs * 64 + lane;
    const bool act = j < nl;
    const int b = slot_solve(live, j, nl);

    const int nrows = ch.r1 - ch.r0, span = ch.h_hi - ch.h_lo, bmax = sg.bmax;
    const DecLds L = dec_lds(span, nrows, NL, bmax, (int)sizeof(T), WAVES, RK, RING);
    T* sW1 = reinterpret_cast<T*>(smem + L.w1);          // [span][NL]
    T* sB1 = reinterpret_cast<T*>(smem + L.b1);          // [span]
    T* sW2 = reinterpret_cast<T*>(smem + L.w2);          // [nrows][3][bmax]
    T* sXR = reinterpret_cast<T*>(smem + L.xr);          // [nrows]
    int2* sBd = reinterpret_cast<int2*>(smem + L.bd);    // [nrows][3]
    T* ring = reinterpret_cast<T*>(smem + L.ring) + (size_t)wave * RING * 64 * RK;
    {
        const T* gW1 = W1 + sg.w1 + (size_t)ch.h_lo * NL;
        for (int i = tid; i < span * NL; i += 64 * WAVES) sW1[i] = gW1[i];
        const T* gB1 = B1 + sg.b1 + ch.h_lo;
        for (int i = tid; i < span; i += 64 * WAVES) sB1[i] = gB1[i];
        const T* gW2 = W2 + sg.w2 + (size_t)ch.r0 * 3 * bmax;
        for (int i = tid; i < nrows * 3 * bmax; i += 64 * WAVES) sW2[i] = gW2[i];
        const T* gXR = XR + sg.xref + ch.r0;
        for (int i = tid; i < nrows; i += 64 * WAVES) sXR[i] = gXR[i];
        const int2* gBd = bands + sg.band + (size_t)ch.r0 * 3;
        for (int i = tid; i < nrows * 3; i += 64 * WAVES) {
            int2 q = gBd[i];
            q.x -= ch.h_lo;
            sBd[i] = q;
        }
    }
    const int xo = xoff_override >= 0 ? xoff_override : sg.xoff;
    T xl[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) xl[k] = act ? (T)xhat[(size_t)b * xstride + xo + k] : (T)0;
    __syncthreads();

    // output rows are numbered from the segment's first row in the model's decoder-output
    // layout, less oshift (nonzero when the output buffer holds this segment alone)
    T* o = out + ((size_t)(sg.out - oshift) + (size_t)ch.r0 * (VO ? 1 : 1 + NL)) * Bp + j;
    // Units [vlo, vhi) (relative to h_lo) are valid in the ring; vhi - vlo <= RING.  Rows
    // ascend, so windows mostly slide right, but near the first rows of a decoder a clipped
    // band can start below the previous row's window: missing units are then computed on
    // whichever side they lie.
    int vlo = 0, vhi = 0;
    auto hidden = [&](int h) {
        const T* w = sW1 + (size_t)h * NL;
        T z = sB1[h];
#pragma unroll
        for (int k = 0; k < NL; ++k) z += w[k] * xl[k];
        T* rs = ring + (size_t)(h % RING) * 64 * RK + lane;
        if (ACT == DDROM_ACT_SIGMOID) {
            rs[0] = sig_fast<T>(z);
        } else if (ACT == DDROM_ACT_SWISH) {
            const T sg_ = sig_fast<T>(z);
            rs[0] = z * sg_;
            rs[64] = sg_ + z * sg_ * ((T)1 - sg_);
        } else {
            rs[0] = z;
        }
    };
    const int r_begin = nrows * part / R, r_end = nrows * (part + 1) / R;
    // band descriptors are the same for every lane: kept in scalar registers, so the row's window
    // and ring-slot bookkeeping run on the scalar unit
    auto ubd = [&](int i) {
        const int2 q = sBd[i];
        return make_int2(__builtin_amdgcn_readfirstlane(q.x), __builtin_amdgcn_readfirstlane(q.y));
    };
    for (int r = r_begin; r < r_end; ++r) {
        const int2 q0 = ubd(r * 3 + 0), q1 = ubd(r * 3 + 1), q2 = ubd(r * 3 + 2);
        int lo = 0x7fffffff, hi = -1;
        if (q0.y > 0) { lo = min(lo, q0.x); hi = max(hi, q0.x + q0.y); }
        if (q1.y > 0) { lo = min(lo, q1.x); hi = max(hi, q1.x + q1.y); }
        if (q2.y > 0) { lo = min(lo, q2.x); hi = max(hi, q2.x + q2.y); }
        if (lo >= vhi || hi <= vlo) {      // disjoint from the valid range: start afresh
            vlo = lo;
            vhi = lo;
        }
        for (int h = lo; h < vlo; ++h) hidden(h);
        vlo = min(vlo, lo);
        for (int h = vhi; h < hi; ++h) hidden(h);
        vhi = max(vhi, hi);
        vlo = max(vlo, vhi - RING);
        T acc = sXR[r];
        T J[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) J[k] = (T)0;
#pragma unroll
        for (int kb = 0; kb < 3; ++kb) {
            const int2 q = kb == 0 ? q0 : (kb == 1 ? q1 : q2);
            const T* w2r = sW2 + ((size_t)r * 3 + kb) * bmax;
            int slot = q.x % RING;
            for (int t = 0; t < q.y; ++t) {
                const T wv = w2r[t];
                const T* rs = ring + (size_t)slot * 64 * RK + lane;
                const T a = rs[0];
                T d;
                if (ACT == DDROM_ACT_SIGMOID) d = a - a * a;
                else if (ACT == DDROM_ACT_SWISH) d = rs[64];
                else d = (T)1;
                acc += wv * a;
                if (!VO) {
                    const T c = wv * d;
                    const T* w = sW1 + (size_t)(q.x + t) * NL;
#pragma unroll
                    for (int k = 0; k < NL; ++k) J[k] += c * w[k];
                }
                slot = slot + 1 == RING ? 0 : slot + 1;
            }
        }
        if (j < Bp) {   // waves past the padded batch (small B) compute but never store
            T* orow = o + (size_t)r * (VO ? 1 : 1 + NL) * Bp;
            orow[0] = acc;
            if (!VO)
#pragma unroll
                for (int k = 0; k < NL; ++k) orow[(size_t)(1 + k) * Bp] = J[k];
        }
    }
}

// ------------------------------------------------------------------------------------
// Pointwise central-difference Burgers residual (eq. burgers_discretized in stencil form)
// v: u_C, u_W, u_E, u_S, u_N, v_C, v_W, v_E, v_S, v_N
// cu: d r_u / d(u_C, u_W, u_E, u_S, u_N, v_C); cv: d r_v / d(v_C, v_W, v_E, v_S, v_N, u_C)
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void burgers_point(const double* v, double nu, double hx, double hy, double& ru, double& rv,
                                              double* cu, double* cv) {
    const double ihx2 = 0.5 / hx, ihy2 = 0.5 / hy, ax = nu / (hx * hx), ay = nu / (hy * hy);
    const double uc = v[S_UC], vc = v[S_VC];
    const double dux = (v[S_UE] - v[S_UW]) * ihx2, duy = (v[S_UN] - v[S_US]) * ihy2;
    const double dvx = (v[S_VE] - v[S_VW]) * ihx2, dvy = (v[S_VN] - v[S_VS]) * ihy2;
    const double lu = ax * (v[S_UE] - 2.0 * uc + v[S_UW]) + ay * (v[S_UN] - 2.0 * uc + v[S_US]);
    const double lv = ax * (v[S_VE] - 2.0 * vc + v[S_VW]) + ay * (v[S_VN] - 2.0 * vc + v[S_VS]);
    ru = -uc * dux - vc * duy + lu;
    rv = -uc * dvx - vc * dvy + lv;
    const double diag = -2.0 * (ax + ay);
    const double cw = uc * ihx2 + ax, ce = -uc * ihx2 + ax, cs = vc * ihy2 + ay, cn = -vc * ihy2 + ay;
    cu[0] = -dux + diag; cu[1] = cw; cu[2] = ce; cu[3] = cs; cu[4] = cn; cu[5] = -duy;
    cv[0] = -dvy + diag; cv[1] = cw; cv[2] = ce; cv[3] = cs; cv[4] = cn; cv[5] = -dvx;
}

__device__ __forceinline__ void exact_uv(double x, double y, double a, double lam, double nu, double& u, double& v) {
    const double ep = exp(lam * (x - 1.0)), em = exp(-lam * (x - 1.0));
    const double c = cos(lam * y), s = sin(lam * y);
    const double psi = a * (1.0 + x) + (ep + em) * c;
    u = -2.0 * nu * (a + lam * (ep - em) * c) / psi;
    v = 2.0 * nu * (lam * (ep + em) * s) / psi;
}

// Dirichlet values at the boundary points touched by sampled stencils, per solve.
__global__ void k_bc(const double* __restrict__ xy, const int* __restrict__ field, int n_bc,
                     const double* __restrict__ mu, int B, int Bp, double nu, double* __restrict__ bc) {
    const int b = blockIdx.y * blockDim.x + threadIdx.x;
    const int k = blockIdx.x;
    if (b >= Bp || k >= n_bc) return;
    double u = 0.0, v = 0.0;
    if (b < B) exact_uv(xy[2 * k], xy[2 * k + 1], mu[2 * b], mu[2 * b + 1], nu, u, v);
    bc[(size_t)k * Bp + b] = field[k] == 0 ? u : v;
}

// ------------------------------------------------------------------------------------
// HR residual, chain rule and Gauss-Newton partial sums
// ------------------------------------------------------------------------------------
// Workgroup -> work item within its 64-solve group (blockIdx.y).  Workgroups go to the 8 XCDs
// round-robin by linear id, so within one group the workgroups with equal blockIdx.x % 8 share
// an XCD; they take one contiguous run of work items, so that neighbouring items, which read many
// of the same decoder rows, share one L2.  Solve groups keep their dispatch order (idle groups
// exit at once, after the live ones).  A bijection on each group's items: the last
// gridDim.x % 8 items keep the plain order.
__device__ __forceinline__ int xcd_item() {
    const int l = blockIdx.x, cpx = (int)gridDim.x >> 3;
    return l < 8 * cpx ? (l & 7) * cpx + (l >> 3) : l;
}

// The ten stencil DoFs of one sampled node for 64 solves (lanes): values and Jacobian rows
// gathered from the decoder output or, for boundary slots, the per-solve Dirichlet buffer.
// All loads of a node are issued before any is used.
template <typename T, int NO>
struct NodeLoads {
    int kind[N_SLOTS];
    double v[N_SLOTS];
    T jv[N_SLOTS][NO];
};

template <typename T, int NO, int NG>
__device__ __forceinline__ void load_node(const int* __restrict__ code, const T* dom, const T* dga, const T* dz,
                                          const double* bcb, int Bp, NodeLoads<T, NO>& L) {
    int cds[N_SLOTS];   // all codes first: one batch of scalar loads per node
#pragma unroll
    for (int t = 0; t < N_SLOTS; ++t) cds[t] = code[t];
#pragma unroll
    for (int t = 0; t < N_SLOTS; ++t) {
        const int cd = cds[t];
        L.kind[t] = src_kind(cd);
        const int idx = src_index(cd);
        // FP64, or up to 12 latents (every lane keeps all its sums in registers): a branch-free
        // gather, every slot reads a value and NO Jacobian entries (a boundary slot an all-zero
        // block, its value from the Dirichlet buffer); measured faster there than the scalar
        // branches below, which add registers
        if constexpr (sizeof(T) == 8 || NO + NG <= 12) {
            const T* base = L.kind[t] == SRC_OMEGA ? dom + (size_t)idx * (1 + NO) * Bp
                          : (L.kind[t] == SRC_GAMMA ? dga + (size_t)idx * (1 + NG) * Bp : dz);
            const double bv = bcb[(size_t)(L.kind[t] == SRC_BOUND ? idx : 0) * Bp];
            const T dv = base[0];
            L.v[t] = L.kind[t] == SRC_BOUND ? bv : (double)dv;
#pragma unroll
            for (int k = 0; k < NO; ++k) L.jv[t][k] = base[(size_t)(1 + k) * Bp];
            continue;
        }
        // the kind is wave-uniform, so these are scalar branches: a boundary slot reads only its
        // Dirichlet value, an interface slot only its NG Jacobian entries
        if (L.kind[t] == SRC_BOUND) {
            L.v[t] = bcb[(size_t)idx * Bp];
        } else if (L.kind[t] == SRC_OMEGA) {
            const T* base = dom + (size_t)idx * (1 + NO) * Bp;
            L.v[t] = (double)base[0];
#pragma unroll
            for (int k = 0; k < NO; ++k) L.jv[t][k] = base[(size_t)(1 + k) * Bp];
        } else {
            const T* base = dga + (size_t)idx * (1 + NG) * Bp;
            L.v[t] = (double)base[0];
#pragma unroll
            for (int k = 0; k < NG; ++k) L.jv[t][k] = base[(size_t)(1 + k) * Bp];
        }
    }
}

template <typename T, int NO, int NG>
__device__ __forceinline__ void node_z(const NodeLoads<T, NO>& L, double nu, double hx, double hy, double* zu,
                                       double* zv, double& ru, double& rv) {
    constexpr int NN = NO + NG;
    double cu[6], cv[6];
    burgers_point(L.v, nu, hx, hy, ru, rv, cu, cv);
#pragma unroll
    for (int e = 0; e < NN; ++e) { zu[e] = 0.0; zv[e] = 0.0; }
    // a u slot feeds d r_u only, a v slot d r_v only, except the two centre slots, which also
    // feed the other field's equation (the advection cross terms); zero products are skipped
#pragma unroll
    for (int t = 0; t < N_SLOTS; ++t) {
        const bool us = t < 5;
        const double a = us ? cu[t] : cv[t - 5];
        const bool cross = t == S_UC || t == S_VC;
        const double ac = t == S_UC ? cv[5] : cu[5];
        // the kind is wave-uniform: scalar branches, all loads already issued
        if (L.kind[t] == SRC_OMEGA) {
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                const double jk = (double)L.jv[t][k];
                if (us) zu[k] = fma(a, jk, zu[k]); else zv[k] = fma(a, jk, zv[k]);
                if (cross) { if (us) zv[k] = fma(ac, jk, zv[k]); else zu[k] = fma(ac, jk, zu[k]); }
            }
        } else if (L.kind[t] == SRC_GAMMA) {
#pragma unroll
            for (int k = 0; k < NG; ++k) {
                const double jk = (double)L.jv[t][k];
                if (us) zu[NO + k] = fma(a, jk, zu[NO + k]); else zv[NO + k] = fma(a, jk, zv[NO + k]);
                if (cross) {
                    if (us) zv[NO + k] = fma(ac, jk, zv[NO + k]); else zu[NO + k] = fma(ac, jk, zu[NO + k]);
                }
            }
        }
    }
}

// Gauss-Newton entries of one node, in packed order: H (upper triangle, row by row), g, rr.
// Entry e of part P (of 4) lives in acc[e - lo(P)]; the part's range is fixed at compile time,
// so each wave of the residual kernel keeps only its quarter of the sums in registers.  z is
// read from LDS ([2 NN + 2][64] doubles: z_u, z_v, r_u, r_v); reads the part does not use are
// dropped by the compiler.
template <int NN>
struct GnEntries {
    static constexpr int NH = NN * (NN + 1) / 2;
    static constexpr int NE = NH + NN + 1;
    static constexpr int lo(int P) { return NE * P / 4; }
    static constexpr int hi(int P) { return NE * (P + 1) / 4; }
    static constexpr int MAXP = (NE + 3) / 4;
};

template <int NN, int P>
__device__ __forceinline__ void gram_part(const double* zl, int lane, double* acc) {
    using G = GnEntries<NN>;
    constexpr int lo = G::lo(P), hi = G::hi(P);
    double zu[NN], zv[NN];
#pragma unroll
    for (int i = 0; i < NN; ++i) {
        zu[i] = zl[i * 64 + lane];
        zv[i] = zl[(NN + i) * 64 + lane];
    }
    const double ru = zl[2 * NN * 64 + lane], rv = zl[(2 * NN + 1) * 64 + lane];
    int e = 0;
#pragma unroll
    for (int i = 0; i < NN; ++i)
#pragma unroll
        for (int j = i; j < NN; ++j, ++e)
            if (e >= lo && e < hi) acc[e - lo] = fma(zv[i], zv[j], fma(zu[i], zu[j], acc[e - lo]));
#pragma unroll
    for (int i = 0; i < NN; ++i, ++e)
        if (e >= lo && e < hi) acc[e - lo] = fma(zv[i], rv, fma(zu[i], ru, acc[e - lo]));
    if (e >= lo && e < hi) acc[e - lo] = fma(rv, rv, fma(ru, ru, acc[e - lo]));
}


// One workgroup = a run of sampled nodes of one subdomain x 64 solve slots (lanes).  For each node
// the ten stencil DoFs are gathered, the pointwise residual and the chain-rule vectors z_u, z_v
// (Z R_i at that node) formed, and the Gauss-Newton entries (H_i upper triangle, g_i, r^T r) summed
// over the run.  Every solve's sums are formed in the same order whatever the batch.  Two layouts:
//
//  * up to 12 latents per subdomain, every lane keeps all entries in registers; the four waves
//    take consecutive quarters of the run and are combined in LDS in a fixed order;
//  * above 12 (whose entries do not fit beside the gather), the run is taken four nodes at a
//    time: each wave gathers one node and puts z_u, z_v, r_u, r_v in LDS, then each wave adds the
//    four nodes, in node order, into its fixed quarter of the entries, which it writes out itself.
template <typename T, int NO, int NG>
__global__ __launch_bounds__(256) void k_res_gn(const ResChunk* __restrict__ rchunks, int rbase,
                                                const ResSeg* __restrict__ rsegs, const DecSeg* __restrict__ segs,
                                                const int* __restrict__ gather, const T* __restrict__ dec,
                                                const double* __restrict__ bc, const int* __restrict__ live,
                                                const int* __restrict__ n_live, int B, int Bp, double nu, double hx,
                                                double hy, double* __restrict__ part, int estride,
                                                long long zero_row) {
    constexpr int NN = NO + NG;
    using G = GnEntries<NN>;
    const int nl = live_count(n_live, B);
    const int j0 = blockIdx.y * 64;
    if (j0 >= nl) return;
    const ResChunk rc = rchunks[rbase + xcd_item()];
    const ResSeg rs = rsegs[rc.sd];
    const long long oo = segs[rs.seg_om].out, og = segs[rs.seg_ga].out;
    // the wave index is uniform: node codes come in by scalar loads and the source-kind
    // branches are scalar, so a node's gathers are issued without waiting
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = j0 + lane;
    const T* dom = dec + (size_t)oo * Bp + j;
    const T* dga = dec + (size_t)og * Bp + j;
    const T* dz = dec + (size_t)zero_row * Bp + j;
    const double* bcb = bc + slot_solve(live, j, nl);   // Dirichlet data are per solve
    const int* gp = gather + rs.gather;
    double* pp = part + (size_t)rc.slot * estride * Bp + j;
    if constexpr (NN <= 12) {
        constexpr int CH = 16;
        __shared__ double red[3][CH][64];
        const int np = rc.p1 - rc.p0;
        const int pb = rc.p0 + np * w / 4, pe = rc.p0 + np * (w + 1) / 4;
        double H[G::NH], g[NN], rr = 0.0;
#pragma unroll
        for (int e = 0; e < G::NH; ++e) H[e] = 0.0;
#pragma unroll
        for (int e = 0; e < NN; ++e) g[e] = 0.0;
        for (int p = pb; p < pe; ++p) {
            NodeLoads<T, NO> A;
            load_node<T, NO, NG>(gp + (size_t)p * N_SLOTS, dom, dga, dz, bcb, Bp, A);
            double zu[NN], zv[NN], ru, rv;
            node_z<T, NO, NG>(A, nu, hx, hy, zu, zv, ru, rv);
            int e = 0;
#pragma unroll
            for (int i = 0; i < NN; ++i) {
                g[i] = fma(zv[i], rv, fma(zu[i], ru, g[i]));
#pragma unroll
                for (int k = i; k < NN; ++k, ++e) H[e] = fma(zv[i], zv[k], fma(zu[i], zu[k], H[e]));
            }
            rr = fma(rv, rv, fma(ru, ru, rr));
        }
        auto val = [&](int e) { return e < G::NH ? H[e] : (e < G::NH + NN ? g[e - G::NH] : rr); };
#pragma unroll
        for (int c0 = 0; c0 < G::NE; c0 += CH) {
            if (w > 0)
#pragma unroll
                for (int e = c0; e < c0 + CH && e < G::NE; ++e) red[w - 1][e - c0][lane] = val(e);
            __syncthreads();
            if (w == 0)
#pragma unroll
                for (int e = c0; e < c0 + CH && e < G::NE; ++e)
                    pp[(size_t)e * Bp] = ((val(e) + red[0][e - c0][lane]) + red[1][e - c0][lane]) + red[2][e - c0][lane];
            __syncthreads();
        }
    } else {
        constexpr int NZ = 2 * NN + 2;
        __shared__ double zs[4][NZ][64];
        double acc[G::MAXP];
#pragma unroll
        for (int e = 0; e < G::MAXP; ++e) acc[e] = 0.0;
        for (int p0 = rc.p0; p0 < rc.p1; p0 += 4) {
            const int p = p0 + w;
            double zu[NN], zv[NN], ru = 0.0, rv = 0.0;
            if (p < rc.p1) {
                NodeLoads<T, NO> A;
                load_node<T, NO, NG>(gp + (size_t)p * N_SLOTS, dom, dga, dz, bcb, Bp, A);
                node_z<T, NO, NG>(A, nu, hx, hy, zu, zv, ru, rv);
            } else {
#pragma unroll
                for (int i = 0; i < NN; ++i) { zu[i] = 0.0; zv[i] = 0.0; }
            }
#pragma unroll
            for (int i = 0; i < NN; ++i) {
                zs[w][i][lane] = zu[i];
                zs[w][NN + i][lane] = zv[i];
            }
            zs[w][2 * NN][lane] = ru;
            zs[w][2 * NN + 1][lane] = rv;
            __syncthreads();
            const int nq = min(4, rc.p1 - p0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q >= nq) break;
                if (w == 0) gram_part<NN, 0>(&zs[q][0][0], lane, acc);
                else if (w == 1) gram_part<NN, 1>(&zs[q][0][0], lane, acc);
                else if (w == 2) gram_part<NN, 2>(&zs[q][0][0], lane, acc);
                else gram_part<NN, 3>(&zs[q][0][0], lane, acc);
            }
            __syncthreads();
        }
        const int lo = w == 0 ? G::lo(0) : (w == 1 ? G::lo(1) : (w == 2 ? G::lo(2) : G::lo(3)));
        const int hi = w == 0 ? G::hi(0) : (w == 1 ? G::hi(1) : (w == 2 ? G::hi(2) : G::hi(3)));
#pragma unroll
        for (int e = 0; e < G::MAXP; ++e)
            if (lo + e < hi) pp[(size_t)(lo + e) * Bp] = acc[e];
    }
}

// ------------------------------------------------------------------------------------
// Gappy-POD hyper-reduction (Section 3.1): the objective takes B_i r_i with
// B_i = (Z_i Phi_i^r)^+ Z_i = P_i Z_i, so the Gauss-Newton sums are those of the projected rows
// Y_i = P_i [Z_i r_i | Z_i R_i]: H_i = sum_j y_j' y_j'^T, g_i = sum_j y_j' y_j0, rr = sum_j y_j0^2
// over the modes j (y_j0 the projected residual, y_j' its latent gradient).  Three passes:
//  k_res_rows  the sampled rows and their gradients by the same stencil code as k_res_gn, stored;
//  k_gappy_y   Y = P R, one workgroup per (subdomain, 8 modes) and 64-solve group;
//  k_gappy_gn  the sums over the modes into the subdomain's partial slot.
// ------------------------------------------------------------------------------------
template <typename T, int NO, int NG>
__global__ __launch_bounds__(256) void k_res_rows(const ResChunk* __restrict__ rchunks, int rbase,
                                                  const ResSeg* __restrict__ rsegs, const DecSeg* __restrict__ segs,
                                                  const GappySeg* __restrict__ gsegs, const int* __restrict__ gather,
                                                  const T* __restrict__ dec, const double* __restrict__ bc,
                                                  const int* __restrict__ live, const int* __restrict__ n_live, int B,
                                                  int Bp, double nu, double hx, double hy, double* __restrict__ R,
                                                  long long zero_row) {
    constexpr int NN = NO + NG;
    const int nl = live_count(n_live, B);
    const int j0 = blockIdx.y * 64;
    if (j0 >= nl) return;
    const ResChunk rc = rchunks[rbase + xcd_item()];
    const ResSeg rs = rsegs[rc.sd];
    const GappySeg gs = gsegs[rc.sd];
    const long long oo = segs[rs.seg_om].out, og = segs[rs.seg_ga].out;
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = j0 + lane;
    const T* dom = dec + (size_t)oo * Bp + j;
    const T* dga = dec + (size_t)og * Bp + j;
    const T* dz = dec + (size_t)zero_row * Bp + j;
    const double* bcb = bc + slot_solve(live, j, nl);
    const int* gp = gather + rs.gather;
    double* Rs = R + (size_t)gs.r_off * Bp + j;
    for (int p = rc.p0 + w; p < rc.p1; p += 4) {
        NodeLoads<T, NO> A;
        load_node<T, NO, NG>(gp + (size_t)p * N_SLOTS, dom, dga, dz, bcb, Bp, A);
        double zu[NN], zv[NN], ru, rv;
        node_z<T, NO, NG>(A, nu, hx, hy, zu, zv, ru, rv);
        double* qu = Rs + (size_t)p * (NN + 1) * Bp;
        double* qv = Rs + (size_t)(gs.nb + p) * (NN + 1) * Bp;
        qu[0] = ru;
        qv[0] = rv;
#pragma unroll
        for (int i = 0; i < NN; ++i) {
            qu[(size_t)(1 + i) * Bp] = zu[i];
            qv[(size_t)(1 + i) * Bp] = zv[i];
        }
    }
}

// Y[j][k][b] = sum_rows P[j][row] R[row][k][b]: the four waves take k = w, w + 4, ...; the
// row sum runs in row order (the same for every solve and batch).
__global__ __launch_bounds__(256) void k_gappy_y(const int2* __restrict__ items, const GappySeg* __restrict__ gsegs,
                                                 const double* __restrict__ P, const double* __restrict__ R,
                                                 double* __restrict__ Y, const int* __restrict__ n_live, int B,
                                                 int Bp) {
    // One work item: modes q0 .. q0 + kGappyModes - 1 of one subdomain for 64 solves.  The
    // operator rows are staged in LDS transposed ([row][mode]), kGappyRowChunk rows at a time;
    // wave w takes the columns k = w, w + 4, ... of the stored rows (value, then one gradient
    // per latent), so each stored row is read once for all of the item's modes.  Every Y entry
    // is the sum over rows in ascending order.
    constexpr int MT = kGappyModes, KW = 4;     // KW: columns per wave (nn + 1 <= 13 over 4 waves)
    __shared__ __align__(16) double sP[kGappyRowChunk * MT];
    const int nl = live_count(n_live, B);
    const int j0 = blockIdx.y * 64;
    if (j0 >= nl) return;
    const int2 it = items[xcd_item()];
    const GappySeg gs = gsegs[it.x];
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = j0 + lane;
    const int nm = min(MT, gs.modes - it.y);
    const double* Pq = P + gs.p_off + (size_t)it.y * gs.rows;
    const size_t rstride = (size_t)(gs.nn + 1) * Bp;
    const double* Rb = R + (size_t)gs.r_off * Bp + j;
    double acc[KW][MT];
#pragma unroll
    for (int c = 0; c < KW; ++c)
#pragma unroll
        for (int q = 0; q < MT; ++q) acc[c][q] = 0.0;
    const int nk = (gs.nn + 1 - w + 3) / 4;    // columns of this wave (wave-uniform)
    for (int r0 = 0; r0 < gs.rows; r0 += kGappyRowChunk) {
        const int nr = min(kGappyRowChunk, gs.rows - r0);
        __syncthreads();     // the previous chunk has been read
        for (int i = tid; i < nr * MT; i += 256) {
            const int row = i / MT, q = i % MT;
            sP[i] = q < nm ? Pq[(size_t)q * gs.rows + r0 + row] : 0.0;
        }
        __syncthreads();
        // U rows per step: their loads are all issued before the products, so a wave keeps up
        // to U * KW loads in flight (one workgroup per CU leaves little else to hide latency)
        constexpr int U = 8;
        for (int row = 0; row < nr; row += U) {
            double rv[U][KW];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double* Rr = Rb + (size_t)(r0 + row + u) * rstride;
#pragma unroll
                for (int c = 0; c < KW; ++c) rv[u][c] = (row + u < nr && c < nk) ? Rr[(size_t)(w + 4 * c) * Bp] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (row + u >= nr) break;
                const double* pr = sP + (row + u) * MT;
                double pv[MT];
#pragma unroll
                for (int q = 0; q < MT; ++q) pv[q] = pr[q];
#pragma unroll
                for (int c = 0; c < KW; ++c)
                    if (c < nk)
#pragma unroll
                        for (int q = 0; q < MT; ++q) acc[c][q] = fma(pv[q], rv[u][c], acc[c][q]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < KW; ++c) {
        if (c >= nk) continue;
        const int k = w + 4 * c;
#pragma unroll
        for (int q = 0; q < MT; ++q)
            if (q < nm) Y[((size_t)gs.y_off + (size_t)(it.y + q) * (gs.nn + 1) + k) * Bp + j] = acc[c][q];
    }
}

// Gauss-Newton sums of one subdomain's projected rows (one wave, 64 solves), written to the
// subdomain's partial slot (slot sd) in the layout k_res_gn uses (H upper triangle row by row,
// g, rr).  Subdomain blockIdx.x; subdomains with another latent size are left to the launch
// of their NN.
template <int NN>
__global__ __launch_bounds__(64) void k_gappy_gn(const GappySeg* __restrict__ gsegs, const double* __restrict__ Y,
                                                 const int* __restrict__ n_live, int B, int Bp,
                                                 double* __restrict__ part, int estride) {
    using G = GnEntries<NN>;
    const int nl = live_count(n_live, B);
    const int j0 = blockIdx.y * 64;
    if (j0 >= nl) return;
    const int sd = blockIdx.x, slot = sd;
    const GappySeg gs = gsegs[sd];
    if (gs.nn != NN) return;
    const int j = j0 + (int)threadIdx.x;
    double H[G::NH], g[NN], rr = 0.0;
#pragma unroll
    for (int e = 0; e < G::NH; ++e) H[e] = 0.0;
#pragma unroll
    for (int e = 0; e < NN; ++e) g[e] = 0.0;
    for (int q = 0; q < gs.modes; ++q) {
        const double* y = Y + ((size_t)gs.y_off + (size_t)q * (NN + 1)) * Bp + j;
        double v[NN + 1];
#pragma unroll
        for (int k = 0; k <= NN; ++k) v[k] = y[(size_t)k * Bp];
        rr = fma(v[0], v[0], rr);
        int e = 0;
#pragma unroll
        for (int i = 0; i < NN; ++i) {
            g[i] = fma(v[1 + i], v[0], g[i]);
#pragma unroll
            for (int k = i; k < NN; ++k, ++e) H[e] = fma(v[1 + i], v[1 + k], H[e]);
        }
    }
    double* pp = part + (size_t)slot * estride * Bp + j;
#pragma unroll
    for (int e = 0; e < G::NH; ++e) pp[(size_t)e * Bp] = H[e];
#pragma unroll
    for (int i = 0; i < NN; ++i) pp[(size_t)(G::NH + i) * Bp] = g[i];
    pp[(size_t)(G::NH + NN) * Bp] = rr;
}

// ------------------------------------------------------------------------------------
// Weak compatibility constraint: c_i = C A_i g_i^Gamma, E_i^Gamma = C A_i dg_i^Gamma/dxhat
// ------------------------------------------------------------------------------------
// One workgroup = (subdomain, 8 constraint rows, a run of interface rows) x 64 solve slots.
// Its four waves take consecutive quarters of the row run (short dependent chains, also when
// few solves run) and their sums are combined in LDS in a fixed order, so every solve's sums
// are formed the same way whatever the batch.  (C A_i)^T is stored row-major with stride ca_ld
// so the 8 multipliers of an interface row are one contiguous scalar load.  Partial sums over
// interface-row runs go to separate slots.
template <typename T, int NG>
__global__ __launch_bounds__(256) void k_con(const ConChunk* __restrict__ cch, int chunk_base,
                                             const ResSeg* __restrict__ rsegs,
                                             const DecSeg* __restrict__ segs, const double* __restrict__ CA, int n_C,
                                             int ca_ld, const T* __restrict__ dec, const int* __restrict__ n_live,
                                             int B, int Bp, double* __restrict__ c_part, double* __restrict__ E_part,
                                             int mmax) {
    constexpr int JB = 8;
    constexpr int NE = JB * (1 + NG);
    constexpr int CH = 16;
    __shared__ double red[3][CH][64];
    const int item = xcd_item(), grp = blockIdx.y;
    const ConChunk cc = cch[chunk_base + item];
    const ResSeg rs = rsegs[cc.sd];
    if (grp * 64 >= live_count(n_live, B)) return;
    const int tid = threadIdx.x, lane = tid & 63, prt = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b = grp * 64 + lane;   // slot
    const T* dga = dec + (size_t)segs[rs.seg_ga].out * Bp + b;
    const double* ca = CA + rs.ca + cc.j0;
    const int nj = cc.j1 - cc.j0;
    const int no = cc.o1 - cc.o0;
    const int ob = cc.o0 + no * prt / 4, oe = cc.o0 + no * (prt + 1) / 4;
    double c[JB], E[JB][NG];
#pragma unroll
    for (int j = 0; j < JB; ++j) {
        c[j] = 0.0;
#pragma unroll
        for (int k = 0; k < NG; ++k) E[j][k] = 0.0;
    }
#pragma unroll 2
    for (int o = ob; o < oe; ++o) {
        const T* row = dga + (size_t)o * (1 + NG) * Bp;
        const double x = (double)row[0];
        double J[NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) J[k] = (double)row[(size_t)(1 + k) * Bp];
        const double* a = ca + (size_t)o * ca_ld;
#pragma unroll
        for (int j = 0; j < JB; ++j) {
            const double aj = a[j];     // slots j >= nj hold zeros (padding of ca_ld) or are discarded
            c[j] += aj * x;
#pragma unroll
            for (int k = 0; k < NG; ++k) E[j][k] += aj * J[k];
        }
    }
    // entry e < JB is c[e]; entry JB + j * NG + k is E[j][k]
    auto val = [&](int e) { return e < JB ? c[e] : E[(e - JB) / NG][(e - JB) % NG]; };
#pragma unroll
    for (int c0 = 0; c0 < NE; c0 += CH) {
        if (prt > 0)
#pragma unroll
            for (int e = c0; e < c0 + CH && e < NE; ++e) red[prt - 1][e - c0][lane] = val(e);
        __syncthreads();
        if (prt == 0)
#pragma unroll
            for (int e = c0; e < c0 + CH && e < NE; ++e) {
                const int j = e < JB ? e : (e - JB) / NG;
                if (j < nj) {
                    const double v = ((val(e) + red[0][e - c0][lane]) + red[1][e - c0][lane]) + red[2][e - c0][lane];
                    const int jj = cc.j0 + j;
                    if (e < JB) c_part[((size_t)cc.part * n_C + jj) * Bp + b] = v;
                    else E_part[(((size_t)cc.part * n_C + jj) * mmax + (e - JB) % NG) * Bp + b] = v;
                }
            }
        __syncthreads();
    }
}

// Strong ROM-port constraint (eq. rom_strong_constraint): subdomain sd's share Ahat_sd xhat_sd^Gamma
// of the constraint at the trial latents and its constant Jacobian block Ahat_sd, written in the
// partial-sum layout the reduction reads (one part per subdomain).  One lane per solve slot.
__global__ __launch_bounds__(64) void k_con_linear(const double* __restrict__ Ahat, int n_C, int mmax,
                                                   const int* __restrict__ n_om, const int* __restrict__ n_ga,
                                                   const int* __restrict__ xoff, const double* __restrict__ xhat,
                                                   int xstride, const int* __restrict__ live,
                                                   const int* __restrict__ n_live, int B, int Bp,
                                                   double* __restrict__ c_part, double* __restrict__ E_part) {
    constexpr int MX = 12;      // n_i^Gamma bound of the update kernel
    const int sd = blockIdx.x;
    const int nl = live_count(n_live, B);
    if ((int)blockIdx.y * 64 >= nl) return;
    const int j = blockIdx.y * 64 + threadIdx.x;     // slot
    const bool act = j < nl;
    const int b = slot_solve(live, j, nl);
    const int m = n_ga[sd], o = xoff[sd] + n_om[sd];
    const double* A = Ahat + (size_t)sd * n_C * mmax;
    double x[MX];
#pragma unroll
    for (int k = 0; k < MX; ++k) x[k] = (act && k < m) ? xhat[(size_t)b * xstride + o + k] : 0.0;
    for (int r = 0; r < n_C; ++r) {
        const double* a = A + (size_t)r * mmax;
        double c = 0.0;
#pragma unroll
        for (int k = 0; k < MX; ++k)
            if (k < m) c += a[k] * x[k];
        c_part[((size_t)sd * n_C + r) * Bp + j] = c;
        for (int k = 0; k < mmax; ++k) E_part[(((size_t)sd * n_C + r) * mmax + k) * Bp + j] = k < m ? a[k] : 0.0;
    }
}

// ------------------------------------------------------------------------------------
// Sum of the partial slots into one contiguous block per solve
// ------------------------------------------------------------------------------------
// Lanes are solve slots, so the partial sums are read coalesced.  The four waves of a
// workgroup take every fourth partial slot (short dependent chains when few solves run) and
// their sums are combined in LDS in a fixed order; a 16-entry LDS tile is then written out
// transposed, so that each slot's block [H packed | g | rr | E] per subdomain, followed by c,
// is contiguous for the update kernel.
constexpr int RED_E = 16;
__global__ __launch_bounds__(256) void k_reduce(int n_sub, int n_C, int mmax, int estride, int rs, int RS, int Bp,
                                                int B, const int* __restrict__ n_om, const int* __restrict__ n_ga,
                                                const int* __restrict__ slot0, const int* __restrict__ cpart0,
                                                int n_cparts, const double* __restrict__ gn_part,
                                                const double* __restrict__ c_part, const double* __restrict__ E_part,
                                                const int* __restrict__ n_live, double* __restrict__ RB) {
    __shared__ double wpart[3][RED_E][64];
    __shared__ double tile[RED_E][65];
    const int sd = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b0 = blockIdx.z * 64, b = b0 + lane;   // slots
    if (b0 >= live_count(n_live, B)) return;
    int n_e, ne_gn = 0, ng = 0;
    size_t dst0;
    if (sd < n_sub) {
        const int NN = n_om[sd] + n_ga[sd];
        ne_gn = NN * (NN + 1) / 2 + NN + 1;
        ng = n_ga[sd];
        n_e = estride + n_C * mmax;
        dst0 = (size_t)sd * rs;
    } else {
        n_e = n_C;
        dst0 = (size_t)n_sub * rs;
    }
    const int e0 = blockIdx.y * RED_E;
    if (e0 >= n_e) return;
    const int cnt = min(RED_E, n_e - e0);
    // loads are unconditional (indices clamped into the buffer) and masked afterwards, so
    // every load of a slot is in flight before any add waits
    double acc[RED_E];
#pragma unroll
    for (int j = 0; j < RED_E; ++j) acc[j] = 0.0;
    if (sd < n_sub) {
        if (e0 < estride) {
            for (int sl = slot0[sd] + wave; sl < slot0[sd + 1]; sl += 4) {
                const double* src = gn_part + (size_t)sl * estride * Bp + b;
                double v[RED_E];
#pragma unroll
                for (int j = 0; j < RED_E; ++j) v[j] = src[(size_t)min(e0 + j, estride - 1) * Bp];
#pragma unroll
                for (int j = 0; j < RED_E; ++j) acc[j] += (e0 + j < ne_gn) ? v[j] : 0.0;
            }
        }
        if (e0 + RED_E > estride) {
            for (int p = cpart0[sd] + wave; p < cpart0[sd + 1]; p += 4) {
                const double* src = E_part + (size_t)p * n_C * mmax * Bp + b;
                double v[RED_E];
#pragma unroll
                for (int j = 0; j < RED_E; ++j) {
                    const int q = min(max(e0 + j - estride, 0), n_C * mmax - 1);
                    v[j] = src[(size_t)q * Bp];
                }
#pragma unroll
                for (int j = 0; j < RED_E; ++j) {
                    const int q = e0 + j - estride;
                    acc[j] += (q >= 0 && q < n_C * mmax && (q % mmax) < ng) ? v[j] : 0.0;
                }
            }
        }
    } else {
        for (int p = wave; p < n_cparts; p += 4) {
            const double* src = c_part + (size_t)p * n_C * Bp + b;
            double v[RED_E];
#pragma unroll
            for (int j = 0; j < RED_E; ++j) v[j] = src[(size_t)min(e0 + j, n_C - 1) * Bp];
#pragma unroll
            for (int j = 0; j < RED_E; ++j) acc[j] += (e0 + j < n_C) ? v[j] : 0.0;
        }
    }
    if (wave > 0)
#pragma unroll
        for (int j = 0; j < RED_E; ++j) wpart[wave - 1][j][lane] = acc[j];
    __syncthreads();
    if (wave == 0)
#pragma unroll
        for (int j = 0; j < RED_E; ++j) tile[j][lane] = ((acc[j] + wpart[0][j][lane]) + wpart[1][j][lane]) + wpart[2][j][lane];
    __syncthreads();
    for (int q = tid; q < 64 * RED_E; q += 256) {
        const int sv = q / RED_E, j = q % RED_E;
        if (j < cnt) RB[(size_t)(b0 + sv) * RS + dst0 + e0 + j] = tile[j][sv];
    }
}

struct UpdArgs {
    int n_sub, n_C, n_D, mg, estride, Bp, B;   // mg = max(1, largest n_i^Gamma): stride of the E blocks
    int lam_given;
    int max_iter, max_bt;
    double tol_abs, tol_rel, c1, stall_tol, stall_ratio;
    const int* n_om;       // [n_sub]
    const int* n_ga;
    const int* xoff;
    const double* RB;      // per-slot reduced blocks [Bp][RS]
    int rs, RS;
    double* x;
    double* xt;
    double* lam;
    double* lamt;
    double* step;
    SolveState* st;
    const int* live;       // slot -> solve
    const int* n_live;
    double* gscr;          // per-slot scratch of the big KKT arrays when they exceed LDS
    long long gstride;
    int sdc;               // subdomains per LDS-staged chunk of the Schur assembly (0: not staged)
    int stage_off;         // LDS offset (doubles) of the staging area
};

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Value of v held by lane l (l wave-uniform).
__device__ __forceinline__ double lane_bcast(double v, int l) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)u, l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int packed_idx(int i, int j, int n) {   // i <= j, upper triangle row-major
    return i * n - i * (i - 1) / 2 + (j - i);
}

// LDS layout of the update kernel (offsets in doubles).
// Memory of the update kernel (offsets in doubles): a small part always in LDS, and the
// per-subdomain blocks and the Schur system, in LDS when they fit beside it (GB = 0), else in
// a per-slot area of global scratch, the Schur system kept in LDS while it fits (GB = 1) or
// in the scratch too (GB = 2).
struct UpdLds {
    int lam, c, sl, red, u, small;   // small part: lam [nC], c [nC], s_lambda [nC], reduction [16],
                                     // Ehat_i^T v per subdomain [n_sub][mg]
    int E, P, q, rho, X, S, big;     // big part, relative to its base
};
__host__ __device__ inline UpdLds upd_lds(int n_sub, int nC, int mg, int NN, int MG) {
    UpdLds L;
    const int nc = nC > 0 ? nC : 1;
    L.lam = 0;
    L.c = L.lam + nc;
    L.sl = L.c + nc;
    L.red = L.sl + nc;
    L.u = L.red + 16;
    L.small = L.u + n_sub * mg;
    L.E = 0;                                 // [n_sub][nC][mg]  Ehat_i
    L.P = L.E + n_sub * nC * mg;             // [n_sub][nC][mg]  Ehat_i (W_i)_Gamma
    L.q = L.P + n_sub * nC * mg;             // [n_sub][nC]      Ehat_i (t_i)_Gamma
    L.rho = L.q + n_sub * nC;                // [n_sub][NN]      rho_i
    L.X = L.rho + n_sub * NN;                // [n_sub][NN][MG+1]  [W_i | t_i]
    L.S = L.X + n_sub * NN * (MG + 1);       // [nC][nC+1]       [S | right-hand side]
    L.big = L.S + nC * (nC + 1);
    return L;
}
constexpr int UPD_LDS_DOUBLES = 8192;        // 64 KiB: everything in LDS up to this size
constexpr int UPD_LDS_MAX_DOUBLES = 19968;   // 156 KiB of the 160 KiB a workgroup may hold

// One wave's Gauss-Jordan elimination without pivoting of a symmetric positive definite n x n
// system held row-per-lane in registers (n <= 64; lanes >= n are ignored).  At step k every
// other row subtracts its multiple of row k, both below and above the diagonal, so no back
// substitution is needed: the solution is r / pivot.  Each row is shifted left by one register
// per step, so the current column is always row[0] and every register index is static; the
// right-hand sides (NR of them) stay in place.  ok is cleared when a pivot is not positive or
// not finite.  On return r[l] holds the solution for this lane's row.
template <int NC, int NR>
__device__ __forceinline__ void wave_gj(double (&row)[NC], double (&r)[NR], int n, int lane, bool& ok) {
    double diag = 1.0;
    for (int k = 0; k < n; ++k) {
        const double rk = row[0];
        const double pv = lane_bcast(rk, k);
        if (!(pv > 0.0) || !isfinite(pv)) ok = false;
        const double rp = 1.0 / pv;
        const double f = (lane != k && lane < n) ? rk * rp : 0.0;
        if (lane == k) diag = rk;
#pragma unroll
        for (int c = 1; c < NC; ++c) row[c - 1] = row[c] - f * lane_bcast(row[c], k);
        row[NC - 1] = 0.0;
#pragma unroll
        for (int l = 0; l < NR; ++l) r[l] -= f * lane_bcast(r[l], k);
    }
    const double rd = 1.0 / diag;
#pragma unroll
    for (int l = 0; l < NR; ++l) r[l] = lane < n ? r[l] * rd : 0.0;
}

// Symmetric positive definite n x n system [M | r] (LDS, row stride n + 1: the Schur complement of
// the KKT matrix, or the normal equations of the initial multiplier) solved by one wave with
// wave_gj; the solution goes to x (LDS).  Returns false if a pivot is not positive (the matrix is
// not positive definite) or not finite.
template <int NCP>
__device__ bool wave_spd_reg(const double* M, int n, double* x, int lane) {
    const int ld = n + 1;
    double row[NCP], r[1];
#pragma unroll
    for (int c = 0; c < NCP; ++c) row[c] = (lane < n && c < n) ? M[lane * ld + c] : 0.0;
    r[0] = lane < n ? M[lane * ld + n] : 0.0;
    bool ok = true;
    wave_gj<NCP, 1>(row, r, n, lane, ok);
    if (lane < n) x[lane] = r[0];
    return ok;
}

__device__ bool wave_spd_solve(const double* M, int n, double* x, int lane) {
    if (n <= 8) return wave_spd_reg<8>(M, n, x, lane);
    if (n <= 16) return wave_spd_reg<16>(M, n, x, lane);
    if (n <= 32) return wave_spd_reg<32>(M, n, x, lane);
    return wave_spd_reg<64>(M, n, x, lane);
}

// Symmetric positive definite systems larger than a wave (64 < n <= 256), M in LDS or global
// memory: elimination without pivoting over the whole workgroup, rows over waves and columns
// over lanes with the pivot row in registers, one barrier per step; wave 0 then back-substitutes
// alone (positions in its lanes, no barriers).  x (LDS) receives the solution; okf: LDS flag.
// Every thread returns the same value.
__device__ bool block_lu_solve(double* M, int n, double* x, int* okf, int tid, int nth) {
    const int ld = n + 1, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), nw = nth >> 6;
    if (tid == 0) okf[0] = 1;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double pv = M[(size_t)k * ld + k];
        if (!(pv > 0.0) || !isfinite(pv)) {
            if (tid == 0) okf[0] = 0;
        } else {
            const double rp = 1.0 / pv;
            double prow[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int j = k + 1 + lane + 64 * c;
                prow[c] = j <= n ? M[(size_t)k * ld + j] : 0.0;
            }
            for (int i = k + 1 + wave; i < n; i += nw) {
                const double f = M[(size_t)i * ld + k] * rp;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int j = k + 1 + lane + 64 * c;
                    if (j <= n) M[(size_t)i * ld + j] -= f * prow[c];
                }
            }
        }
        __syncthreads();
    }
    const bool ok = okf[0] != 0;
    if (wave == 0 && ok) {
        double rhs[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int q = lane + 64 * t;
            rhs[t] = q < n ? M[(size_t)q * ld + n] : 0.0;
        }
        for (int i = n - 1; i >= 0; --i) {
            const int slot = i >> 6;
            double ri = 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t == slot) ri = rhs[t];
            const double xi = lane_bcast(ri, i & 63) / M[(size_t)i * ld + i];
            if (lane == 0) x[i] = xi;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int q = lane + 64 * t;
                if (q < i) rhs[t] -= M[(size_t)q * ld + i] * xi;
            }
        }
    }
    __syncthreads();
    return ok;
}

// S[i][j] = sum over subdomains sd and l < mg of A[sd][i][l] Bm[sd][j][l] for i, j < nC, written
// to S with row stride ld; A and Bm are [ns][nC][mg] with subdomain strides sdsA, sdsB.  Each thread
// accumulates a T x T block in registers (2T loads per T^2 FMAs), subdomains in ascending
// order, so every entry is the same fixed-order sum whatever the block size or thread count.
template <int T, int MG>
__device__ void gram_sum_t(const double* A, size_t sdsA, const double* Bm, size_t sdsB, int ns, int nC, int mg,
                           double* S, int ld, int tid, int nth) {
    const int nT = (nC + T - 1) / T;
    for (int t = tid; t < nT * nT; t += nth) {
        const int i0 = (t / nT) * T, j0 = (t % nT) * T;
        double acc[T][T];
#pragma unroll
        for (int a = 0; a < T; ++a)
#pragma unroll
            for (int b = 0; b < T; ++b) acc[a][b] = 0.0;
        for (int sd = 0; sd < ns; ++sd) {
            const double* As = A + sd * sdsA;
            const double* Bs = Bm + sd * sdsB;
            // all columns of this subdomain's rows are loaded before any product (mg <= MG)
            double av[T][MG], bv[T][MG];
#pragma unroll
            for (int a = 0; a < T; ++a)
#pragma unroll
                for (int l = 0; l < MG; ++l) {
                    av[a][l] = (i0 + a < nC && l < mg) ? As[(i0 + a) * mg + l] : 0.0;
                    bv[a][l] = (j0 + a < nC && l < mg) ? Bs[(j0 + a) * mg + l] : 0.0;
                }
#pragma unroll
            for (int l = 0; l < MG; ++l)
#pragma unroll
                for (int a = 0; a < T; ++a)
#pragma unroll
                    for (int b = 0; b < T; ++b) acc[a][b] += av[a][l] * bv[b][l];
        }
#pragma unroll
        for (int a = 0; a < T; ++a)
#pragma unroll
            for (int b = 0; b < T; ++b)
                if (i0 + a < nC && j0 + b < nC) S[(i0 + a) * ld + j0 + b] = acc[a][b];
    }
}

// Block size by the work per thread: single entries while nC^2 gives each thread few of them,
// larger register blocks once every thread would otherwise loop over many entries.
template <int MG>
__device__ __forceinline__ void gram_sum(const double* A, size_t sdsA, const double* Bm, size_t sdsB, int ns, int nC,
                                         int mg, double* S, int ld, int tid, int nth) {
    if (nC * nC >= 16 * nth) gram_sum_t<4, MG>(A, sdsA, Bm, sdsB, ns, nC, mg, S, ld, tid, nth);
    else if (nC * nC >= 4 * nth) gram_sum_t<2, MG>(A, sdsA, Bm, sdsB, ns, nC, mg, S, ld, tid, nth);
    else gram_sum_t<1, MG>(A, sdsA, Bm, sdsB, ns, nC, mg, S, ld, tid, nth);
}

// The same sums for arrays in global memory, staged through LDS: chunks of sdc subdomains of A
// and Bm are copied to stage as [sdc * mg][nC] (one (subdomain, row) per thread, its mg <= MG
// contiguous entries; the next chunk's entries are loaded into registers while the current
// chunk's products run), then each thread adds the chunk's products into its own tiles of the
// upper triangle (tile row <= tile column), at most two 4 x 4 tiles per thread held in
// registers across the chunks; the lower triangle is mirrored at the end, so S is exactly
// symmetric (A Bm^T is symmetric when A_sd = Bm_sd W_sd with symmetric W_sd).  Needs
// (nC / 4 rounded up)^2 / 2 tiles <= 2 nth and sdc nC <= nth.  Every thread must call it (it
// holds barriers).
template <int MG>
__device__ void gram_sum_staged(const double* A, size_t sdsA, const double* Bm, size_t sdsB, int ns, int nC, int mg,
                                double* S, int ld, double* stage, int sdc, int tid, int nth) {
    const int nT = (nC + 3) >> 2;
    const int ntile = nT * (nT + 1) / 2;
    int ti[2], tj[2];
    bool own[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        int t = tid + q * nth;
        own[q] = t < ntile;
        // t -> (row r, column c >= r) of the upper triangle, row by row
        int r = 0;
        while (own[q] && t >= nT - r) {
            t -= nT - r;
            ++r;
        }
        ti[q] = r * 4;
        tj[q] = (r + t) * 4;
    }
    double acc[2][4][4];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[q][a][b] = 0.0;
    double* sA = stage;
    double* sB = stage + (size_t)sdc * mg * nC;
    // this thread's (subdomain in chunk, row) of the copy
    const int cd = tid / nC, cj = tid - cd * nC;
    double pa[MG], pb[MG];
    auto fetch = [&](int s0) {
        const bool on = cd < sdc && s0 + cd < ns;
#pragma unroll
        for (int l = 0; l < MG; ++l) {
            pa[l] = (on && l < mg) ? A[(s0 + cd) * sdsA + cj * mg + l] : 0.0;
            pb[l] = (on && l < mg) ? Bm[(s0 + cd) * sdsB + cj * mg + l] : 0.0;
        }
    };
    fetch(0);
    for (int s0 = 0; s0 < ns; s0 += sdc) {
        const int nsd = min(sdc, ns - s0), kc = nsd * mg;
        __syncthreads();   // the previous chunk's products are done
        if (cd < nsd)
#pragma unroll
            for (int l = 0; l < MG; ++l)
                if (l < mg) {
                    sA[(cd * mg + l) * nC + cj] = pa[l];
                    sB[(cd * mg + l) * nC + cj] = pb[l];
                }
        __syncthreads();
        if (s0 + sdc < ns) fetch(s0 + sdc);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (!own[q]) continue;
            for (int k = 0; k < kc; ++k) {
                double av[4], bv[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    av[a] = ti[q] + a < nC ? sA[k * nC + ti[q] + a] : 0.0;
                    bv[a] = tj[q] + a < nC ? sB[k * nC + tj[q] + a] : 0.0;
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[q][a][b] += av[a] * bv[b];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (!own[q]) continue;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = ti[q] + a, j = tj[q] + b;
                if (i < nC && j < nC && i <= j) {
                    S[i * ld + j] = acc[q][a][b];
                    S[j * ld + i] = acc[q][a][b];
                }
            }
    }
}

// u[sd][l] = sum_j Ehat_sd[j][l] v[j] for l < n_sd^Gamma (0 for l up to mg), one (sd, l) per
// thread, j ascending.
__device__ void et_vec(const double* Es, size_t esds, int ns, int nC, int mg, const int* n_ga, const double* v,
                       double* u, int tid, int nth) {
    for (int t = tid; t < ns * mg; t += nth) {
        const int sd = t / mg, l = t % mg;
        double acc = 0.0;
        if (l < n_ga[sd]) {
            const double* E = Es + sd * esds + l;
#pragma unroll 8
            for (int jj = 0; jj < nC; ++jj) acc += E[jj * mg] * v[jj];
        }
        u[t] = acc;
    }
}

// The same for 64 < n <= 128 and n + 1 <= CWM * waves with the augmented matrix in registers:
// wave w holds columns [w CW, (w + 1) CW) of every row (rows lane and lane + 64).  At step k the
// wave owning column k forms the multipliers M[r][k] / M[k][k] of the rows below and publishes
// them through a double-buffered LDS array; every wave then updates its columns with the
// pivot row taken from its own registers.  One barrier per step.  The factors are written back
// to M (LDS or global) and wave 0 back-substitutes.  fbuf: 256 doubles of LDS; sh: 1 int.
template <int CWM>
__device__ bool block_lu_reg(double* M, int n, double* x, double* fbuf, int* sh, int tid, int nth) {
    const int ld = n + 1, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), nw = nth >> 6;
    const int CW = (n + 1 + nw - 1) / nw;
    const int jb = wave * CW;
    double rw0[CWM], rw1[CWM];
#pragma unroll
    for (int c = 0; c < CWM; ++c) {
        const int j = jb + c;
        const bool cj = c < CW && j <= n;
        rw0[c] = (cj && lane < n) ? M[(size_t)lane * ld + j] : 0.0;
        rw1[c] = (cj && lane + 64 < n) ? M[(size_t)(lane + 64) * ld + j] : 0.0;
    }
    if (tid == 0) sh[0] = 1;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const int wk = k / CW, ck = k - wk * CW;
        double* fb = fbuf + (k & 1) * 128;
        const int pl = k & 63;
        const bool hi = k >= 64;
        if (wave == wk) {
            double v0 = 0.0, v1 = 0.0;
#pragma unroll
            for (int c = 0; c < CWM; ++c)
                if (c == ck) { v0 = rw0[c]; v1 = rw1[c]; }
            const double pv = lane_bcast(hi ? v1 : v0, pl);
            const bool pok = pv > 0.0 && isfinite(pv);
            const double rp = pok ? 1.0 / pv : 0.0;
            fb[lane] = lane > k ? v0 * rp : 0.0;
            fb[lane + 64] = lane + 64 > k ? v1 * rp : 0.0;
            if (lane == 0 && !pok) sh[0] = 0;
        }
        __syncthreads();
        const double f0 = fb[lane], f1 = fb[lane + 64];
#pragma unroll
        for (int c = 0; c < CWM; ++c) {
            const int j = jb + c;
            if (c < CW && j > k && j <= n) {
                const double pr = lane_bcast(hi ? rw1[c] : rw0[c], pl);
                rw0[c] -= f0 * pr;
                rw1[c] -= f1 * pr;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CWM; ++c) {
        const int j = jb + c;
        if (c < CW && j <= n) {
            if (lane < n) M[(size_t)lane * ld + j] = rw0[c];
            if (lane + 64 < n) M[(size_t)(lane + 64) * ld + j] = rw1[c];
        }
    }
    __syncthreads();
    const bool ok = sh[0] != 0;
    if (wave == 0 && ok) {
        double rhs0 = lane < n ? M[(size_t)lane * ld + n] : 0.0;
        double rhs1 = lane + 64 < n ? M[(size_t)(lane + 64) * ld + n] : 0.0;
        for (int i = n - 1; i >= 0; --i) {
            const double ri = lane_bcast(i >= 64 ? rhs1 : rhs0, i & 63);
            const double xi = ri / M[(size_t)i * ld + i];
            if (lane == 0) x[i] = xi;
            if (lane < i) rhs0 -= M[(size_t)lane * ld + i] * xi;
            if (lane + 64 < i) rhs1 -= M[(size_t)(lane + 64) * ld + i] * xi;
        }
    }
    __syncthreads();
    return ok;
}

// Solve [M | r] with every thread of the workgroup calling: one wave when n <= 64, else the
// workgroup.  The result is valid for all threads after the call.
__device__ __forceinline__ bool kkt_lu(double* M, int n, double* x, int* okf, double* fbuf, int tid, int nth) {
    constexpr int CWM = 17;
    if (n > 64 && n <= 128 && n + 1 <= CWM * (nth >> 6)) return block_lu_reg<CWM>(M, n, x, fbuf, okf, tid, nth);
    if (n <= 64) {
        if (tid == 0) okf[0] = 1;
        __syncthreads();
        if ((tid >> 6) == 0) {
            const bool ok = wave_spd_solve(M, n, x, tid & 63);
            if (!ok && (tid & 63) == 0) okf[0] = 0;
        }
        __syncthreads();
        return okf[0] != 0;
    }
    return block_lu_solve(M, n, x, okf, tid, nth);
}

// ------------------------------------------------------------------------------------
// Per-solve update: merit, Armijo test, KKT step (one workgroup of NW waves per solve slot)
// ------------------------------------------------------------------------------------
// Block-arrow KKT (eq. sqp_system) by the Schur complement.  E_i = [0, Ehat_i] has only the m_i
// interface columns, so only W_i = H_i^{-1} [0; I_m] (m right-hand sides) and t_i = H_i^{-1} rho_i
// are needed:  S = sum_i Ehat_i (W_i)_Gamma Ehat_i^T,  S s_lambda = c - sum_i Ehat_i (t_i)_Gamma,
// s_i = -(t_i + W_i Ehat_i^T s_lambda).
// Each wave solves its subdomains' systems H_i [W_i | t_i] = [[0; I_m] | rho_i] in registers:
// row r of the augmented block lives in lane r and pivot rows are broadcast lane to lane, so
// these solves need no LDS traffic and no workgroup barrier.  S (a sum over subdomains in a
// fixed order) and its pivoted solve then go through LDS (or global scratch, GB = 2).
// NN >= n_i^Omega + n_i^Gamma and MG >= n_i^Gamma bound every block (smaller blocks are padded
// with identity rows).
template <int NN, int MG, int GB>
__global__ __launch_bounds__(512) void k_update(UpdArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sm = reinterpret_cast<double*>(smem_raw);
    __shared__ int flag_bad;
    __shared__ int lu_ok[1];
    __shared__ double lu_f[256];
    const int slot = blockIdx.x;
    const int nl = live_count(a.n_live, a.B);
    if (slot >= nl) return;
    const int b = slot_solve(a.live, slot, nl);
    SolveState S = a.st[b];
    if (S.phase == PH_DONE) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nth = blockDim.x, nw = nth >> 6;
    const int nC = a.n_C, nD = a.n_D, mg = a.mg, ns = a.n_sub;
    const UpdLds L = upd_lds(ns, nC, mg, NN, MG);
    double* lam_s = sm + L.lam;
    double* c_s = sm + L.c;
    double* sl_s = sm + L.sl;
    double* red = sm + L.red;
    double* us = sm + L.u;
    constexpr int MGS = MG > 0 ? MG : 1;      // mg = max(1, max_i n_i^Gamma) <= MGS
    double* big = GB ? a.gscr + (size_t)slot * a.gstride : sm + L.small;
    const double* rb = a.RB + (size_t)slot * a.RS;
    // E_hat blocks: copied into LDS with everything else (GB = 0), else read where the reduction
    // left them (subdomain stride rs)
    double* Es = GB ? const_cast<double*>(rb) + a.estride : big + L.E;
    const size_t esds = GB ? (size_t)a.rs : (size_t)nC * mg;
    double* Ps = big + L.P;
    double* qs = big + L.q;
    double* rho = big + L.rho;
    double* Xs = big + L.X;
    double* Sm = GB == 1 ? sm + L.small : big + L.S;     // GB = 1: the Schur system alone in LDS
    const int ld = nC + 1;

    for (int jj = tid; jj < nC; jj += nth) {
        c_s[jj] = rb[(size_t)ns * a.rs + jj];
        lam_s[jj] = a.lamt[(size_t)b * nC + jj];
    }
    if (!GB)
        for (int e = tid; e < ns * nC * mg; e += nth) {
            const int sd = e / (nC * mg), r = e % (nC * mg);
            Es[e] = rb[(size_t)sd * a.rs + a.estride + r];
        }
    if (tid == 0) flag_bad = 0;
    __syncthreads();
    auto gv = [&](int sd, int e) {
        const int NNi = a.n_om[sd] + a.n_ga[sd];
        return rb[(size_t)sd * a.rs + NNi * (NNi + 1) / 2 + e];
    };

    // ---- initial multiplier: argmin || [g_i^Gamma + (E_i^Gamma)^T lambda]_i ||, by its normal
    //      equations (sum_i Ehat_i Ehat_i^T) lambda = -sum_i Ehat_i g_i^Gamma ----
    const bool ls_start = S.phase == PH_ZERO || (S.phase == PH_INIT && !(S.flags & SF_LAMFIX));
    // normal equations not positive definite: the constraint Jacobian lacks full row rank, the
    // least-squares multiplier is not unique (Lemma 1 fails); lambda = 0 is kept instead
    bool lam_bad = false;
    if (ls_start && !a.lam_given && nC > 0) {
        // (entries k >= n_i^Gamma of each Ehat_i row are zero)
        if (GB && a.sdc > 0)
            gram_sum_staged<MGS>(Es, esds, Es, esds, ns, nC, mg, Sm, ld, sm + a.stage_off, a.sdc, tid, nth);
        else
            gram_sum<MGS>(Es, esds, Es, esds, ns, nC, mg, Sm, ld, tid, nth);
        for (int i = tid; i < nC; i += nth) {
            double s = 0.0;
            for (int sd = 0; sd < ns; ++sd) {
                const int m = a.n_ga[sd], no = a.n_om[sd];
                const double* E = Es + sd * esds;
                double ev[MGS], gk[MGS];
#pragma unroll
                for (int k = 0; k < MGS; ++k) {
                    ev[k] = k < m ? E[i * mg + k] : 0.0;
                    gk[k] = k < m ? gv(sd, no + k) : 0.0;
                }
#pragma unroll
                for (int k = 0; k < MGS; ++k)
                    if (k < m) s -= ev[k] * gk[k];
            }
            Sm[i * ld + nC] = s;
        }
        __syncthreads();
        lam_bad = !kkt_lu(Sm, nC, lam_s, lu_ok, lu_f, tid, nth);
        __syncthreads();
        if (lam_bad) {
            for (int jj = tid; jj < nC; jj += nth) lam_s[jj] = 0.0;
            __syncthreads();
        }
    }

    // ---- merit at the trial point: phi = 0.5 (sum_i ||rho_i||^2 + ||c||^2), rho_i kept;
    //      rho_i^Gamma = g_i^Gamma + Ehat_i^T lambda ----
    if (nC > 0) {
        et_vec(Es, esds, ns, nC, mg, a.n_ga, lam_s, us, tid, nth);
        __syncthreads();
    }
    {
        double acc = 0.0;
        for (int e = tid; e < ns * NN; e += nth) {
            const int sd = e / NN, r = e % NN;
            const int no = a.n_om[sd], NNi = no + a.n_ga[sd];
            double v = 0.0;
            if (r < NNi) {
                v = gv(sd, r);
                if (r >= no && nC > 0) v += us[sd * mg + (r - no)];
            }
            rho[e] = v;
            acc += v * v;
        }
        for (int jj = tid; jj < nC; jj += nth) acc += c_s[jj] * c_s[jj];
        acc = wave_sum(acc);
        if (lane == 0) red[wave] = acc;
        __syncthreads();
    }
    double phi_t = 0.0;
    for (int w = 0; w < nw; ++w) phi_t += red[w];
    phi_t *= 0.5;
    const double fn_t = sqrt(2.0 * phi_t);

    // ---- decision (every thread evaluates it identically) ----
    int action = 0;   // 0: compute step, 1: backtrack, 2: stop
    bool slow = false;
    if (S.phase == PH_ZERO) {
        // zero start of a warm solve: keep its norm and multiplier, then evaluate the proposal
        // (held in x, lam); the multiplier waits in the step buffer's lambda part
        double* stp = a.step + (size_t)b * (nD + nC);
        for (int jj = tid; jj < nC; jj += nth) {
            stp[nD + jj] = lam_s[jj];
            a.lamt[(size_t)b * nC + jj] = a.lam[(size_t)b * nC + jj];
        }
        for (int e = tid; e < nD; e += nth) a.xt[(size_t)b * nD + e] = a.x[(size_t)b * nD + e];
        if (tid == 0) {
            S.fz = isfinite(fn_t) ? fn_t : INFINITY;
            S.flags |= SF_WARM | SF_LAMFIX | SF_REF;
            S.phase = PH_INIT;
            a.st[b] = S;
        }
        return;
    }
    if (S.phase == PH_INIT && (S.flags & SF_WARM)) {
        S.flags &= ~SF_WARM;
        if (!(isfinite(fn_t) && fn_t <= S.fz)) {
            // fallback: the proposal's first residual is larger than the zero start's
            const double* stp = a.step + (size_t)b * (nD + nC);
            for (int jj = tid; jj < nC; jj += nth) a.lamt[(size_t)b * nC + jj] = stp[nD + jj];
            for (int e = tid; e < nD; e += nth) {   // both the accepted and the trial point restart at zero
                a.x[(size_t)b * nD + e] = 0.0;
                a.xt[(size_t)b * nD + e] = 0.0;
            }
            if (tid == 0) {
                S.flags |= SF_FALLBACK;
                a.st[b] = S;
            }
            return;
        }
    }
    if (S.phase == PH_INIT) {
        S.f0 = (S.flags & SF_REF) ? S.fz : fn_t;
        S.tol = fmax(a.tol_abs, a.tol_rel * S.f0);
        S.fn = fn_t;
        if (!isfinite(fn_t)) {
            S.status = DDROM_STATUS_NONFINITE;
            action = 2;
        } else if (lam_bad) {
            S.status = DDROM_STATUS_KKT_NOT_PD;
            action = 2;
        }
        for (int jj = tid; jj < nC; jj += nth) {
            a.lam[(size_t)b * nC + jj] = lam_s[jj];
            a.lamt[(size_t)b * nC + jj] = lam_s[jj];
        }
    } else {
        const bool ok = isfinite(phi_t) && phi_t <= (1.0 - 2.0 * a.c1 * S.alpha) * S.phi0;
        if (!ok && S.fn <= a.stall_tol * S.f0) {
            S.status = DDROM_STATUS_STALLED;
            action = 2;
        } else if (!ok) {
            S.nbt += 1;
            if (S.nbt > a.max_bt) {
                S.status = DDROM_STATUS_LINESEARCH_FAIL;
                action = 2;
            } else {
                S.alpha *= 0.5;
                action = 1;
            }
        } else {
            for (int e = tid; e < nD; e += nth) a.x[(size_t)b * nD + e] = a.xt[(size_t)b * nD + e];
            for (int jj = tid; jj < nC; jj += nth) a.lam[(size_t)b * nC + jj] = lam_s[jj];
            S.iters += 1;
            // progress of the accepted step near the noise floor
            slow = a.stall_ratio > 0.0 && fn_t <= a.stall_tol * S.f0 && fn_t > a.stall_ratio * S.fn;
            S.fn = fn_t;
        }
    }
    if (action == 0) {
        if (S.fn <= S.tol) {
            S.status = DDROM_STATUS_CONVERGED;
            action = 2;
        } else if (slow) {
            S.status = DDROM_STATUS_STALLED;
            action = 2;
        } else if (S.iters >= a.max_iter) {
            S.status = DDROM_STATUS_MAX_ITER;
            action = 2;
        }
    }
    if (action == 1) {
        for (int e = tid; e < nD; e += nth)
            a.xt[(size_t)b * nD + e] = a.x[(size_t)b * nD + e] + S.alpha * a.step[(size_t)b * (nD + nC) + e];
        for (int jj = tid; jj < nC; jj += nth)
            a.lamt[(size_t)b * nC + jj] = a.lam[(size_t)b * nC + jj] + S.alpha * a.step[(size_t)b * (nD + nC) + nD + jj];
        if (tid == 0) a.st[b] = S;
        return;
    }
    if (action == 2) {
        if (tid == 0) {
            S.phase = PH_DONE;
            a.st[b] = S;
        }
        return;
    }

    // ---- per-subdomain solves H_i [W_i | t_i] = [[0; I_m] | rho_i], one wave per subdomain ----
    constexpr int NA = NN + MG + 1;   // augmented row: NN entries of H_i, MG + 1 right-hand sides
    for (int sd = wave; sd < ns; sd += nw) {
        const int no = a.n_om[sd], ng = a.n_ga[sd], NNi = no + ng;
        const double* hp = rb + (size_t)sd * a.rs;
        const bool real_row = lane < NNi;
        double A[NA];
#pragma unroll
        for (int c = 0; c < NN; ++c) {
            double v = (lane == c) ? 1.0 : 0.0;
            if (real_row && c < NNi) v = hp[lane <= c ? packed_idx(lane, c, NNi) : packed_idx(c, lane, NNi)];
            A[c] = v;
        }
#pragma unroll
        for (int l = 0; l < MG; ++l) A[NN + l] = (l < ng && lane == no + l) ? 1.0 : 0.0;
        A[NN + MG] = (real_row && lane < NN) ? rho[sd * NN + lane] : 0.0;
        // Gauss-Jordan elimination without pivoting (H_i is symmetric positive definite; a
        // non-positive pivot marks the block as not positive definite) over the NNi real rows
        double Hr[NN], Xr[MG + 1];
#pragma unroll
        for (int c = 0; c < NN; ++c) Hr[c] = A[c];
#pragma unroll
        for (int l = 0; l <= MG; ++l) Xr[l] = A[NN + l];
        // Ehat_i rows of the first 64 constraints: loaded before the elimination, which hides
        // their latency
        const double* E = Es + sd * esds;
        double ev0[MG > 0 ? MG : 1];
#pragma unroll
        for (int k = 0; k < MG; ++k) ev0[k] = (k < ng && lane < nC) ? E[lane * mg + k] : 0.0;
        bool okb = true;
        wave_gj<NN, MG + 1>(Hr, Xr, NNi, lane, okb);
        const bool bad = !okb;
        if (bad && lane == 0) flag_bad = 1;
        if (lane < NN)
#pragma unroll
            for (int l = 0; l <= MG; ++l) Xs[((size_t)sd * NN + lane) * (MG + 1) + l] = Xr[l];
        // P_i = Ehat_i (W_i)_Gamma, q_i = Ehat_i (t_i)_Gamma (constraint row j0 + lane in lane)
        for (int j0 = 0; j0 < nC; j0 += 64) {
            const int jj = j0 + lane;
            double P[MG + 1], ev[MG > 0 ? MG : 1];
#pragma unroll
            for (int l = 0; l <= MG; ++l) P[l] = 0.0;
#pragma unroll
            for (int k = 0; k < MG; ++k)
                ev[k] = j0 == 0 ? ev0[k] : ((k < ng && jj < nC) ? E[jj * mg + k] : 0.0);   // loads first
#pragma unroll
            for (int k = 0; k < MG; ++k) {
                if (k < ng) {
#pragma unroll
                    for (int l = 0; l <= MG; ++l) P[l] += ev[k] * lane_bcast(Xr[l], no + k);
                }
            }
            if (jj < nC) {
#pragma unroll
                for (int l = 0; l < MG; ++l)
                    if (l < mg) Ps[((size_t)sd * nC + jj) * mg + l] = l < ng ? P[l] : 0.0;
                qs[(size_t)sd * nC + jj] = P[MG];
            }
        }
    }
    __syncthreads();
    if (flag_bad) {
        if (tid == 0) {
            S.status = DDROM_STATUS_KKT_NOT_PD;
            S.phase = PH_DONE;
            a.st[b] = S;
        }
        return;
    }
    double* stp = a.step + (size_t)b * (nD + nC);
    if (nC > 0) {
        // [S | c - q] with S = sum_i P_i Ehat_i^T, summed over subdomains in a fixed order
        if (GB && a.sdc > 0)
            gram_sum_staged<MGS>(Ps, (size_t)nC * mg, Es, esds, ns, nC, mg, Sm, ld, sm + a.stage_off, a.sdc, tid,
                                 nth);
        else
            gram_sum<MGS>(Ps, (size_t)nC * mg, Es, esds, ns, nC, mg, Sm, ld, tid, nth);
        for (int i = tid; i < nC; i += nth) {
            double s = 0.0;
            for (int sd = 0; sd < ns; ++sd) s += qs[(size_t)sd * nC + i];
            Sm[i * ld + nC] = c_s[i] - s;
        }
        __syncthreads();
        if (!kkt_lu(Sm, nC, sl_s, lu_ok, lu_f, tid, nth) && tid == 0) flag_bad = 1;
        __syncthreads();
        if (flag_bad) {
            if (tid == 0) {
                S.status = DDROM_STATUS_KKT_NOT_PD;
                S.phase = PH_DONE;
                a.st[b] = S;
            }
            return;
        }
    }
    // s_i = -(t_i + W_i u_i),  u_i = Ehat_i^T s_lambda
    if (nC > 0) {
        et_vec(Es, esds, ns, nC, mg, a.n_ga, sl_s, us, tid, nth);
        __syncthreads();
    }
    for (int e = tid; e < ns * NN; e += nth) {
        const int sd = e / NN, r = e % NN;
        const int ng = a.n_ga[sd], NNi = a.n_om[sd] + ng;
        if (r >= NNi) continue;
        const double* X = Xs + ((size_t)sd * NN + r) * (MG + 1);
        double s = X[MG];
        for (int l = 0; l < ng; ++l) s += X[l] * us[sd * mg + l];
        stp[a.xoff[sd] + r] = -s;
    }
    for (int jj = tid; jj < nC; jj += nth) stp[nD + jj] = sl_s[jj];
    __syncthreads();
    for (int e = tid; e < nD; e += nth) a.xt[(size_t)b * nD + e] = a.x[(size_t)b * nD + e] + stp[e];
    for (int jj = tid; jj < nC; jj += nth) a.lamt[(size_t)b * nC + jj] = a.lam[(size_t)b * nC + jj] + stp[nD + jj];
    if (tid == 0) {
        S.phi0 = phi_t;
        S.alpha = 1.0;
        S.nbt = 0;
        S.phase = PH_TRIAL;
        a.st[b] = S;
    }
}

// List of the still-running solves, ascending (one workgroup of 1024 threads), and its length
// in n_live[0] (the host reads it to stop replaying rounds).
__global__ __launch_bounds__(1024) void k_compact(int B, const SolveState* __restrict__ st, int* __restrict__ live,
                                                  int* __restrict__ n_live) {
    __shared__ int wcount[16];
    __shared__ int base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int c0 = 0; c0 < B; c0 += 1024) {
        const int b = c0 + tid;
        const bool run = b < B && st[b].phase != PH_DONE;
        const unsigned long long m = __ballot(run);
        const int below = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wave] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wcount[w];
        if (run) live[off + below] = b;
        __syncthreads();
        if (tid == 0) {
            int t = base;
            for (int w = 0; w < 16; ++w) t += wcount[w];
            base = t;
        }
        __syncthreads();
    }
    if (tid == 0) n_live[0] = base;
}

// warm != 0: x and lam already hold a proposal; the first round evaluates the zero start.
__global__ void k_init(int B, int Bp, int nD, int nC, const double* __restrict__ mu, const double* __restrict__ x0,
                       const double* __restrict__ l0, double* __restrict__ mu_ws, double* __restrict__ x,
                       double* __restrict__ xt, double* __restrict__ lam, double* __restrict__ lamt,
                       SolveState* __restrict__ st, int warm) {
    const int b = blockIdx.x;
    if (b >= Bp) return;
    for (int e = threadIdx.x; e < nD; e += blockDim.x) {
        if (warm) {
            xt[(size_t)b * nD + e] = 0.0;
            continue;
        }
        const double v = (b < B && x0) ? x0[(size_t)b * nD + e] : 0.0;
        x[(size_t)b * nD + e] = v;
        xt[(size_t)b * nD + e] = v;
    }
    for (int j = threadIdx.x; j < nC; j += blockDim.x) {
        if (warm) {
            lamt[(size_t)b * nC + j] = 0.0;
            continue;
        }
        const double v = (b < B && l0) ? l0[(size_t)b * nC + j] : 0.0;
        lam[(size_t)b * nC + j] = v;
        lamt[(size_t)b * nC + j] = v;
    }
    if (threadIdx.x == 0) {
        mu_ws[2 * b] = b < B ? mu[2 * b] : 1.0;
        mu_ws[2 * b + 1] = b < B ? mu[2 * b + 1] : 5.0;
        SolveState s;
        s.phase = b < B ? (warm ? PH_ZERO : PH_INIT) : PH_DONE;
        s.flags = 0;
        s.pad = 0;
        s.fz = 0.0;
        s.status = DDROM_STATUS_MAX_ITER;
        s.iters = 0;
        s.nbt = 0;
        s.alpha = 1.0;
        s.phi0 = 0.0;
        s.tol = 0.0;
        s.f0 = 0.0;
        s.fn = 0.0;
        st[b] = s;
    }
}

__global__ void k_finalize(int B, int nD, int nC, const double* __restrict__ x, const double* __restrict__ lam,
                           const SolveState* __restrict__ st, double* __restrict__ xo, double* __restrict__ lo,
                           int* __restrict__ it, int* __restrict__ status, double* __restrict__ fn,
                           double* __restrict__ f0, int* __restrict__ fallback) {
    const int b = blockIdx.x;
    if (b >= B) return;
    for (int e = threadIdx.x; e < nD; e += blockDim.x) xo[(size_t)b * nD + e] = x[(size_t)b * nD + e];
    if (lo)
        for (int j = threadIdx.x; j < nC; j += blockDim.x) lo[(size_t)b * nC + j] = lam[(size_t)b * nC + j];
    if (threadIdx.x == 0) {
        if (it) it[b] = st[b].iters;
        if (status) status[b] = st[b].status;
        if (fn) fn[b] = st[b].fn;
        if (f0) f0[b] = st[b].f0;
        if (fallback) fallback[b] = (st[b].flags & SF_FALLBACK) ? 1 : 0;
    }
}

// Sum of the GN partials into dense per-solve outputs (ddrom_gn_blocks).
__global__ void k_collect(int B, int Bp, int n_sub, int n_C, int nD, int nmax, int mmax, int estride,
                          const int* __restrict__ n_om, const int* __restrict__ n_ga, const int* __restrict__ xoff,
                          const int* __restrict__ slot0, const int* __restrict__ cpart0, int n_cparts,
                          const double* __restrict__ part,
                          const double* __restrict__ c_part, const double* __restrict__ E_part, double* H, double* g,
                          double* EG, double* c, double* rr) {
    const int b = blockIdx.x;
    if (b >= B) return;
    double rrs = 0.0;
    for (int sd = 0; sd < n_sub; ++sd) {
        const int NN = n_om[sd] + n_ga[sd], NH = NN * (NN + 1) / 2;
        for (int e = threadIdx.x; e < NH + NN + 1; e += blockDim.x) {
            double s = 0.0;
            for (int sl = slot0[sd]; sl < slot0[sd + 1]; ++sl) s += part[((size_t)sl * estride + e) * Bp + b];
            if (e < NH) {
                int i = 0, rem = e;
                while (rem >= NN - i) { rem -= NN - i; ++i; }
                const int j = i + rem;
                if (H) {
                    H[(((size_t)b * n_sub + sd) * nmax + i) * nmax + j] = s;
                    H[(((size_t)b * n_sub + sd) * nmax + j) * nmax + i] = s;
                }
            } else if (e < NH + NN) {
                if (g) g[(size_t)b * nD + xoff[sd] + (e - NH)] = s;
            } else {
                rrs += s;
            }
        }
        if (EG)
            for (int e = threadIdx.x; e < n_C * mmax; e += blockDim.x) {
                const int j = e / mmax, k = e % mmax;
                double sum = 0.0;
                if (k < n_ga[sd])
                    for (int p = cpart0[sd]; p < cpart0[sd + 1]; ++p) sum += E_part[(((size_t)p * n_C + j) * mmax + k) * Bp + b];
                EG[(((size_t)b * n_sub + sd) * n_C + j) * mmax + k] = sum;
            }
    }
    if (c)
        for (int j = threadIdx.x; j < n_C; j += blockDim.x) {
            double s = 0.0;
            for (int p = 0; p < n_cparts; ++p) s += c_part[((size_t)p * n_C + j) * Bp + b];
            c[(size_t)b * n_C + j] = s;
        }
    // rr: reduce across the block
    __shared__ double red[256];
    red[threadIdx.x] = rrs;
    __syncthreads();
    if (threadIdx.x == 0 && rr) {
        double s = 0.0;
        for (int t = 0; t < (int)blockDim.x; ++t) s += red[t];
        rr[b] = s;
    }
}

// Transpose decoder output [rows*(1+n)][Bp] -> x [B][rows], J [B][rows][n]
template <typename T>
__global__ void k_dec_transpose(const T* __restrict__ dec, long long out_row0, int rows, int n, int B, int Bp,
                                T* __restrict__ x, T* __restrict__ J) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)rows * (1 + n) * B;
    if (idx >= tot) return;
    const int b = (int)(idx % B);
    const long long rj = idx / B;
    const int r = (int)(rj / (1 + n)), j = (int)(rj % (1 + n));
    const T v = dec[(size_t)(out_row0 + rj) * Bp + b];
    if (j == 0) {
        if (x) x[(size_t)b * rows + r] = v;
    } else if (J) {
        J[((size_t)b * rows + r) * n + (j - 1)] = v;
    }
}

// DD FOM residual (all owned nodes of all subdomains), one thread per (node slot, solve).
__global__ void k_fom_residual(int total_own, int B, const int* __restrict__ src, const int* __restrict__ sd_of,
                               const long long* __restrict__ meta, const double* __restrict__ mu,
                               const double* __restrict__ xsd, int n_state, int N_x, double nu, double hx,
                               double hy, double* __restrict__ r, double* __restrict__ jac) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)total_own * B) return;
    const int q = (int)(idx % total_own), b = (int)(idx / total_own);
    const int sd = sd_of[q];
    const long long* me = meta + 6 * sd;
    const long long own_off = me[0], n_own = me[1], nint = me[2], nif = me[3], soff = me[4], roff = me[5];
    const double* xs = xsd + (size_t)b * n_state + soff;
    double v[N_SLOTS];
    for (int t = 0; t < 5; ++t) {
        const int code = src[(size_t)q * 5 + t];
        const int kind = src_kind(code), ix = src_index(code);
        if (kind == SRC_OMEGA) {
            v[t] = xs[ix];
            v[5 + t] = xs[ix + nint];
        } else if (kind == SRC_GAMMA) {
            v[t] = xs[2 * nint + ix];
            v[5 + t] = xs[2 * nint + ix + nif];
        } else {
            const int I = ix >> 14, J = ix & 0x3fff;
            exact_uv(-1.0 + I * hx, J * hy, mu[2 * b], mu[2 * b + 1], nu, v[t], v[5 + t]);
        }
    }
    double ru, rv, cu[6], cv[6];
    burgers_point(v, nu, hx, hy, ru, rv, cu, cv);
    const long long l = q - own_off;
    double* rb = r + (size_t)b * N_x + roff;
    rb[l] = ru;
    rb[n_own + l] = rv;
    if (jac) {
        double* ju = jac + ((size_t)b * N_x + roff + l) * 6;
        double* jv = jac + ((size_t)b * N_x + roff + n_own + l) * 6;
        for (int t = 0; t < 6; ++t) {
            // zero the entries that multiply a Dirichlet value
            const int slot = t < 5 ? t : 0;
            const bool bnd = src_kind(src[(size_t)q * 5 + slot]) == SRC_BOUND;
            ju[t] = bnd ? 0.0 : cu[t];
            jv[t] = bnd ? 0.0 : cv[t];
        }
    }
}

// ------------------------------------------------------------------------------------
// Decoded states and the relative error against FOM states (eq. relative_error)
// ------------------------------------------------------------------------------------
// States [n_state][Bp] -> caller layout [B][n_state] (FP64).
template <typename T>
__global__ void k_state_out(const T* __restrict__ st, int n_state, int B, int Bp, double* __restrict__ x) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n_state * B) return;
    const int b = (int)(e / n_state), r = (int)(e % n_state);
    x[e] = (double)st[(size_t)r * Bp + b];
}

// Per subdomain and 64 solves: sum over the subdomain's state rows of (x_FOM - g)^2 and
// x_FOM^2, the FOM state read at each row's global DoF.  Four waves take quarters of the rows
// and are combined in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_err_part(const T* __restrict__ st, const int* __restrict__ dof,
                                                  const long long* __restrict__ meta, int B, int Bp, int N_x,
                                                  const double* __restrict__ xfom, double* __restrict__ part) {
    __shared__ double red[3][2][64];
    const int sd = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int b = blockIdx.y * 64 + lane;
    const long long* me = meta + 6 * sd;
    const long long r0 = me[4], nr = 2 * (me[2] + me[3]);   // state rows of [x^Omega; x^Gamma]
    const long long rb = r0 + nr * w / 4, re = r0 + nr * (w + 1) / 4;
    double num = 0.0, den = 0.0;
    if (b < B) {
        const double* xf = xfom + (size_t)b * N_x;
        for (long long r = rb; r < re; ++r) {
            const double t = xf[dof[r]];
            const double d = t - (double)st[(size_t)r * Bp + b];
            num += d * d;
            den += t * t;
        }
    }
    if (w > 0) {
        red[w - 1][0][lane] = num;
        red[w - 1][1][lane] = den;
    }
    __syncthreads();
    if (w == 0 && b < B) {
        num = ((num + red[0][0][lane]) + red[1][0][lane]) + red[2][0][lane];
        den = ((den + red[0][1][lane]) + red[1][1][lane]) + red[2][1][lane];
        part[((size_t)sd * 2 + 0) * Bp + b] = num;
        part[((size_t)sd * 2 + 1) * Bp + b] = den;
    }
}

__global__ void k_err_final(const double* __restrict__ part, int n_sub, int B, int Bp, double* __restrict__ err) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double t = 0.0;
    for (int sd = 0; sd < n_sub; ++sd) t += part[((size_t)sd * 2) * Bp + b] / part[((size_t)sd * 2 + 1) * Bp + b];
    err[b] = sqrt(t / n_sub);
}

// ====================================================================================
// Host side
// ====================================================================================
namespace {

template <int TAG, int VO = 0>
static int launch_decode_items(const ddrom_model* m, int prec, int act, int c0, int c1, int n, long long stage,
                               const double* xhat, int xstride, int xoff_override, const int* live, const int* n_live,
                               int B, void* out, int Bp, hipStream_t s, long long oshift = 0) {
    if (c1 <= c0) return 0;
    const int rk = act == DDROM_ACT_SWISH ? 2 : 1;
    const int waves = prec == DDROM_PREC_FP64 ? 1 : (act == DDROM_ACT_SWISH ? 2 : 4);
    const int esz = prec == DDROM_PREC_FP64 ? 8 : 4;
    DecLds L;
    L.total = (size_t)stage + (size_t)waves * m->ring * 64 * esz * rk;
    if (L.total > 65536) {
        set_error("decode work item exceeds 64 KiB of LDS");
        return DDROM_EINVAL;
    }
    dim3 grid(c1 - c0, (Bp + 64 * waves - 1) / (64 * waves)), block(64 * waves);
    const unsigned lds = (unsigned)L.total;
#define DEC_LAUNCH(T, NLV, ACTV, WV, W1p, B1p, W2p, XRp)                                                          \
    do {                                                                                                          \
        if (m->ring == DEC_RING)                                                                                  \
            hipLaunchKernelGGL((k_decode<T, NLV, ACTV, WV, TAG, VO, DEC_RING>), grid, block, lds, s, m->chunks_d,  \
                               c0, m->segs_d, W1p, B1p, m->bands, W2p, XRp, xhat, xstride, xoff_override, live,    \
                               n_live, B, (T*)out, Bp, oshift);                                                   \
        else                                                                                                      \
            hipLaunchKernelGGL((k_decode<T, NLV, ACTV, WV, TAG, VO, DEC_RING_WIDE>), grid, block, lds, s,          \
                               m->chunks_d, c0, m->segs_d, W1p, B1p, m->bands, W2p, XRp, xhat, xstride,           \
                               xoff_override, live, n_live, B, (T*)out, Bp, oshift);                              \
    } while (0)
#define DEC_ACT(NLV, ACTV)                                                                                        \
    if (prec == DDROM_PREC_FP64) DEC_LAUNCH(double, NLV, ACTV, 1, m->W1d, m->b1d, m->W2d, m->xrefd);            \
    else if (ACTV == DDROM_ACT_SWISH) DEC_LAUNCH(float, NLV, ACTV, 2, m->W1f, m->b1f, m->W2f, m->xreff);         \
    else DEC_LAUNCH(float, NLV, ACTV, 4, m->W1f, m->b1f, m->W2f, m->xreff);
#define DEC_CASE(NLV)                                                                                             \
    case NLV:                                                                                                     \
        if (act == DDROM_ACT_SIGMOID) { DEC_ACT(NLV, DDROM_ACT_SIGMOID) }                                       \
        else if (act == DDROM_ACT_SWISH) { DEC_ACT(NLV, DDROM_ACT_SWISH) }                                       \
        else { DEC_ACT(NLV, DDROM_ACT_IDENTITY) }                                                                 \
        break;
    switch (n) {
        DEC_CASE(2) DEC_CASE(3) DEC_CASE(4) DEC_CASE(5) DEC_CASE(6) DEC_CASE(8) DEC_CASE(10) DEC_CASE(12)
        DEC_CASE(16)
        default:
            set_error("unsupported latent size " + std::to_string(n));
            return DDROM_EINVAL;
    }
#undef DEC_CASE
#undef DEC_ACT
#undef DEC_LAUNCH
    HIPCHECK(hipGetLastError());
    return 0;
}

// Work items of one segment (seg_chunk0/1), or every work item of a decoder family's plan.
template <int TAG, int VO = 0>
static int launch_decode_seg(const ddrom_model* m, int prec, int g, const double* xhat, int xstride,
                             int xoff_override, const int* live, const int* n_live, int B, void* out, int Bp,
                             hipStream_t s, long long oshift = 0) {
    // segments of families 1 and 3 are interface decoders
    const int act = ((g / m->n_sub) & 1) ? m->act_ga : m->act;
    return launch_decode_items<TAG, VO>(m, prec, act, m->seg_chunk0[g], m->seg_chunk1[g], m->segs_h[g].n,
                                        prec == DDROM_PREC_FP64 ? m->seg_stage_f64[g] : m->seg_stage_f32[g], xhat,
                                        xstride, xoff_override, live, n_live, B, out, Bp, s, oshift);
}

template <int TAG, int VO = 0>
static int launch_decode_family(const ddrom_model* m, int prec, int f, const double* xhat, const int* live,
                                const int* n_live, int B, void* out, int Bp, hipStream_t s) {
    const int act = (f & 1) ? m->act_ga : m->act;
    for (const auto& pl : m->dec_plan[f]) {
        const int rc = launch_decode_items<TAG, VO>(m, prec, act, pl.c0, pl.c1, pl.n,
                                                    prec == DDROM_PREC_FP64 ? pl.stage_f64 : pl.stage_f32, xhat,
                                                    m->n_D, -1, live, n_live, B, out, Bp, s);
        if (rc) return rc;
    }
    return 0;
}


// One launch per latent class of the residual plan.
static int launch_res_item(const ddrom_model* m, int prec, const ddrom_model::ResPlan& rs, const ddrom_workspace* ws,
                           const int* live, const int* n_live, int B, hipStream_t s) {
    const int c0 = rs.c0, c1 = rs.c1;
    dim3 grid(c1 - c0, ws->Bp / 64), block(256);
#define RES_CASE(A, G)                                                                                            \
    if (rs.n_om == A && rs.n_ga == G) {                                                                           \
        if (prec == DDROM_PREC_FP64)                                                                              \
            hipLaunchKernelGGL((k_res_gn<double, A, G>), grid, block, 0, s, m->rchunks_d, c0, m->rsegs_d,          \
                               m->segs_d, m->gather_d, (const double*)ws->dec_out, ws->bc, live, n_live, B, ws->Bp, \
                               m->nu, m->hx, m->hy, ws->gn_part, m->estride, ws->zero_row);                       \
        else                                                                                                      \
            hipLaunchKernelGGL((k_res_gn<float, A, G>), grid, block, 0, s, m->rchunks_d, c0, m->rsegs_d,           \
                               m->segs_d, m->gather_d, (const float*)ws->dec_out, ws->bc, live, n_live, B, ws->Bp,  \
                               m->nu, m->hx, m->hy, ws->gn_part, m->estride, ws->zero_row);                       \
        HIPCHECK(hipGetLastError());                                                                              \
        return 0;                                                                                                 \
    }
    RES_CASE(2, 1) RES_CASE(3, 2) RES_CASE(4, 2) RES_CASE(4, 4) RES_CASE(6, 3) RES_CASE(8, 4) RES_CASE(12, 6) RES_CASE(4, 0)
    RES_CASE(10, 5) RES_CASE(16, 8)
    RES_CASE(6, 0) RES_CASE(8, 0)
#undef RES_CASE
    set_error("unsupported latent sizes (" + std::to_string(rs.n_om) + ", " + std::to_string(rs.n_ga) + ")");
    return DDROM_EINVAL;
}

// Gappy POD: stored rows of one latent class of the residual plan.
static int launch_res_rows(const ddrom_model* m, int prec, const ddrom_model::ResPlan& rs, const ddrom_workspace* ws,
                           const int* live, const int* n_live, int B, hipStream_t s) {
    dim3 grid(rs.c1 - rs.c0, ws->Bp / 64), block(256);
#define ROWS_CASE(A, G)                                                                                           \
    if (rs.n_om == A && rs.n_ga == G) {                                                                           \
        if (prec == DDROM_PREC_FP64)                                                                              \
            hipLaunchKernelGGL((k_res_rows<double, A, G>), grid, block, 0, s, m->rchunks_d, rs.c0, m->rsegs_d,     \
                               m->segs_d, m->gseg_d, m->gather_d, (const double*)ws->dec_out, ws->bc, live, n_live, \
                               B, ws->Bp, m->nu, m->hx, m->hy, ws->g_R, ws->zero_row);                            \
        else                                                                                                      \
            hipLaunchKernelGGL((k_res_rows<float, A, G>), grid, block, 0, s, m->rchunks_d, rs.c0, m->rsegs_d,      \
                               m->segs_d, m->gseg_d, m->gather_d, (const float*)ws->dec_out, ws->bc, live, n_live,  \
                               B, ws->Bp, m->nu, m->hx, m->hy, ws->g_R, ws->zero_row);                            \
        HIPCHECK(hipGetLastError());                                                                              \
        return 0;                                                                                                 \
    }
    ROWS_CASE(2, 1) ROWS_CASE(3, 2) ROWS_CASE(4, 2) ROWS_CASE(4, 4) ROWS_CASE(6, 3) ROWS_CASE(8, 4) ROWS_CASE(4, 0)
    ROWS_CASE(6, 0) ROWS_CASE(8, 0)
#undef ROWS_CASE
    set_error("gappy POD: unsupported latent sizes (" + std::to_string(rs.n_om) + ", " + std::to_string(rs.n_ga) + ")");
    return DDROM_EINVAL;
}

static int launch_gappy(const ddrom_model* m, const ddrom_workspace* ws, const int* n_live, int B, hipStream_t s) {
    if (m->n_gitems > 0)
        hipLaunchKernelGGL(k_gappy_y, dim3(m->n_gitems, ws->Bp / 64), dim3(256), 0, s, m->gitems_d, m->gseg_d,
                           m->gP_d, ws->g_R, ws->g_Y, n_live, B, ws->Bp);
    // one launch per latent size present (every subdomain's sums go to its own slot, sd)
    std::vector<int> sizes;
    for (int sd = 0; sd < m->n_sub; ++sd) {
        if (m->rsegs_h[sd].slot0 != sd) {
            set_error("gappy POD: partial slot of a subdomain is not its index");
            return DDROM_EINVAL;
        }
        if (std::find(sizes.begin(), sizes.end(), m->gseg_h[sd].nn) == sizes.end()) sizes.push_back(m->gseg_h[sd].nn);
    }
    for (const int nn : sizes) {
        const dim3 grid(m->n_sub, ws->Bp / 64);
#define GN_CASE(NV)                                                                                               \
    case NV:                                                                                                      \
        hipLaunchKernelGGL(k_gappy_gn<NV>, grid, dim3(64), 0, s, m->gseg_d, ws->g_Y, n_live, B, ws->Bp,            \
                           ws->gn_part, m->estride);                                                              \
        break;
        switch (nn) {
            GN_CASE(3) GN_CASE(4) GN_CASE(5) GN_CASE(6) GN_CASE(8) GN_CASE(9) GN_CASE(12)
            default:
                set_error("gappy POD: unsupported latent size " + std::to_string(nn));
                return DDROM_EINVAL;
        }
#undef GN_CASE
    }
    HIPCHECK(hipGetLastError());
    return 0;
}

static int launch_res(const ddrom_model* m, int prec, const ddrom_workspace* ws, const int* live, const int* n_live,
                      int B, hipStream_t s) {
    for (const auto& pl : m->res_plan) {
        const int rc = m->gappy ? launch_res_rows(m, prec, pl, ws, live, n_live, B, s)
                                : launch_res_item(m, prec, pl, ws, live, n_live, B, s);
        if (rc) return rc;
    }
    return m->gappy ? launch_gappy(m, ws, n_live, B, s) : 0;
}

struct ModelDevInts {
    int *n_om, *n_ga, *xoff, *slot0, *cpart0;
};
static ModelDevInts get_ints(const ddrom_model* m);

// The model struct has no slot for these, so keep them in a side table keyed by model.
static std::mutex g_mu;
static std::map<const ddrom_model*, ModelDevInts> g_ints;

static ModelDevInts get_ints(const ddrom_model* m) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ints[m];
}

static int launch_con(const ddrom_model* m, int prec, const ddrom_workspace* ws, const double* xhat, const int* live,
                      const int* n_live, int B, hipStream_t s) {
    if (m->srpc) {
        if (m->n_C == 0) return 0;
        ModelDevInts di = get_ints(m);
        hipLaunchKernelGGL(k_con_linear, dim3(m->n_sub, ws->Bp / 64), dim3(64), 0, s, m->Ahat_d, m->n_C,
                           std::max(1, m->mmax), di.n_om, di.n_ga, di.xoff, xhat, m->n_D, live, n_live, B, ws->Bp,
                           ws->c_part, ws->E_part);
        HIPCHECK(hipGetLastError());
        return 0;
    }
    if (m->n_cchunks == 0 || m->n_C == 0) return 0;
    // one launch per interface latent size
    for (const auto& pl : m->con_plan) {
        const int c0 = pl.c0, c1 = pl.c1, ng = pl.n_ga;
        {
            dim3 grid(c1 - c0, ws->Bp / 64), block(256);
#define CON_CASE(G)                                                                                               \
    case G:                                                                                                       \
        if (prec == DDROM_PREC_FP64)                                                                              \
            hipLaunchKernelGGL((k_con<double, G>), grid, block, 0, s, m->cchunks_d, c0, m->rsegs_d, m->segs_d,    \
                               m->CA_d, m->n_C, m->ca_ld, (const double*)ws->dec_out, n_live, B, ws->Bp,          \
                               ws->c_part, ws->E_part, std::max(1, m->mmax));                                     \
        else                                                                                                      \
            hipLaunchKernelGGL((k_con<float, G>), grid, block, 0, s, m->cchunks_d, c0, m->rsegs_d, m->segs_d,     \
                               m->CA_d, m->n_C, m->ca_ld, (const float*)ws->dec_out, n_live, B, ws->Bp,           \
                               ws->c_part, ws->E_part, std::max(1, m->mmax));                                     \
        break;
            switch (ng) {
                CON_CASE(1) CON_CASE(2) CON_CASE(3) CON_CASE(4) CON_CASE(5) CON_CASE(6) CON_CASE(8)
                default:
                    set_error("unsupported interface latent size " + std::to_string(ng));
                    return DDROM_EINVAL;
            }
#undef CON_CASE
            HIPCHECK(hipGetLastError());
        }
    }
    return 0;
}

}  // namespace

// Device copies of small per-subdomain integer tables, kept next to the model.
// One evaluation of all active solves at their trial points (xt).  The interface decoders
// and the constraint sums run on a second stream forked from `s` (they depend only on the
// interface latents), overlapping the interior decoders and the residual kernel.
static int evaluate_round(const ddrom_model* m, ddrom_workspace* ws, int prec, int B, const int* live,
                          const int* n_live, const double* xhat, hipStream_t s) {
    int rc;
    hipStream_t s2 = ws->stream2;
    HIPCHECK(hipEventRecord(ws->ev_fork, s));
    HIPCHECK(hipStreamWaitEvent(s2, ws->ev_fork, 0));
    if ((rc = launch_decode_family<0>(m, prec, 1, xhat, live, n_live, B, ws->dec_out, ws->Bp, s2))) return rc;
    HIPCHECK(hipEventRecord(ws->ev_ga, s2));
    if ((rc = launch_con(m, prec, ws, xhat, live, n_live, B, s2))) return rc;
    HIPCHECK(hipEventRecord(ws->ev_con, s2));
    if ((rc = launch_decode_family<0>(m, prec, 0, xhat, live, n_live, B, ws->dec_out, ws->Bp, s))) return rc;
    HIPCHECK(hipStreamWaitEvent(s, ws->ev_ga, 0));
    if ((rc = launch_res(m, prec, ws, live, n_live, B, s))) return rc;
    HIPCHECK(hipStreamWaitEvent(s, ws->ev_con, 0));
    return 0;
}

static UpdArgs upd_args(const ddrom_model* m, ddrom_workspace* ws, int B, const ddrom_opts* o, int lam_given) {
    ModelDevInts di = get_ints(m);
    UpdArgs a;
    a.n_sub = m->n_sub; a.n_C = m->n_C; a.n_D = m->n_D; a.mg = std::max(1, m->mmax); a.estride = m->estride;
    a.Bp = ws->Bp; a.B = B; a.lam_given = lam_given; a.max_iter = o->max_iter; a.max_bt = o->max_backtracks;
    a.tol_abs = o->tol_abs; a.tol_rel = o->tol_rel; a.c1 = o->armijo_c1; a.stall_tol = o->stall_tol;
    a.stall_ratio = o->stall_ratio;
    a.n_om = di.n_om; a.n_ga = di.n_ga; a.xoff = di.xoff;
    a.RB = ws->RB; a.rs = ws->rs; a.RS = ws->RS;
    a.x = ws->x; a.xt = ws->xt; a.lam = ws->lam; a.lamt = ws->lamt; a.step = ws->step;
    a.st = ws->st; a.live = ws->live; a.n_live = ws->counter;
    return a;
}

// Block bounds (NN >= n_i^Omega + n_i^Gamma, MG >= n_i^Gamma) of the compiled update kernels.
static const int kUpdShapes[][2] = {{3, 1}, {4, 0}, {5, 2}, {6, 0}, {6, 2}, {8, 0}, {9, 3}, {12, 4}, {18, 6}, {20, 12},
                                     {24, 8}};

// Block bounds of the update kernel for a model, and whether its big arrays need global scratch
// (doubles per slot in *gbig, 0 when they fit in LDS).
static int update_shape(const ddrom_model* m, int* NN, int* MG, long long* gbig) {
    int pick = -1;
    for (int k = 0; k < (int)(sizeof(kUpdShapes) / sizeof(kUpdShapes[0])); ++k)
        if (kUpdShapes[k][0] >= m->NNmax && kUpdShapes[k][1] >= m->mmax) { pick = k; break; }
    if (pick < 0) {
        set_error("subdomain block too large for the update kernel");
        return DDROM_EINVAL;
    }
    *NN = kUpdShapes[pick][0];
    *MG = kUpdShapes[pick][1];
    const UpdLds L = upd_lds(m->n_sub, m->n_C, std::max(1, m->mmax), *NN, *MG);
    *gbig = L.small + L.big <= UPD_LDS_DOUBLES ? 0 : L.big;
    return 0;
}

// 0: all update arrays in LDS; 1: the Schur system in LDS, the per-subdomain arrays in global
// scratch; 2: all of them in global scratch.  LDS doubles needed in *lds_doubles.
static int update_mode(const ddrom_model* m, int NN, int MG, long long gbig, long long* lds_doubles) {
    const UpdLds L = upd_lds(m->n_sub, m->n_C, std::max(1, m->mmax), NN, MG);
    if (gbig == 0) {
        *lds_doubles = L.small + L.big;
        return 0;
    }
    const long long s = (long long)m->n_C * (m->n_C + 1);
    if (L.small + s <= UPD_LDS_MAX_DOUBLES) {
        *lds_doubles = L.small + s;
        return 1;
    }
    *lds_doubles = L.small;
    return 2;
}

static int launch_update(const ddrom_model* m, const ddrom_workspace* ws, const UpdArgs& ua, int B, hipStream_t s) {
    int NN, MG, rc;
    long long gbig;
    if ((rc = update_shape(m, &NN, &MG, &gbig))) return rc;
    long long lds_doubles = 0;
    const int GB = update_mode(m, NN, MG, gbig, &lds_doubles);
    if (GB && (!ws->kkt_scr || ws->kkt_stride < gbig)) {
        set_error("workspace lacks KKT scratch");
        return DDROM_EINVAL;
    }
    const int nw = std::max(1, std::min(8, m->n_sub));
    UpdArgs a = ua;
    a.gscr = ws->kkt_scr;
    a.gstride = ws->kkt_stride;
    // Schur assembly staged through the LDS left over (at most two upper-triangle tiles per thread)
    a.sdc = 0;
    a.stage_off = (int)lds_doubles;
    if (GB && m->n_C > 0) {
        const int nT = (m->n_C + 3) / 4, mg = std::max(1, m->mmax);
        const long long per_sd = 2LL * mg * m->n_C;
        const long long room = UPD_LDS_MAX_DOUBLES - lds_doubles;
        if (nT * (nT + 1) / 2 <= 2 * 64 * nw && room >= per_sd && m->n_C <= 64 * nw) {
            a.sdc = (int)std::min<long long>({(long long)m->n_sub, room / per_sd, (long long)(64 * nw / m->n_C)});
            lds_doubles += (long long)a.sdc * per_sd;
        }
    }
    const size_t lds = (size_t)lds_doubles * sizeof(double);
#define UPD_CASE(A, G)                                                                                   \
    if (NN == A && MG == G) {                                                                            \
        if (GB == 2) hipLaunchKernelGGL((k_update<A, G, 2>), dim3(B), dim3(64 * nw), lds, s, a);       \
        else if (GB == 1) hipLaunchKernelGGL((k_update<A, G, 1>), dim3(B), dim3(64 * nw), lds, s, a);  \
        else hipLaunchKernelGGL((k_update<A, G, 0>), dim3(B), dim3(64 * nw), lds, s, a);               \
    }
    UPD_CASE(3, 1) UPD_CASE(4, 0) UPD_CASE(5, 2) UPD_CASE(6, 0) UPD_CASE(6, 2) UPD_CASE(8, 0) UPD_CASE(9, 3)
    UPD_CASE(12, 4) UPD_CASE(18, 6) UPD_CASE(20, 12) UPD_CASE(24, 8)
#undef UPD_CASE
    HIPCHECK(hipGetLastError());
    return 0;
}

static int round_launch(const ddrom_model* m, ddrom_workspace* ws, int prec, int B, const UpdArgs& ua, hipStream_t s) {
    int rc;
    if ((rc = evaluate_round(m, ws, prec, B, ws->live, ws->counter, ws->xt, s))) return rc;
    ModelDevInts di = get_ints(m);
    const int n_etiles = (m->estride + m->n_C * std::max(1, m->mmax) + RED_E - 1) / RED_E;
    hipLaunchKernelGGL(k_reduce, dim3(m->n_sub + 1, n_etiles, ws->Bp / 64), dim3(256), 0, s, m->n_sub, m->n_C,
                       std::max(1, m->mmax), m->estride, ws->rs, ws->RS, ws->Bp, B, di.n_om, di.n_ga, di.slot0,
                       di.cpart0, m->n_cparts, ws->gn_part, ws->c_part, ws->E_part, ws->counter, ws->RB);
    if ((rc = launch_update(m, ws, ua, B, s))) return rc;
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, B, ws->st, ws->live, ws->counter);
    HIPCHECK(hipGetLastError());
    return 0;
}

extern "C" {

const char* ddrom_last_error(void) { return g_err.c_str(); }

int ddrom_model_create(const ddrom_model_desc* desc, ddrom_model** out) {
    if (!out) {
        set_error("out is NULL");
        return DDROM_EINVAL;
    }
    *out = nullptr;
    std::unique_ptr<ddrom_model> m(new ddrom_model());
    int rc = build_model(desc, m.get());
    if (rc) {
        free_model(m.get());
        return rc;
    }
    ModelDevInts di{};
    std::vector<int> slot0(m->n_sub + 1);
    for (int sd = 0; sd < m->n_sub; ++sd) slot0[sd] = m->rsegs_h[sd].slot0;
    slot0[m->n_sub] = m->n_slots;
    std::vector<int> cpart0(m->n_sub + 1);
    for (int sd = 0; sd < m->n_sub; ++sd) cpart0[sd] = m->rsegs_h[sd].cpart0;
    cpart0[m->n_sub] = m->n_cparts;
    auto up = [&](int** p, const std::vector<int>& v) -> int {
        if (hipMalloc((void**)p, v.size() * sizeof(int)) != hipSuccess) return DDROM_ENOMEM;
        if (hipMemcpy(*p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return DDROM_EHIP;
        return 0;
    };
    if ((rc = up(&di.n_om, m->n_om)) || (rc = up(&di.n_ga, m->n_ga)) || (rc = up(&di.xoff, m->xoff)) ||
        (rc = up(&di.slot0, slot0)) || (rc = up(&di.cpart0, cpart0))) {
        set_error("device allocation failed");
        free_model(m.get());
        return rc;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_ints[m.get()] = di;
    }
    *out = m.release();
    return 0;
}

void ddrom_model_destroy(ddrom_model* m) {
    if (!m) return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ints.find(m);
        if (it != g_ints.end()) {
            (void)hipFree(it->second.n_om);
            (void)hipFree(it->second.n_ga);
            (void)hipFree(it->second.xoff);
            (void)hipFree(it->second.slot0);
            (void)hipFree(it->second.cpart0);
            g_ints.erase(it);
        }
    }
    free_model(m);
    delete m;
}

long long ddrom_model_size(const ddrom_model* m, int q, int sd) {
    if (!m) return -1;
    if (sd >= 0 && sd >= m->n_sub) return -1;
    switch (q) {
        case 0: return m->n_sub;
        case 1: return m->n_D;
        case 2: return m->n_C;
        case 3: return m->N_A;
        case 4: return m->N_x;
        case 5: return m->n_state;
        case 6: { long long t = 0; for (int v : m->nb) t += v; return t; }
        case 7: return m->tile_dec_rows;
        case 8: return m->tile_res_nodes;
        case 9: return m->tile_con_orows;
        case 10: return sd < 0 ? -1 : m->n_om[sd];
        case 11: return sd < 0 ? -1 : m->n_ga[sd];
        case 12: return sd < 0 ? -1 : m->N_om[sd];
        case 13: return sd < 0 ? -1 : m->N_ga[sd];
        case 14: return sd < 0 ? -1 : (long long)m->subnet_rows[sd].size();
        case 15: return sd < 0 ? -1 : m->hid_om[sd];
        case 16: return sd < 0 ? -1 : m->nb[sd];
        case 17: return sd < 0 ? -1 : m->xoff[sd];
        case 18: return sd < 0 ? -1 : m->n_own[sd];
        case 19: return sd < 0 ? -1 : m->band_nnz[sd];
        case 20: return sd < 0 ? -1 : m->band_nnz[m->n_sub + sd];
        case 21: return sd < 0 ? -1 : m->segs_h[m->n_sub + sd].hid;
        default: return -1;
    }
}

int ddrom_subnet_rows(const ddrom_model* m, int sd, int part, int* rows_h) {
    if (!m || sd < 0 || sd >= m->n_sub || !rows_h || (part != 0 && part != 1)) {
        set_error("bad arguments to ddrom_subnet_rows");
        return DDROM_EINVAL;
    }
    if (part == 0)
        for (size_t k = 0; k < m->subnet_rows[sd].size(); ++k) rows_h[k] = m->subnet_rows[sd][k];
    else
        for (int k = 0; k < m->N_ga[sd]; ++k) rows_h[k] = k;
    return 0;
}

int ddrom_workspace_create(const ddrom_model* m, int max_batch, ddrom_workspace** out) {
    if (!m || !out || max_batch <= 0) {
        set_error("bad arguments to ddrom_workspace_create");
        return DDROM_EINVAL;
    }
    *out = nullptr;
    std::unique_ptr<ddrom_workspace> w(new ddrom_workspace());
    w->m = m;
    w->max_B = max_batch;
    w->Bp = (max_batch + 63) / 64 * 64;
    w->rs = m->estride + m->n_C * std::max(1, m->mmax);
    w->RS = m->n_sub * w->rs + std::max(1, m->n_C);
    const size_t Bp = w->Bp;
    const int ld = m->n_C + 1;
    struct A { void** p; size_t bytes; } allocs[] = {
        {(void**)&w->dec_out, (size_t)(m->dec_rows + 1 + m->nmax) * Bp * sizeof(double)},
        {(void**)&w->bc, std::max<size_t>(1, (size_t)m->n_bc) * Bp * sizeof(double)},
        {(void**)&w->gn_part, (size_t)m->n_slots * m->estride * Bp * sizeof(double)},
        {(void**)&w->c_part, std::max<size_t>(1, (size_t)m->n_cparts * m->n_C) * Bp * sizeof(double)},
        {(void**)&w->E_part, std::max<size_t>(1, (size_t)m->n_cparts * m->n_C * std::max(1, m->mmax)) * Bp * sizeof(double)},
        {(void**)&w->x, Bp * m->n_D * sizeof(double)},
        {(void**)&w->xt, Bp * m->n_D * sizeof(double)},
        {(void**)&w->lam, Bp * std::max(1, m->n_C) * sizeof(double)},
        {(void**)&w->lamt, Bp * std::max(1, m->n_C) * sizeof(double)},
        {(void**)&w->step, Bp * (m->n_D + m->n_C) * sizeof(double)},
        {(void**)&w->live, Bp * sizeof(int)},
        {(void**)&w->mu, Bp * 2 * sizeof(double)},
        {(void**)&w->RB, Bp * (size_t)(m->n_sub * (m->estride + m->n_C * std::max(1, m->mmax)) + std::max(1, m->n_C)) * sizeof(double)},
        {(void**)&w->st, Bp * sizeof(SolveState)},
        {(void**)&w->counter, sizeof(int) * 4},
        {(void**)&w->g_R, std::max<size_t>(1, (size_t)m->g_rrows) * Bp * sizeof(double)},
        {(void**)&w->g_Y, std::max<size_t>(1, (size_t)m->g_yrows) * Bp * sizeof(double)},
    };
    for (auto& a : allocs) {
        if (hipMalloc(a.p, a.bytes) != hipSuccess) {
            set_error("workspace allocation failed");
            ddrom_workspace_destroy(w.release());
            return DDROM_ENOMEM;
        }
    }
    {
        int NN, MG, rc;
        long long gbig;
        if ((rc = update_shape(m, &NN, &MG, &gbig))) {
            ddrom_workspace_destroy(w.release());
            return rc;
        }
        if (gbig > 0) {
            w->kkt_stride = gbig;
            if (hipMalloc((void**)&w->kkt_scr, (size_t)gbig * Bp * sizeof(double)) != hipSuccess) {
                set_error("workspace allocation failed (KKT scratch)");
                ddrom_workspace_destroy(w.release());
                return DDROM_ENOMEM;
            }
        }
    }
    // all-zero block after the decoder outputs (read by boundary stencil slots)
    w->zero_row = m->dec_rows;
    if (hipMemset(w->dec_out, 0, (size_t)(m->dec_rows + 1 + m->nmax) * Bp * sizeof(double)) != hipSuccess) {
        set_error("workspace clear failed");
        ddrom_workspace_destroy(w.release());
        return DDROM_EHIP;
    }
    if (hipHostMalloc((void**)&w->counter_h, sizeof(int) * 4, hipHostMallocDefault) != hipSuccess) {
        set_error("pinned allocation failed");
        ddrom_workspace_destroy(w.release());
        return DDROM_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&w->stream2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&w->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&w->ev_ga, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&w->ev_con, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&w->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&w->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&w->t0) != hipSuccess || hipEventCreate(&w->t1) != hipSuccess) {
        set_error("stream/event creation failed");
        ddrom_workspace_destroy(w.release());
        return DDROM_EHIP;
    }
    *out = w.release();
    return 0;
}

void ddrom_workspace_destroy(ddrom_workspace* w) {
    if (!w) return;
    void* ptrs[] = {w->dec_out, w->bc, w->gn_part, w->g_R, w->g_Y, w->c_part, w->E_part, w->x, w->xt, w->lam, w->lamt,
                    w->step, w->live, w->mu, w->st, w->counter, w->RB};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (w->counter_h) (void)hipHostFree(w->counter_h);
    if (w->state_out) (void)hipFree(w->state_out);
    if (w->kkt_scr) (void)hipFree(w->kkt_scr);
    if (w->err_part) (void)hipFree(w->err_part);
    if (w->graph) (void)hipGraphExecDestroy(w->graph);
    if (w->graph_tail) (void)hipGraphExecDestroy(w->graph_tail);
    if (w->ev_in) (void)hipEventDestroy(w->ev_in);
    if (w->ev_out) (void)hipEventDestroy(w->ev_out);
    if (w->t0) (void)hipEventDestroy(w->t0);
    if (w->t1) (void)hipEventDestroy(w->t1);
    if (w->ev_fork) (void)hipEventDestroy(w->ev_fork);
    if (w->ev_ga) (void)hipEventDestroy(w->ev_ga);
    if (w->ev_con) (void)hipEventDestroy(w->ev_con);
    if (w->stream) (void)hipStreamDestroy(w->stream);
    if (w->stream2) (void)hipStreamDestroy(w->stream2);
    delete w;
}

int dd_fom_residual(const ddrom_model* m, const double* mu_d, const double* xsd_d, int B, double* r_d, double* jac_d,
                    hipStream_t s) {
    if (!m || !mu_d || !xsd_d || !r_d || B < 0) {
        set_error("bad arguments to dd_fom_residual");
        return DDROM_EINVAL;
    }
    if (B == 0) return 0;
    const long long tot = (long long)m->total_own * B;
    const int bs = 256;
    hipLaunchKernelGGL(k_fom_residual, dim3((unsigned)((tot + bs - 1) / bs)), dim3(bs), 0, s, m->total_own, B,
                       m->fom_src_d, m->fom_sd_of_row_d, m->fom_meta_d, mu_d, xsd_d, m->n_state, m->N_x, m->nu,
                       m->hx, m->hy, r_d, jac_d);
    HIPCHECK(hipGetLastError());
    return 0;
}

static int check_ws(const ddrom_model* m, const ddrom_workspace* ws, int B) {
    if (!m || !ws || ws->m != m) {
        set_error("workspace missing or created for another model");
        return DDROM_EINVAL;
    }
    if (B > ws->max_B) {
        set_error("batch larger than the workspace capacity");
        return DDROM_ESHAPE;
    }
    return 0;
}

static int decode_args_ok(const ddrom_model* m, int sd, int part, const double* xhat_d, int prec) {
    if (!m || sd < 0 || sd >= m->n_sub || (part != 0 && part != 1) || !xhat_d || (prec != 0 && prec != 1)) {
        set_error("bad arguments to ae_decode_hr / ae_jacobian_hr");
        return DDROM_EINVAL;
    }
    return 0;
}

// Decode one segment into a staging buffer laid out [row][1 + n][Bp] (stage holds the segment's
// rows from the model's row `first_row` on), then write the caller's [B][rows] / [B][rows][n].
static int decode_staged(const ddrom_model* m, int sd, int part, const double* xhat_d, int B, int prec, void* x_d,
                         void* J_d, void* stage, int Bp, long long first_row, hipStream_t s) {
    const int seg = part * m->n_sub + sd;
    const ddrom::DecSeg& sg = m->segs_h[seg];
    int rc = launch_decode_seg<0>(m, prec, seg, xhat_d, sg.n, 0, nullptr, nullptr, B, stage, Bp, s, first_row);
    if (rc) return rc;
    const long long tot = (long long)sg.rows * (1 + sg.n) * B;
    if (tot == 0) return 0;
    const int bs = 256;
    dim3 grid((unsigned)((tot + bs - 1) / bs));
    if (prec == DDROM_PREC_FP64)
        hipLaunchKernelGGL(k_dec_transpose<double>, grid, dim3(bs), 0, s, (const double*)stage, sg.out - first_row,
                           sg.rows, sg.n, B, Bp, (double*)x_d, (double*)J_d);
    else
        hipLaunchKernelGGL(k_dec_transpose<float>, grid, dim3(bs), 0, s, (const float*)stage, sg.out - first_row,
                           sg.rows, sg.n, B, Bp, (float*)x_d, (float*)J_d);
    HIPCHECK(hipGetLastError());
    return 0;
}

static int decode_common(const ddrom_model* m, ddrom_workspace* ws, int sd, int part, const double* xhat_d, int B,
                         int prec, void* x_d, void* J_d, hipStream_t s) {
    int rc = check_ws(m, ws, B);
    if (rc) return rc;
    if ((rc = decode_args_ok(m, sd, part, xhat_d, prec))) return rc;
    if (B == 0) return 0;
    return decode_staged(m, sd, part, xhat_d, B, prec, x_d, J_d, ws->dec_out, ws->Bp, 0, s);
}

// ---- Allocation-free decoder entry point ----------------------------------------------------
// Its staging buffer is this file-scope device array: every GPU the library runs on holds its own
// copy from module load until the process ends.  Host code never uses the name `scratch` as an
// address (in host code it is only a stand-in for the symbol): the device address of the current
// GPU's copy is looked up once per device with hipGetSymbolAddress and kept in g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[DDROM_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices] = {};

static int scratch_address(void** out) {
    int dev = -1;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device ordinal out of range for the allocation-free entry point");
        return DDROM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
            return DDROM_EHIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return 0;
}

int ae_decode_hr(const ddrom_model* m, ddrom_workspace* ws, int sd, int part, const double* xhat_d, int B,
                 int precision, void* x_d, hipStream_t s) {
    if (!x_d) {
        set_error("x_d is NULL");
        return DDROM_EINVAL;
    }
    return decode_common(m, ws, sd, part, xhat_d, B, precision, x_d, nullptr, s);
}

int ae_jacobian_hr(const ddrom_model* m, ddrom_workspace* ws, int sd, int part, const double* xhat_d, int B,
                   int precision, void* x_d, void* J_d, hipStream_t s) {
    if (!J_d) {
        set_error("J_d is NULL");
        return DDROM_EINVAL;
    }
    return decode_common(m, ws, sd, part, xhat_d, B, precision, x_d, J_d, s);
}

int ae_jacobian_hr_noalloc(const ddrom_model* m, int sd, int part, const double* xhat_d, int B, int precision,
                           void* x_d, void* J_d, hipStream_t s) {
    if (!J_d) {
        set_error("J_d is NULL");
        return DDROM_EINVAL;
    }
    int rc = decode_args_ok(m, sd, part, xhat_d, precision);
    if (rc) return rc;
    if (B < 0) {
        set_error("negative batch");
        return DDROM_EINVAL;
    }
    if (B == 0) return 0;
    const ddrom::DecSeg& sg = m->segs_h[part * m->n_sub + sd];
    const long long Bp = ((long long)B + 63) / 64 * 64;
    const long long esz = precision == DDROM_PREC_FP64 ? 8 : 4;
    const long long need = (long long)sg.rows * (1 + sg.n) * Bp * esz;
    if (need > (long long)DDROM_NOALLOC_SCRATCH_BYTES) {
        set_error("ae_jacobian_hr_noalloc: this decoder and batch need " + std::to_string(need) +
                  " bytes of staging; the allocation-free entry point holds " +
                  std::to_string((long long)DDROM_NOALLOC_SCRATCH_BYTES) + " (use ae_jacobian_hr with a workspace)");
        return DDROM_ESHAPE;
    }
    void* stage = nullptr;
    if ((rc = scratch_address(&stage))) return rc;
    return decode_staged(m, sd, part, xhat_d, B, precision, x_d, J_d, stage, (int)Bp, sg.out, s);
}

int ddrom_gn_blocks(const ddrom_model* m, ddrom_workspace* ws, const double* mu_d, const double* xhat_d, int B,
                    int precision, double* H_d, double* g_d, double* EG_d, double* c_d, double* rr_d, hipStream_t s) {
    int rc = check_ws(m, ws, B);
    if (rc) return rc;
    if (!mu_d || !xhat_d || (precision != 0 && precision != 1)) {
        set_error("bad arguments to ddrom_gn_blocks");
        return DDROM_EINVAL;
    }
    if (B == 0) return 0;
    hipLaunchKernelGGL(k_init, dim3(ws->Bp), dim3(64), 0, s, B, ws->Bp, m->n_D, m->n_C, mu_d, xhat_d,
                       (const double*)nullptr, ws->mu, ws->x, ws->xt, ws->lam, ws->lamt, ws->st, 0);
    if (m->n_bc > 0)
        hipLaunchKernelGGL(k_bc, dim3(m->n_bc, ws->Bp / 64), dim3(64), 0, s, m->bc_xy_d, m->bc_field_d, m->n_bc, ws->mu,
                           B, ws->Bp, m->nu, ws->bc);
    if ((rc = evaluate_round(m, ws, precision, B, nullptr, nullptr, ws->xt, s))) return rc;
    ModelDevInts di = get_ints(m);
    hipLaunchKernelGGL(k_collect, dim3(B), dim3(256), 0, s, B, ws->Bp, m->n_sub, m->n_C, m->n_D, m->nmax,
                       std::max(1, m->mmax), m->estride, di.n_om, di.n_ga, di.xoff, di.slot0, di.cpart0, m->n_cparts, ws->gn_part,
                       ws->c_part, ws->E_part, H_d, g_d, EG_d, c_d, rr_d);
    HIPCHECK(hipGetLastError());
    return 0;
}

struct FinalOut {
    double *x, *lam, *fn, *f0;
    int *it, *status, *fallback;
};

// prop != nullptr: warm start from the network's proposal, the zero start as fallback.
// Rounds captured per graph launch; the host checks the live count between launches.  Once at
// most kTailLive solves still run, graphs of kTailRounds rounds are launched instead, so that
// few rounds run after the last solve stops.
constexpr int kGraphRounds = 8;
constexpr int kTailRounds = 2;
constexpr int kTailLive = 64;

// Upper bound on solver rounds: the first evaluation, max_iter steps of at most max_backtracks + 1
// trial evaluations each, one more, and the two extra evaluations of a warm start.
static long long solver_max_rounds(const ddrom_opts* o, int warm) {
    return 1 + (long long)std::max(1, o->max_iter) * (o->max_backtracks + 1) + 1 + 2 * warm;
}

// The workspace's captured graph of kGraphRounds solver rounds for this batch size and these
// options (captured on first use, kept until the key changes).
static int solver_graph(const ddrom_model* m, ddrom_workspace* ws, int B, const ddrom_opts* o, const UpdArgs& ua,
                        int lam_given, int warm) {
    const int prec = o->precision;
    // Doubles enter the key as exact hexadecimal floating-point text, so options that differ
    // in any bit capture a new graph.
    std::ostringstream key;
    key << std::hexfloat;
    key << B << ":" << prec << ":" << o->max_iter << ":" << o->tol_abs << ":" << o->tol_rel << ":" << o->armijo_c1
        << ":" << o->max_backtracks << ":" << o->stall_tol << ":" << o->stall_ratio << ":" << lam_given << ":"
        << warm;
    if (ws->graph && ws->graph_tail && ws->graph_key == key.str()) return 0;
    for (hipGraphExec_t* ge : {&ws->graph, &ws->graph_tail})
        if (*ge) {
            (void)hipGraphExecDestroy(*ge);
            *ge = nullptr;
        }
    hipStream_t s = ws->stream;
    for (int which = 0; which < 2; ++which) {
        const int rounds = which == 0 ? kGraphRounds : kTailRounds;
        hipGraphExec_t* ge = which == 0 ? &ws->graph : &ws->graph_tail;
        hipGraph_t g;
        HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int crc = 0;
        for (int k = 0; k < rounds && !crc; ++k) crc = round_launch(m, ws, prec, B, ua, s);
        hipError_t ce = hipStreamEndCapture(s, &g);
        if (crc) return crc;
        if (ce != hipSuccess) {
            set_error(std::string("graph capture failed: ") + hipGetErrorString(ce));
            return DDROM_EHIP;
        }
        hipError_t ie = hipGraphInstantiate(ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            *ge = nullptr;
            set_error(std::string("graph instantiation failed: ") + hipGetErrorString(ie));
            return DDROM_EHIP;
        }
    }
    ws->graph_key = key.str();
    return 0;
}

static int solve_common(const ddrom_model* m, ddrom_workspace* ws, const double* mu_d, int B, const double* x0,
                        const double* l0, const ddrom_opts* o, hipStream_t caller, int use_graph, const FinalOut& fo,
                        const ddrom_mlp* prop = nullptr) {
    int rc = check_ws(m, ws, B);
    if (rc) return rc;
    if (!mu_d || !o || o->max_iter < 0 || o->max_backtracks < 0 || (o->precision != 0 && o->precision != 1)) {
        set_error("bad arguments to the solver");
        return DDROM_EINVAL;
    }
    const int warm = prop != nullptr;
    if (warm && (ddrom_mlp_size(prop, 2) != m->n_D || ddrom_mlp_size(prop, 1) != (long long)m->n_D + m->n_C)) {
        set_error("proposal network outputs do not match the model's latents and multipliers");
        return DDROM_ESHAPE;
    }
    hipStream_t s = ws->stream;
    HIPCHECK(hipEventRecord(ws->ev_in, caller));
    HIPCHECK(hipStreamWaitEvent(s, ws->ev_in, 0));
    if (warm) {
        if ((rc = mlp_proposal(prop, mu_d, B, ws->x, m->n_C > 0 ? ws->lam : nullptr, s))) return rc;
        x0 = nullptr;
        l0 = nullptr;
    }
    hipLaunchKernelGGL(k_init, dim3(ws->Bp), dim3(64), 0, s, B, ws->Bp, m->n_D, m->n_C, mu_d, x0, l0, ws->mu, ws->x,
                       ws->xt, ws->lam, ws->lamt, ws->st, warm);
    if (m->n_bc > 0)
        hipLaunchKernelGGL(k_bc, dim3(m->n_bc, ws->Bp / 64), dim3(64), 0, s, m->bc_xy_d, m->bc_field_d, m->n_bc, ws->mu,
                           B, ws->Bp, m->nu, ws->bc);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, B, ws->st, ws->live, ws->counter);
    HIPCHECK(hipGetLastError());
    const UpdArgs ua = upd_args(m, ws, B, o, l0 != nullptr);
    const int prec = o->precision;
    // The first round evaluates the initial latents; later rounds are line-search trials
    // (a warm solve first evaluates the zero start, then the proposal, maybe the zero start again).
    const long long max_rounds = solver_max_rounds(o, warm);
    long long done = 0;
    if (use_graph) {
        if ((rc = solver_graph(m, ws, B, o, ua, l0 != nullptr, warm))) return rc;
        int live = B;
        while (done < max_rounds) {
            const bool tail = live <= kTailLive;
            HIPCHECK(hipGraphLaunch(tail ? ws->graph_tail : ws->graph, s));
            done += tail ? kTailRounds : kGraphRounds;
            HIPCHECK(hipMemcpyAsync(ws->counter_h, ws->counter, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            live = *ws->counter_h;
            if (live == 0) break;
        }
    } else {
        while (done < max_rounds) {
            if ((rc = round_launch(m, ws, prec, B, ua, s))) return rc;
            ++done;
            HIPCHECK(hipMemcpyAsync(ws->counter_h, ws->counter, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            if (*ws->counter_h == 0) break;
        }
    }
    hipLaunchKernelGGL(k_finalize, dim3(B), dim3(64), 0, s, B, m->n_D, m->n_C, ws->x, ws->lam, ws->st, fo.x, fo.lam,
                       fo.it, fo.status, fo.fn, fo.f0, fo.fallback);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipEventRecord(ws->ev_out, s));
    HIPCHECK(hipStreamWaitEvent(caller, ws->ev_out, 0));
    return 0;
}

int sqp_step(const ddrom_model* m, ddrom_workspace* ws, const double* mu_d, int B, double* xhat_d, double* lam_d,
             double* fnorm_d, int* status_d, const ddrom_opts* o, hipStream_t s) {
    if (B == 0) return 0;
    if (!xhat_d || !lam_d || !o) {
        set_error("bad arguments to sqp_step");
        return DDROM_EINVAL;
    }
    ddrom_opts one = *o;
    one.max_iter = 1;
    one.tol_abs = 0.0;
    one.tol_rel = 0.0;
    one.stall_ratio = 0.0;      // one iteration: an accepted step always reports DDROM_STATUS_MAX_ITER
    FinalOut fo{xhat_d, lam_d, fnorm_d, nullptr, nullptr, status_d, nullptr};
    return solve_common(m, ws, mu_d, B, xhat_d, lam_d, &one, s, 0, fo);
}

int rom_solve_batch(const ddrom_model* m, ddrom_workspace* ws, const double* mu_d, int B, const double* xhat0_d,
                    const double* lam0_d, const ddrom_opts* o, double* xhat_d, double* lam_d, int* iters_d,
                    int* status_d, double* fnorm_d, double* fnorm0_d, hipStream_t s) {
    if (B == 0) return 0;
    if (!xhat_d) {
        set_error("xhat_d is NULL");
        return DDROM_EINVAL;
    }
    FinalOut fo{xhat_d, lam_d, fnorm_d, fnorm0_d, iters_d, status_d, nullptr};
    return solve_common(m, ws, mu_d, B, xhat0_d, lam0_d, o, s, 1, fo);
}

// Multi-model solve: every model replays its own captured graph of solver rounds (the one
// rom_solve_batch uses for the same batch size and options) on its own streams, so the models'
// rounds run concurrently; the host relaunches only the models that still have running solves.
int rom_solve_multi(int n_models, const ddrom_model* const* models, ddrom_workspace* const* wss,
                    const double* const* mu_d, const int* Bs, const ddrom_opts* o, double* const* xhat_d,
                    double* const* lam_d, int* const* iters_d, int* const* status_d, double* const* fnorm_d,
                    hipStream_t caller) {
    if (n_models <= 0 || !models || !wss || !mu_d || !Bs || !o || !xhat_d || o->max_iter < 0 ||
        o->max_backtracks < 0 || (o->precision != 0 && o->precision != 1)) {
        set_error("bad arguments to rom_solve_multi");
        return DDROM_EINVAL;
    }
    int rc;
    for (int k = 0; k < n_models; ++k) {
        if ((rc = check_ws(models[k], wss[k], Bs[k]))) return rc;
        if (Bs[k] <= 0 || !mu_d[k] || !xhat_d[k]) {
            set_error("every model of rom_solve_multi needs a batch, parameters and an output");
            return DDROM_EINVAL;
        }
        for (int q = 0; q < k; ++q)
            if (wss[q] == wss[k]) {
                set_error("rom_solve_multi needs one workspace per model");
                return DDROM_EINVAL;
            }
    }
    HIPCHECK(hipEventRecord(wss[0]->ev_in, caller));
    std::vector<char> running(n_models, 1);
    for (int k = 0; k < n_models; ++k) {
        ddrom_workspace* ws = wss[k];
        const ddrom_model* m = models[k];
        const int B = Bs[k];
        HIPCHECK(hipStreamWaitEvent(ws->stream, wss[0]->ev_in, 0));
        hipLaunchKernelGGL(k_init, dim3(ws->Bp), dim3(64), 0, ws->stream, B, ws->Bp, m->n_D, m->n_C, mu_d[k],
                           (const double*)nullptr, (const double*)nullptr, ws->mu, ws->x, ws->xt, ws->lam, ws->lamt,
                           ws->st, 0);
        if (m->n_bc > 0)
            hipLaunchKernelGGL(k_bc, dim3(m->n_bc, ws->Bp / 64), dim3(64), 0, ws->stream, m->bc_xy_d, m->bc_field_d,
                               m->n_bc, ws->mu, B, ws->Bp, m->nu, ws->bc);
        hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, ws->stream, B, ws->st, ws->live, ws->counter);
        HIPCHECK(hipGetLastError());
        if ((rc = solver_graph(m, ws, B, o, upd_args(m, ws, B, o, 0), 0, 0))) return rc;
    }
    const long long max_rounds = solver_max_rounds(o, 0);
    // per model: rounds done and solves still running (2-round tail graphs once few run)
    std::vector<long long> done(n_models, 0);
    std::vector<int> live(Bs, Bs + n_models);
    for (;;) {
        int any = 0;
        for (int k = 0; k < n_models; ++k) {
            if (!running[k]) continue;
            const bool tail = live[k] <= kTailLive;
            HIPCHECK(hipGraphLaunch(tail ? wss[k]->graph_tail : wss[k]->graph, wss[k]->stream));
            done[k] += tail ? kTailRounds : kGraphRounds;
            HIPCHECK(hipMemcpyAsync(wss[k]->counter_h, wss[k]->counter, sizeof(int), hipMemcpyDeviceToHost,
                                    wss[k]->stream));
        }
        for (int k = 0; k < n_models; ++k) {
            if (!running[k]) continue;
            HIPCHECK(hipStreamSynchronize(wss[k]->stream));
            live[k] = *wss[k]->counter_h;
            running[k] = live[k] != 0 && done[k] < max_rounds;
            any |= running[k];
        }
        if (!any) break;
    }
    for (int k = 0; k < n_models; ++k) {
        const ddrom_model* m = models[k];
        ddrom_workspace* ws = wss[k];
        hipLaunchKernelGGL(k_finalize, dim3(Bs[k]), dim3(64), 0, ws->stream, Bs[k], m->n_D, m->n_C, ws->x, ws->lam,
                           ws->st, xhat_d[k], lam_d ? lam_d[k] : nullptr, iters_d ? iters_d[k] : nullptr,
                           status_d ? status_d[k] : nullptr, fnorm_d ? fnorm_d[k] : nullptr, (double*)nullptr,
                           (int*)nullptr);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipEventRecord(ws->ev_out, ws->stream));
        HIPCHECK(hipStreamWaitEvent(caller, ws->ev_out, 0));
    }
    return 0;
}

int rom_solve_warm(const ddrom_model* m, ddrom_workspace* ws, const ddrom_mlp* p, const double* mu_d, int B,
                   const ddrom_opts* o, double* xhat_d, double* lam_d, int* iters_d, int* status_d, double* fnorm_d,
                   double* fnorm0_d, int* fallback_d, hipStream_t s) {
    if (B == 0) return 0;
    if (!p || !xhat_d) {
        set_error("bad arguments to rom_solve_warm");
        return DDROM_EINVAL;
    }
    FinalOut fo{xhat_d, lam_d, fnorm_d, fnorm0_d, iters_d, status_d, fallback_d};
    return solve_common(m, ws, mu_d, B, nullptr, nullptr, o, s, 1, fo, p);
}

// Decoded DD states of B solves into ws->state_out (allocated on the first call).
static int decode_states(const ddrom_model* m, ddrom_workspace* ws, const double* xhat_d, int B, int prec,
                         hipStream_t s) {
    if (!ws->state_out) {
        if (hipMalloc(&ws->state_out, (size_t)m->n_state * ws->Bp * sizeof(double)) != hipSuccess ||
            hipMalloc((void**)&ws->err_part, (size_t)m->n_sub * 2 * ws->Bp * sizeof(double)) != hipSuccess) {
            set_error("state buffer allocation failed");
            return DDROM_ENOMEM;
        }
    }
    int rc;
    for (int f = 2; f < 4; ++f)
        if ((rc = launch_decode_family<0, 1>(m, prec, f, xhat_d, nullptr, nullptr, B, ws->state_out, ws->Bp, s)))
            return rc;
    return 0;
}

int rom_decode_states(const ddrom_model* m, ddrom_workspace* ws, const double* xhat_d, int B, int precision,
                      double* xsd_d, hipStream_t s) {
    int rc = check_ws(m, ws, B);
    if (rc) return rc;
    if (B > 0 && (!xhat_d || !xsd_d || (precision != 0 && precision != 1))) {
        set_error("bad arguments to rom_decode_states");
        return DDROM_EINVAL;
    }
    if (B == 0) return 0;
    if ((rc = decode_states(m, ws, xhat_d, B, precision, s))) return rc;
    const long long tot = (long long)m->n_state * B;
    const dim3 grid((unsigned)((tot + 255) / 256));
    if (precision == DDROM_PREC_FP64)
        hipLaunchKernelGGL(k_state_out<double>, grid, dim3(256), 0, s, (const double*)ws->state_out, m->n_state, B,
                           ws->Bp, xsd_d);
    else
        hipLaunchKernelGGL(k_state_out<float>, grid, dim3(256), 0, s, (const float*)ws->state_out, m->n_state, B,
                           ws->Bp, xsd_d);
    HIPCHECK(hipGetLastError());
    return 0;
}

int rom_relative_error(const ddrom_model* m, ddrom_workspace* ws, const double* xhat_d, int B, int precision,
                       const double* xfom_d, double* err_d, hipStream_t s) {
    int rc = check_ws(m, ws, B);
    if (rc) return rc;
    if (B > 0 && (!xhat_d || !xfom_d || !err_d || (precision != 0 && precision != 1))) {
        set_error("bad arguments to rom_relative_error");
        return DDROM_EINVAL;
    }
    if (B == 0) return 0;
    if ((rc = decode_states(m, ws, xhat_d, B, precision, s))) return rc;
    const dim3 grid(m->n_sub, ws->Bp / 64);
    if (precision == DDROM_PREC_FP64)
        hipLaunchKernelGGL(k_err_part<double>, grid, dim3(256), 0, s, (const double*)ws->state_out, m->state_dof_d,
                           m->fom_meta_d, B, ws->Bp, m->N_x, xfom_d, ws->err_part);
    else
        hipLaunchKernelGGL(k_err_part<float>, grid, dim3(256), 0, s, (const float*)ws->state_out, m->state_dof_d,
                           m->fom_meta_d, B, ws->Bp, m->N_x, xfom_d, ws->err_part);
    hipLaunchKernelGGL(k_err_final, dim3((B + 255) / 256), dim3(256), 0, s, ws->err_part, m->n_sub, B, ws->Bp, err_d);
    HIPCHECK(hipGetLastError());
    return 0;
}

int ddrom_time_kernels(const ddrom_model* m, ddrom_workspace* ws, const double* mu_d, const double* xhat_d, int B,
                       int precision, int reps, float* ms_h) {
    int rc = check_ws(m, ws, B);
    if (rc) return rc;
    if (!mu_d || !xhat_d || !ms_h || reps <= 0 || B <= 0 || (precision != 0 && precision != 1)) {
        set_error("bad arguments to ddrom_time_kernels");
        return DDROM_EINVAL;
    }
    hipStream_t s = ws->stream;
    HIPCHECK(hipDeviceSynchronize());
    hipLaunchKernelGGL(k_init, dim3(ws->Bp), dim3(64), 0, s, B, ws->Bp, m->n_D, m->n_C, mu_d, xhat_d,
                       (const double*)nullptr, ws->mu, ws->x, ws->xt, ws->lam, ws->lamt, ws->st, 0);
    if (m->n_bc > 0)
        hipLaunchKernelGGL(k_bc, dim3(m->n_bc, ws->Bp / 64), dim3(64), 0, s, m->bc_xy_d, m->bc_field_d, m->n_bc, ws->mu,
                           B, ws->Bp, m->nu, ws->bc);
    // warm the decoder outputs once so the residual and constraint kernels read real data
    if ((rc = evaluate_round(m, ws, precision, B, nullptr, nullptr, ws->xt, s))) return rc;
    auto timed = [&](int which, float* out) -> int {
        HIPCHECK(hipEventRecord(ws->t0, s));
        for (int r = 0; r < reps; ++r) {
            int c = 0;
            if (which < 2)
                c = launch_decode_family<1>(m, precision, which, ws->xt, nullptr, nullptr, B, ws->dec_out, ws->Bp, s);
            else if (which == 2) c = launch_res(m, precision, ws, nullptr, nullptr, B, s);
            else c = launch_con(m, precision, ws, ws->xt, nullptr, nullptr, B, s);
            if (c) return c;
        }
        HIPCHECK(hipEventRecord(ws->t1, s));
        HIPCHECK(hipEventSynchronize(ws->t1));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, ws->t0, ws->t1));
        *out = ms / reps;
        return 0;
    };
    for (int k = 0; k < 4; ++k)
        if ((rc = timed(k, ms_h + k))) return rc;
    return 0;
}

}  // extern "C"
