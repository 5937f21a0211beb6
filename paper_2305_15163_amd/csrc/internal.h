// Internal structures shared by the host model builder and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ddrom.h"

namespace ddrom {

// Stencil source codes of the HR residual gather: top two bits select the source.
constexpr int SRC_OMEGA = 0;     // row of the interior subnet output (index into I_o)
constexpr int SRC_GAMMA = 1;     // row of the interface decoder output
constexpr int SRC_BOUND = 2;     // Dirichlet value slot (per-solve boundary buffer)
__host__ __device__ inline int src_kind(int code) { return (code >> 28) & 3; }
__host__ __device__ inline int src_index(int code) { return code & 0x0fffffff; }
__host__ __device__ inline int src_code(int kind, int idx) { return (kind << 28) | idx; }

// Slot order of the 10 gathered DoFs of one sampled node.
enum { S_UC = 0, S_UW, S_UE, S_US, S_UN, S_VC, S_VW, S_VE, S_VS, S_VN, N_SLOTS };

// One decoder as seen by the decode kernel (interior subnet or full interface decoder).
struct DecSeg {
    int n;          // latent size
    int rows;       // output rows kept
    int hid;        // hidden units kept
    int bmax;       // b (values per band slot)
    int xoff;       // offset of this decoder's latent inside xhat (n_D vector)
    int sd;
    long long w1;   // element offset into the W1 pool  [hid][n]
    long long b1;   // element offset into the b1 pool  [hid]
    long long band; // offset into the band pool        [rows][3] (compressed start, length)
    long long w2;   // element offset into the W2 pool  [rows][3][bmax]
    long long xref; // element offset into the x_ref pool [rows]
    long long out;  // first Bp-row of the output: row r, column j (0 value, 1+k Jacobian) at (out + r*(1+n) + j)*Bp
};

// Dynamic LDS layout of one decode work item (byte offsets, 16-byte aligned regions):
// staged W1~ rows [span][nl], biases [span], W2~ values [rows][3][bmax], x_ref [rows],
// band descriptors [rows][3] (int2), then one hidden-activation ring per wave.
// Hidden-unit ring of the decode kernel: every decoded row's three bands must lie in a window
// of at most DEC_RING consecutive (compressed) hidden units (2 b s + b <= DEC_RING for the
// three-band masks).  A model whose windows all fit in DEC_RING units uses that ring; one with
// wider windows (up to DEC_RING_WIDE, e.g. the band-5, shift-5 masks, window 55) uses the wide
// ring and stages fewer weights per work item.  At 46, four waves' FP32 rings take 46 KiB, so
// with a work item's staged weights three workgroups fit in a CU.
constexpr int DEC_RING = 46;
constexpr int DEC_RING_WIDE = 56;

struct DecLds {
    size_t w1, b1, w2, xr, bd, ring, total;
};
__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ inline DecLds dec_lds(int span, int rows, int nl, int bmax, int esz, int waves, int rk, int ring) {
    DecLds L;
    L.w1 = 0;
    L.b1 = al16(L.w1 + (size_t)span * nl * esz);
    L.w2 = al16(L.b1 + (size_t)span * esz);
    L.xr = al16(L.w2 + (size_t)rows * 3 * bmax * esz);
    L.bd = al16(L.xr + (size_t)rows * esz);
    L.ring = al16(L.bd + (size_t)rows * 3 * 8);
    L.total = L.ring + (size_t)waves * ring * 64 * esz * rk;
    return L;
}

struct DecChunk {
    int seg;
    int r0, r1;         // kept rows [r0, r1) of the segment
    int h_lo, h_hi;     // compressed hidden units read by those rows
    int pad[3];
};

// A contiguous range of sampled nodes of one subdomain (one residual/GN work item).
struct ResChunk {
    int sd;
    int p0, p1;     // node range inside the subdomain's HR node list
    int slot;       // GN partial-sum slot
};

struct ResSeg {
    int n_om, n_ga;
    int seg_om, seg_ga;     // decoder segment ids
    long long gather;       // offset into the gather pool [nb][N_SLOTS]
    long long ca;           // offset of (C A_i)^T [N_i^Gamma][ca_ld] in the CA pool
    int slot0, slot1;       // GN partial slots of this subdomain
    int n_rows_ga;          // N_i^Gamma
    int cpart0, cpart1;     // constraint partial-sum slots of this subdomain
    int pad;
};

// Gappy-POD hyper-reduction of one subdomain: the stored residual rows R [rows][nn + 1][Bp]
// (r_u rows of the sampled nodes, then their r_v rows; entry 0 the residual, 1..nn its latent
// gradient), the projected rows Y = P R [modes][nn + 1][Bp] and P [modes][rows] (offsets in
// Bp-rows for R and Y, in doubles for P).
struct GappySeg {
    int nn, nb, rows, modes;
    long long r_off, y_off, p_off;
};

// Gappy-POD projection: modes per work item (each item streams its subdomain's stored rows once
// for this many modes), and the operator rows staged in LDS at a time.
constexpr int kGappyModes = 8;
constexpr int kGappyRowChunk = 256;

struct ConChunk {
    int sd;
    int j0, j1;             // constraint rows
    int o0, o1;             // interface rows summed by this work item
    int part;               // constraint partial-sum slot
    int pad[2];
};

}  // namespace ddrom

struct ddrom_model {
    int nx, ny, nsx, nsy, n_sub, act, n_C, N_A, n_D, N_x, n_state;
    int act_ga = 0;                              // activation of the interface decoders (ports' for SRPC)
    int srpc = 0;                                // 1: strong ROM-port constraint (ports, linear constraint)
    double* Ahat_d = nullptr;                    // SRPC: per subdomain [n_C][mmax] constraint matrix Ahat_i
    int n_ports = 0;
    double nu, ly, hx, hy;
    int nmax, mmax, NNmax, estride;     // max latent sizes, GN partial stride
    std::vector<int> n_om, n_ga, N_om, N_ga, xoff, n_own, nb, hid_om;
    std::vector<long long> band_nnz;            // valid band entries over kept rows, per decoder segment
    std::vector<std::vector<int>> subnet_rows;   // I_o per subdomain (interior local indices)
    std::vector<long long> state_off;            // offset of [x_i^Omega; x_i^Gamma] inside the DD state vector
    std::vector<long long> res_off;              // offset of r_i inside the DD residual vector

    // decoder pools (both precisions)
    float *W1f = nullptr, *b1f = nullptr, *W2f = nullptr, *xreff = nullptr;
    double *W1d = nullptr, *b1d = nullptr, *W2d = nullptr, *xrefd = nullptr;
    int2* bands = nullptr;
    // [0, n_sub): interior subnets; [n_sub, 2 n_sub): interface decoders (value + Jacobian rows
    // in dec_out); [2 n_sub, 3 n_sub): full interior, [3 n_sub, 4 n_sub): full interface
    // decoders (values only, rows of the DD state buffer)
    std::vector<ddrom::DecSeg> segs_h;
    ddrom::DecSeg* segs_d = nullptr;
    std::vector<ddrom::DecChunk> chunks_h;       // grouped by family and latent size, each segment's contiguous
    ddrom::DecChunk* chunks_d = nullptr;
    std::vector<int> seg_chunk0, seg_chunk1;     // chunk range per segment
    long long dec_rows = 0;                      // Bp-rows of the decoder output buffer

    // residual / GN
    int* gather_d = nullptr;
    std::vector<ddrom::ResSeg> rsegs_h;
    ddrom::ResSeg* rsegs_d = nullptr;
    std::vector<ddrom::ResChunk> rchunks_h;
    ddrom::ResChunk* rchunks_d = nullptr;
    int n_slots = 0;
    int n_bc = 0;
    double* bc_xy_d = nullptr;                   // [n_bc][2] boundary point coordinates
    int* bc_field_d = nullptr;                   // [n_bc] 0 = u, 1 = v

    // constraint
    double* CA_d = nullptr;                      // per subdomain [n_C][N_i^Gamma]
    std::vector<long long> CA_off;
    ddrom::ConChunk* cchunks_d = nullptr;
    int n_cchunks = 0;
    int n_cparts = 0;
    int ca_ld = 0;                               // row stride of (C A_i)^T (n_C rounded up to 8)
    std::vector<long long> seg_stage_f32, seg_stage_f64;   // largest staged bytes of a chunk, per segment

    // DD FOM residual: per subdomain, per owned node, 5 stencil sources (C, W, E, S, N)
    int* fom_src_d = nullptr;                    // code: kind<<28 | node position; boundary: (I<<14)|J
    long long* fom_meta_d = nullptr;             // per subdomain: [own_off, n_own, n_int_nodes, n_if_nodes, state_off, res_off]
    int total_own = 0;
    int* fom_sd_of_row_d = nullptr;              // owner subdomain of each flattened own-node slot
    int* state_dof_d = nullptr;                  // [n_state] global DoF of each row of the DD state
    int tile_dec_rows = 0, tile_res_nodes = 0, tile_con_orows = 0;   // work-item shapes in use
    int ring = ddrom::DEC_RING;                  // decode kernel's hidden-unit ring (DEC_RING or DEC_RING_WIDE)

    // Launch plans: the work items of each kernel family are stored grouped by latent class, so
    // that one launch covers every subdomain of a class.  Decoder families: 0 interior subnets,
    // 1 interface decoders, 2 full interior, 3 full interface.
    struct DecPlan { int c0, c1, n; long long stage_f32, stage_f64; };
    struct ResPlan { int c0, c1, n_om, n_ga; };
    struct ConPlan { int c0, c1, n_ga; };
    std::vector<DecPlan> dec_plan[4];
    std::vector<ResPlan> res_plan;
    std::vector<ConPlan> con_plan;

    // gappy-POD hyper-reduction (empty: collocation)
    int gappy = 0;
    std::vector<ddrom::GappySeg> gseg_h;
    ddrom::GappySeg* gseg_d = nullptr;
    double* gP_d = nullptr;                      // all subdomains' P
    int2* gitems_d = nullptr;                    // (subdomain, mode) work items of the projection
    int n_gitems = 0;
    long long g_rrows = 0, g_yrows = 0;          // Bp-rows of R and Y
};

struct SolveState {
    int phase;      // 0 initial evaluation, 1 line-search trial, 2 stopped, 3 zero start of a warm solve
    int status;
    int iters;
    int nbt;
    int flags;      // SF_* bits
    int pad;
    double alpha, phi0, tol, f0, fn;
    double fz;      // first KKT residual norm of the zero start (warm solves)
};
// SolveState::flags
constexpr int SF_WARM = 1;       // the proposal's first evaluation is pending comparison with fz
constexpr int SF_FALLBACK = 2;   // the proposal was rejected; the solve runs from the zero start
constexpr int SF_LAMFIX = 4;     // the initial multiplier is given (no least-squares start)
constexpr int SF_REF = 8;        // tolerances are relative to fz

struct ddrom_workspace {
    const ddrom_model* m = nullptr;
    int max_B = 0, Bp = 0;
    void* dec_out = nullptr;        // decoder values + Jacobians, [dec_rows][Bp] (float or double)
    double* bc = nullptr;           // [n_bc][Bp]
    double* gn_part = nullptr;      // [n_slots][estride][Bp]
    double* g_R = nullptr;          // gappy POD: stored residual rows [g_rrows][Bp]
    double* g_Y = nullptr;          // gappy POD: projected rows [g_yrows][Bp]
    double* c_part = nullptr;       // [n_cparts][n_C][Bp]
    double* E_part = nullptr;       // [n_cparts][n_C][mmax][Bp]
    long long zero_row = 0;         // first Bp-row of an all-zero block at the end of dec_out
    double* x = nullptr;            // accepted latents  [Bp][n_D]
    double* xt = nullptr;           // trial latents     [Bp][n_D]
    double* lam = nullptr;          // [Bp][n_C]
    double* lamt = nullptr;
    double* step = nullptr;         // [Bp][n_D + n_C]
    int* live = nullptr;            // [Bp] original index of each still-running solve, ascending
    void* state_out = nullptr;      // decoded DD states [n_state][Bp], allocated on first use
    int state_prec = -1;            // precision state_out was allocated for
    double* err_part = nullptr;     // [n_sub][2][Bp] error numerators / denominators
    double* kkt_scr = nullptr;      // [Bp][kkt_stride] KKT blocks of models too large for LDS
    long long kkt_stride = 0;
    double* mu = nullptr;           // [Bp][2]
    double* RB = nullptr;           // per-solve reduced blocks [Bp][RS]
    int rs = 0, RS = 0;             // per-subdomain block size, per-solve stride
    SolveState* st = nullptr;       // [Bp]
    int* counter = nullptr;         // [0]: number of running solves (length of `live`)
    int* counter_h = nullptr;       // pinned host mirror
    // private stream (default priority) on which solves run and graphs are captured
    hipStream_t stream = nullptr;
    hipStream_t stream2 = nullptr;  // interface decoders + constraint run here, forked from `stream`
    hipEvent_t ev_in = nullptr, ev_out = nullptr, t0 = nullptr, t1 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_ga = nullptr, ev_con = nullptr;
    // cached graph of solver rounds
    hipGraphExec_t graph = nullptr;         // kGraphRounds solver rounds
    hipGraphExec_t graph_tail = nullptr;    // kTailRounds solver rounds, once few solves still run
    std::string graph_key;
};

namespace ddrom {
void set_error(const std::string& msg);
int build_model(const ddrom_model_desc* desc, ddrom_model* m);   // host tables + device upload
void free_model(ddrom_model* m);
}  // namespace ddrom
