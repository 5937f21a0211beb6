/*
 * ddrom.h - C ABI of the MI355X library for the online solve of the domain-decomposition
 * nonlinear-manifold ROM with collocation hyper-reduction (HR DD NM-ROM) of
 * Diaz, Choi and Heinkenschloss, "A fast and accurate domain decomposition nonlinear
 * manifold reduced order model" (arXiv 2305.15163), applied to the steady 2D viscous
 * Burgers problem of its Section 7.1.
 *
 * Conventions shared by every entry point
 *   - Pointers named *_d are device memory (HIP, current device), owned by the caller.
 *     Pointers named *_h are host memory.  The library never frees or keeps caller buffers.
 *   - All device work is enqueued asynchronously on the given stream (0 = null stream).
 *   - Return value: 0 on success; a negative DDROM_E* code on bad arguments, shape
 *     mismatches, allocation or launch failures, with a message in ddrom_last_error().
 *     Numerical outcomes of a solve never produce a negative return; they are written
 *     per solve to status_d (DDROM_STATUS_*).
 *   - Parameters mu are (a, lambda) of the exact solution psi, u_ex, v_ex (Section 7.1).
 *   - Latent vectors follow the ordering of the SQP section: for subdomains i = 1..n,
 *     xhat = [xhat_1^Omega; xhat_1^Gamma; ...; xhat_n^Omega; xhat_n^Gamma] (length n_D).
 *   - A model is immutable after creation; calls on different streams may share it,
 *     but each call that takes a workspace needs its own workspace.
 */
#ifndef DDROM_H
#define DDROM_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DDROM_OK 0
#define DDROM_EINVAL (-1)
#define DDROM_ENOMEM (-2)
#define DDROM_EHIP (-3)
#define DDROM_ESHAPE (-4)

/* Per-solve outcome codes written to status_d. */
#define DDROM_STATUS_CONVERGED 0
#define DDROM_STATUS_MAX_ITER 1
#define DDROM_STATUS_LINESEARCH_FAIL 2
#define DDROM_STATUS_KKT_NOT_PD 3     /* Lemma 1 hypotheses fail: an H_i or the Schur complement is not positive
                                         definite, or (at the start) the normal equations of the least-squares
                                         multiplier are not: the constraint Jacobian lacks full row rank; the
                                         solve then stops at its start point with lambda = 0 */
#define DDROM_STATUS_NONFINITE 4
#define DDROM_STATUS_STALLED 5        /* near the arithmetic's noise floor (||F|| <= stall_tol ||F_0||): Armijo failed,
                                         or an accepted step made too little progress (stall_ratio) */

#define DDROM_ACT_SIGMOID 0
#define DDROM_ACT_SWISH 1
#define DDROM_ACT_IDENTITY 2

#define DDROM_PREC_FP64 0            /* decoders, residual, KKT all in FP64 */
#define DDROM_PREC_FP32_DECODER 1    /* decoders in FP32; residual, GN blocks, KKT, line search in FP64 */

/* One decoder g(xhat) = x_ref + W2 sigma(W1 xhat + b1) of eq. autoencoder_architecture b/d,
 * with the de-normalisation layer folded into W2 and x_ref.  Host memory, row-major:
 *   W1 [w][n], b1 [w], W2 [N][3][b], x_ref [N].
 * W2 holds the values of the three-band mask of Section 7.3: slot (r, k, t) is column
 * r*s + (k-1)*b*s + t of the dense N x w matrix; slots whose column falls outside [0, w)
 * are ignored.  w must equal N*s.
 * dense != 0: W2 is the full N x w matrix ([N][w], every hidden unit feeds every state; b and s
 * are ignored; w <= 56).  With the identity activation, W1 = I_n and b1 = 0 this is the affine
 * map x_ref + Phi xhat of the LS-ROM (Section 3.3) with Phi = W2. */
typedef struct {
    int N, n, w, b, s;
    const double* W1;
    const double* b1;
    const double* W2;
    const double* x_ref;
    int dense;
} ddrom_decoder_desc;

/* Everything the online solve needs (host memory; deep-copied by ddrom_model_create).
 * Grid: nx x ny interior nodes of [-1, 1] x [0, ly]; a uniform nsx x nsy block split
 * (subdomain i = sy*nsx + sx).  hr_nodes[i] lists hr_count[i] global node ids
 * (node = j*nx + i, 0-based interior indices) owned by subdomain i, ascending; they are
 * the rows kept by the collocation operator Z_i (both the r_u and r_v row of each node).
 * C is the n_C x N_A Gaussian test matrix of the weak compatibility constraint
 * (eq. dd_lspg_NLP b), its columns ordered by the library's constraint-row convention:
 * rows are ordered by the global DoF they duplicate, ascending; a DoF shared by
 * subdomains i_1 < ... < i_k contributes rows x_{i_t} - x_{i_{t+1}} = 0, t = 1..k-1. */
typedef struct {
    int nx, ny;
    double nu, ly;
    int nsx, nsy;
    int activation;                         /* DDROM_ACT_* */
    int n_C, N_A;
    const double* C;                        /* [n_C][N_A] */
    const ddrom_decoder_desc* dec_om;       /* [n_sub] interior decoders g_i^Omega */
    const ddrom_decoder_desc* dec_ga;       /* [n_sub] interface decoders g_i^Gamma */
    const int* hr_count;                    /* [n_sub] */
    const int* const* hr_nodes;             /* [n_sub] -> [hr_count[i]] */
    /* Work-item shapes (0: library default): [0] decoder rows per decode work item (1..64),
     * [1] sampled nodes per residual work item (>= 4), [2] interface rows per constraint
     * work item (>= 4).  They change the schedule only; results are identical up to the
     * order of partial sums. */
    int tile[3];
    /* Strong ROM-port constraint formulation (Section 3.2, eq. dd_lspg_NLP_rom_port) when
     * n_ports > 0: dec_port[j] is the decoder g_j^p of port j (activation port_activation),
     * ports being the groups of interface nodes shared by the same set of subdomains, ordered
     * by their lowest node id; a port's states are its nodes' u values then v values, nodes
     * ascending.  dec_ga, n_C and C are then ignored: subdomain i's interface decoder is
     * eq. gamma_map_port over the ports it carries (ascending port order, one latent copy
     * each, so n_i^Gamma = sum of their n_j^p) and the constraint is sum_i Ahat_i xhat_i^Gamma
     * = 0, one row per port latent component and consecutive carrier pair i_t < i_{t+1}
     * (+1 on i_t, -1 on i_{t+1}), rows ordered port, pair, component; n_C = sum_j
     * (|P(j)| - 1) n_j^p.  n_ports = 0: the weak FOM-port constraint with dec_ga and C. */
    int n_ports;
    const ddrom_decoder_desc* dec_port;     /* [n_ports] */
    int port_activation;                    /* DDROM_ACT_* */
    /* Gappy-POD hyper-reduction (Section 3.1) when hr_modes is not NULL: subdomain i's
     * residual enters the objective as B_i r_i with B_i = (Z_i Phi_i^r)^+ Z_i, given as the
     * dense matrix hr_gappy[i] = (Z_i Phi_i^r)^+, [hr_modes[i]][2 hr_count[i]] row-major, whose
     * columns are the r_u rows of the sampled nodes (ascending) followed by their r_v rows;
     * 1 <= hr_modes[i] <= 2 hr_count[i] and n_i^Omega + n_i^Gamma <= 12.  NULL: collocation,
     * B_i = Z_i. */
    const int* hr_modes;                    /* [n_sub] or NULL */
    const double* const* hr_gappy;          /* [n_sub] -> [hr_modes[i]][2 hr_count[i]] */
} ddrom_model_desc;

typedef struct ddrom_model ddrom_model;
typedef struct ddrom_workspace ddrom_workspace;

typedef struct {
    int max_iter;           /* SQP iterations (accepted steps) */
    double tol_abs;         /* stop when ||F||_2 <= max(tol_abs, tol_rel * ||F_0||_2) */
    double tol_rel;
    double armijo_c1;       /* accept alpha when phi(alpha) <= (1 - 2 c1 alpha) phi(0) */
    int max_backtracks;     /* halvings of alpha before LINESEARCH_FAIL */
    int precision;          /* DDROM_PREC_* */
    double stall_tol;       /* 0 disables; else an Armijo failure with ||F|| <= stall_tol ||F_0|| stops the
                               solve with DDROM_STATUS_STALLED (meant for the FP32-decoder mode) */
    double stall_ratio;     /* 0 disables; else (with stall_tol > 0) an accepted step that ends above the
                               tolerance, at ||F|| <= stall_tol ||F_0||, but reduces ||F|| by less than the
                               factor stall_ratio (||F_new|| > stall_ratio ||F_old||) stops the solve at the
                               new point with DDROM_STATUS_STALLED: progress has slowed to the noise floor */
} ddrom_opts;

const char* ddrom_last_error(void);

/* Build the device model: DD maps (Section 2), ports and A_i, C A_i, the interior
 * decoder subnets of eq. subnet for the HR-sampled stencils (Section 5.4), full interface
 * decoders (Section 5.3: the weak constraint needs every interface row), stencil gather
 * tables and the boundary points touched by sampled stencils.  Synchronous.
 * Supported latent sizes: each decoder's n in {2, 3, 4, 5, 6, 8, 10, 12, 16}; per subdomain
 * (n_i^Omega, n_i^Gamma) among the residual kernel's classes (2,1), (3,2), (4,2), (4,4), (6,3),
 * (8,4), (10,5), (12,6), (16,8) and (4|6|8, 0), with n_i^Omega + n_i^Gamma <= 20 and
 * n_i^Gamma <= 12, or <= 24 with n_i^Gamma <= 8.  Other sizes return DDROM_EINVAL (at creation
 * or at the first launch that needs them). */
int ddrom_model_create(const ddrom_model_desc* desc, ddrom_model** out);
void ddrom_model_destroy(ddrom_model* m);

/* Sizes: query = 0 n_sub, 1 n_D, 2 n_C, 3 N_A, 4 N_x (= 2 nx ny), 5 sum_i (N_i^Omega + N_i^Gamma),
 * 6 total HR nodes, 7..9 the work-item shapes in use (decoder rows, residual nodes,
 * constraint rows).  Per subdomain (sd >= 0): 10 n_i^Omega, 11 n_i^Gamma, 12 N_i^Omega, 13 N_i^Gamma, 14 |I_o| of the interior subnet, 15 |I_h| of the interior subnet,
 * 16 HR nodes, 17 offset of xhat_i^Omega in xhat, 18 own nodes, 19 mask entries of the kept
 * interior rows, 20 mask entries of the interface decoder, 21 hidden units of the interface
 * decoder. */
long long ddrom_model_size(const ddrom_model* m, int query, int sd);

/* Subnet output rows I_o (local indices into x_i^Omega, ascending) of subdomain sd's
 * interior decoder (part 0), or all interface rows (part 1).  rows_h has room for
 * ddrom_model_size(m, 14, sd) (part 0) or N_i^Gamma (part 1) ints. */
int ddrom_subnet_rows(const ddrom_model* m, int sd, int part, int* rows_h);

/* Workspaces hold the per-batch device buffers (decoder outputs, GN partial sums, KKT
 * scratch, per-solve state) for up to max_batch solves; allocated once, reused by calls. */
int ddrom_workspace_create(const ddrom_model* m, int max_batch, ddrom_workspace** out);
void ddrom_workspace_destroy(ddrom_workspace* ws);

/* DD FOM residual (eq. subdomain_residual_def and eq. burgers_discretized) for B
 * subdomain-state vectors.  xsd_d [B][sum_i (N_i^Omega + N_i^Gamma)]: per subdomain
 * [x_i^Omega; x_i^Gamma] in the library's ascending-global-DoF order.  r_d [B][N_x]:
 * per subdomain r_i = [r_u rows of owned nodes ascending; r_v rows], subdomains in
 * order.  jac_d (nullable) [B][N_x][6]: row r_u holds d/du_C, d/du_W, d/du_E, d/du_S,
 * d/du_N, d/dv_C; row r_v holds d/dv_C, d/dv_W, d/dv_E, d/dv_S, d/dv_N, d/du_C; entries
 * whose neighbour is a Dirichlet boundary point are 0.  mu_d [B][2]. */
int dd_fom_residual(const ddrom_model* m, const double* mu_d, const double* xsd_d, int B,
                    double* r_d, double* jac_d, hipStream_t s);

/* Decoder subnet at the HR-sampled rows (eq. subnet): x_d[b][r] = g(xhat_b)[I_o[r]] for
 * part 0 (interior subnet of subdomain sd) or every interface row (part 1).
 * xhat_d [B][n] FP64.  x_d is FP64 [B][rows] when precision = FP64, FP32 otherwise. */
int ae_decode_hr(const ddrom_model* m, ddrom_workspace* ws, int sd, int part, const double* xhat_d, int B,
                 int precision, void* x_d, hipStream_t s);

/* As ae_decode_hr, plus the Jacobian J_d [B][rows][n] = W2~ diag(sigma'(z)) W1~
 * (the rows of dg/dxhat, Section 4.1); x_d may be NULL. */
int ae_jacobian_hr(const ddrom_model* m, ddrom_workspace* ws, int sd, int part, const double* xhat_d, int B,
                   int precision, void* x_d, void* J_d, hipStream_t s);

/* For callers that cannot allocate device memory (work under HIP graph capture, serving loops
 * or harnesses that forbid hipMalloc): ae_jacobian_hr without a workspace.  It calls no
 * allocating routine; the decoder's staging output ([rows][1 + n][Bp] values, Bp = B rounded up
 * to a multiple of 64) lives in a library-owned device array of DDROM_NOALLOC_SCRATCH_BYTES that
 * every GPU the library runs on holds until the process ends.  A decoder and batch needing more
 * (rows (1 + n) Bp times 8 bytes in FP64, 4 in FP32) return DDROM_ESHAPE.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (different streams without ordering, or
 * host threads) race and must be serialised by the caller.  Outputs and errors as in
 * ae_jacobian_hr. */
#define DDROM_NOALLOC_SCRATCH_BYTES (16u << 20)
int ae_jacobian_hr_noalloc(const ddrom_model* m, int sd, int part, const double* xhat_d, int B, int precision,
                           void* x_d, void* J_d, hipStream_t s);

/* Per-subdomain SQP blocks at xhat (eq. gauss_newton_hessian, optimality_residuals_GN):
 * H_d [B][n_sub][nmax][nmax] (H_i = (Z R_i)^T Z R_i, upper-left n_i x n_i used),
 * g_d [B][n_D] ((Z R_i)^T Z r_i stacked), EG_d [B][n_sub][n_C][mmax] (C A_i dg_i^Gamma/dxhat),
 * c_d [B][n_C] (sum_i C A_i g_i^Gamma), rr_d [B] (sum_i ||Z r_i||^2); any output may be NULL.
 * nmax = max_i n_i, mmax = max_i n_i^Gamma. */
int ddrom_gn_blocks(const ddrom_model* m, ddrom_workspace* ws, const double* mu_d, const double* xhat_d, int B,
                    int precision, double* H_d, double* g_d, double* EG_d, double* c_d, double* rr_d,
                    hipStream_t s);

/* One Lagrange-Gauss-Newton SQP iteration (eqs. sqp_system, sqp_update) from
 * (xhat, lambda) for B solves: KKT step with H_i from eq. gauss_newton_hessian, then
 * Armijo backtracking on phi = 0.5 ||F||^2.  xhat_d [B][n_D], lam_d [B][n_C] in/out;
 * fnorm_d [B] receives ||F||_2 at the returned point; status_d [B] receives
 * DDROM_STATUS_MAX_ITER for an accepted step, else the failure code. */
int sqp_step(const ddrom_model* m, ddrom_workspace* ws, const double* mu_d, int B, double* xhat_d,
             double* lam_d, double* fnorm_d, int* status_d, const ddrom_opts* o, hipStream_t s);

/* Batched solve of eq. dd_lspg_NLP for B parameters.  xhat0_d (nullable: zero start)
 * [B][n_D]; lam0_d (nullable: least-squares multiplier of eq. optimality_residuals b at
 * the initial latents).  Outputs xhat_d [B][n_D], lam_d [B][n_C], iters_d [B],
 * status_d [B], fnorm_d [B] (||F||_2 at the returned point), fnorm0_d (nullable) [B].
 * Rounds of (decode, residual + GN blocks, constraint, KKT/line-search update) are
 * replayed from a captured HIP graph; solves that have stopped cost no work. */
int rom_solve_batch(const ddrom_model* m, ddrom_workspace* ws, const double* mu_d, int B,
                    const double* xhat0_d, const double* lam0_d, const ddrom_opts* o,
                    double* xhat_d, double* lam_d, int* iters_d, int* status_d, double* fnorm_d,
                    double* fnorm0_d, hipStream_t s);

/* ---- Learned initial iterate --------------------------------------------------------
 * A dense network maps the Burgers parameters mu = (a, lambda) to a proposal for every
 * subdomain's latents and the multipliers; it stands where the paper interpolates training
 * solutions to start its online solves (Section 7.2).  Inputs (log10 a, lambda), each mapped
 * affinely onto [-1, 1] over a in [1, 1e4], lambda in [5, 20]; layers W_k [out][in], b_k [out]
 * with SiLU after every layer but the last; the outputs are standardised, so the proposal is
 * y * out_std + out_mean: components [0, n_D) are xhat, the rest lambda.  FP32 arithmetic. */
typedef struct ddrom_mlp ddrom_mlp;
typedef struct ddrom_mlp_trainer ddrom_mlp_trainer;

typedef struct {
    int n_layers;               /* dense layers, 1..8 */
    const int* sizes;           /* [n_layers + 1] widths, input first (2); hidden widths <= 512 */
    const float* params;        /* host: W_0, b_0, W_1, b_1, ... packed, W_k row-major [out][in] */
    const double* out_mean;     /* host [sizes[n_layers]] (unused by the trainer) */
    const double* out_std;      /* host [sizes[n_layers]] (unused by the trainer) */
    int n_D;                    /* leading outputs that are latents */
} ddrom_mlp_desc;

/* Device copy of a trained network (immutable after create). */
int ddrom_mlp_create(const ddrom_mlp_desc* d, ddrom_mlp** out);
void ddrom_mlp_destroy(ddrom_mlp* p);
/* query 0: parameter count, 1: output width, 2: n_D; -1 on error. */
long long ddrom_mlp_size(const ddrom_mlp* p, int query);

/* Proposal for B parameters: mu_d [B][2] -> xhat0_d [B][n_D], lam0_d (nullable)
 * [B][outputs - n_D], all FP64 device memory owned by the caller. */
int mlp_proposal(const ddrom_mlp* p, const double* mu_d, int B, double* xhat0_d, double* lam0_d, hipStream_t s);

/* Trainer: FP32 master weights initialised from d->params, Adam moments (beta 0.9, 0.999,
 * eps 1e-8) and activation buffers for minibatches of up to max_batch rows. */
int ddrom_mlp_trainer_create(const ddrom_mlp_desc* d, int max_batch, ddrom_mlp_trainer** out);
void ddrom_mlp_trainer_destroy(ddrom_mlp_trainer* t);
/* query 0: parameter count, 1: output width. */
long long ddrom_mlp_trainer_size(const ddrom_mlp_trainer* t, int query);
/* Copy the current weights (packed as in ddrom_mlp_desc) to device memory params_d. */
int ddrom_mlp_trainer_params(const ddrom_mlp_trainer* t, float* params_d, hipStream_t s);

/* One minibatch: rows_d [B] index the training set mu_d [N][2] (FP64) and standardised
 * targets target_d [N][outputs] (FP32).  Forward, mean squared error over the B x outputs
 * entries, gradient by back-propagation; grad_d (nullable, device [n_params]) receives the
 * gradient; loss_d (nullable, device [1]) the loss before the update; update != 0 applies
 * one Adam step with learning rate lr.  1 <= B <= max_batch. */
int mlp_train_step(ddrom_mlp_trainer* t, const double* mu_d, const float* target_d, const int* rows_d, int B,
                   float lr, int update, float* loss_d, float* grad_d, hipStream_t s);

/* Uneven batch: n_models models, each with its own workspace (distinct), parameters mu_d[k]
 * [Bs[k]][2] and outputs (host arrays of device pointers; lam_d, iters_d, status_d, fnorm_d
 * and their entries may be NULL).  Zero start, options as in rom_solve_batch.  Each model
 * replays its workspace's captured graph of solver rounds (the one rom_solve_batch captures
 * for the same batch size and options) on its own streams, concurrently with the other models;
 * only models with running solves are relaunched.  Results equal separate rom_solve_batch
 * calls bitwise. */
int rom_solve_multi(int n_models, const ddrom_model* const* models, ddrom_workspace* const* wss,
                    const double* const* mu_d, const int* Bs, const ddrom_opts* o, double* const* xhat_d,
                    double* const* lam_d, int* const* iters_d, int* const* status_d, double* const* fnorm_d,
                    hipStream_t s);

/* rom_solve_batch warm-started from the network's proposal, with the zero start (zero
 * latents, least-squares multiplier) as fallback: each solve evaluates the zero start's first
 * KKT residual norm f_zero, then the proposal's; the proposal is kept only if its norm is
 * finite and not larger than f_zero.  Tolerances are relative to f_zero (fnorm0_d receives
 * it).  fallback_d (nullable) [B]: 1 where the zero start was used.  Outputs as in
 * rom_solve_batch. */
int rom_solve_warm(const ddrom_model* m, ddrom_workspace* ws, const ddrom_mlp* p, const double* mu_d, int B,
                   const ddrom_opts* o, double* xhat_d, double* lam_d, int* iters_d, int* status_d, double* fnorm_d,
                   double* fnorm0_d, int* fallback_d, hipStream_t s);

/* ---- Autoencoder training -------------------------------------------------------------
 * One shallow band-masked autoencoder (eq. autoencoder_architecture, Sections 3.4 and 7.3):
 * N state components, latent n, hidden width w = N s, three-band mask of b entries per band
 * shifted by s per row (band k in {-1,0,1} of row r covers columns r s + k b s + t, t < b).
 * BF16 matrix-core products with FP32 accumulation; FP32 master weights; Adam (0.9, 0.999,
 * 1e-8).  Parameters, packed FP32:
 *   W1e [N][3][b]  encoder input layer by band slot (its entry for column c = r s + k b s + t
 *                  connects input r to hidden unit c; slots with c outside [0, w) are zero)
 *   b1e [w], W2e [n][w], W1d [w][n], b1d [w]
 *   W2d [N][3][b]  decoder output layer by band slot (row r, column r s + k b s + t)
 * The loss of a minibatch is (1/B) sum_b ||scale o (y_b - x~_b)||^2 on normalised snapshots
 * x~ (eq. autoencoder_AbsMSE_loss with the de-normalisation scale). */
typedef struct ddrom_ae_trainer ddrom_ae_trainer;

/* params_h: host, packed as above (ddrom_ae_trainer_size(t, 0) floats).  precision 0: BF16
 * operands; 1: each FP32 operand split into a BF16 head and tail, three matrix-core products
 * per tile (about 16 significant bits, FP32-class gradients at three times the matrix work). */
int ddrom_ae_trainer_create(int N, int n, int b, int s, int activation, int max_batch, int precision,
                            const float* params_h, ddrom_ae_trainer** out);
void ddrom_ae_trainer_destroy(ddrom_ae_trainer* t);
/* query 0: parameter count, 1: hidden width w, 2: band slots 3 N b. */
long long ddrom_ae_trainer_size(const ddrom_ae_trainer* t, int query);
/* Copy the FP32 master weights (packed) to device memory params_d. */
int ddrom_ae_trainer_params(const ddrom_ae_trainer* t, float* params_d, hipStream_t s);
/* One minibatch: rows_d [B] index the normalised snapshots X_d [n_snap][N] (FP32, device);
 * scale_d [N] the de-normalisation scale.  loss_d (nullable, device [1]) receives the loss
 * before the update, grad_d (nullable, device, packed) the gradient; update != 0 applies one
 * Adam step with learning rate lr.  1 <= B <= max_batch. */
int ae_train_step(ddrom_ae_trainer* t, const float* X_d, const int* rows_d, int B, const float* scale_d, float lr,
                  int update, float* loss_d, float* grad_d, hipStream_t s);

/* ---- After a solve ------------------------------------------------------------------
 * Decoded subdomain states g_i(xhat_i) of B solves from their latents xhat_d [B][n_D] with the
 * full interior and interface decoders (every row, values only): xsd_d [B][n_state] FP64 in the
 * layout of dd_fom_residual ([x_1^Omega; x_1^Gamma; x_2^Omega; ...]).  The workspace allocates
 * its n_state x max_batch state buffer on the first call of this or the next function. */
int rom_decode_states(const ddrom_model* m, ddrom_workspace* ws, const double* xhat_d, int B, int precision,
                      double* xsd_d, hipStream_t s);

/* Relative error of the decoded states against FOM states (eq. relative_error, Section 7):
 * err_d[b] = sqrt( (1/n_sub) sum_i ||x_FOM|_i - g_i(xhat_i)||^2 / ||x_FOM|_i||^2 ) where x_FOM|_i
 * restricts xfom_d [B][N_x] (FP64, global order [u; v], x-fastest) to subdomain i's interior
 * and interface DoFs.  Decodes in `precision`; sums in FP64. */
int rom_relative_error(const ddrom_model* m, ddrom_workspace* ws, const double* xhat_d, int B, int precision,
                       const double* xfom_d, double* err_d, hipStream_t s);

/* Work-item shape search for one model description and batch (host-driven, synchronous):
 * the batched solve (zero start, options o) of the B parameters mu_d [B][2] is timed with
 * HIP events, median of `reps` runs after one untimed run, for candidate shapes (decoder rows
 * 16..64, residual nodes 8..48, constraint rows 32..256) by coordinate descent from the
 * library defaults: each dimension in turn keeps its fastest value.  Writes the chosen
 * shape to tile_out[3] (for desc->tile) and, if table_h is non-NULL, up to max_table rows
 * [decoder rows, residual nodes, constraint rows, ms] of the shapes tried, their count in
 * *n_tried.  desc->tile is ignored.  Builds and frees a model and workspace per shape. */
int ddrom_autotune(const ddrom_model_desc* desc, const double* mu_d, int B, const ddrom_opts* o, int reps,
                   int* tile_out, float* table_h, int max_table, int* n_tried);

/* Measurement helper: average device time (ms) per launch of the four evaluation kernels
 * of one solver round, ms_h[0] interior decoder subnets, [1] interface decoders,
 * [2] HR residual + Gauss-Newton blocks, [3] weak constraint, each launched `reps` times
 * back to back between two HIP events on the workspace's stream, with every solve live
 * at the latents xhat_d [B][n_D].  Synchronous. */
int ddrom_time_kernels(const ddrom_model* m, ddrom_workspace* ws, const double* mu_d, const double* xhat_d, int B,
                       int precision, int reps, float* ms_h);

#ifdef __cplusplus
}
#endif

#endif
