/*
 * dfpt2.h -- C ABI of libdfpt2.so, the MI355X (gfx950) DF-DSRG-PT2 virtual
 * natural-orbital pass of frozen-natural-orbital SA-DSRG
 * (Li, Mao, Huang, Evangelista, arXiv 2312.07008).
 *
 * What the library computes (paper Sec. 2 and App. A):
 *   For every ordered hole pair (i, j) and virtuals a, b:
 *     V^{ij}_{ab} = sum_Q B^Q_ia B^Q_jb                    density-fitted <ab|ij> (Sec. 3)
 *     Delta       = eps_i + eps_j - eps_a - eps_b          (after Eq. A7)
 *     t^{ij}_{ab} = V (1 - exp(-s Delta^2)) / Delta         (Eq. A7)
 *     Vr^{ij}_{ab}= V (1 + exp(-s Delta^2))                 renormalized integrals
 *   the PT2 energy  E  = 1/4 sum_{ijkl} gamma_ik gamma_jl <Vr_ij, 2T_kl - T_kl^T>,
 *   and the virtual block of the unrelaxed second-order 1-RDM (Eq. A9 with zero
 *   cumulants and no singles)
 *                   D  = 1/2 sum_{ijkl} gamma_ik gamma_jl T_ij (2T_kl - T_kl^T)^T,
 *   gamma = 2 I_core (+) Gamma_act the spin-summed hole density (Eq. A1).
 *   fno_truncate diagonalizes D (Eq. 8) and keeps the natural orbitals whose
 *   cumulative occupation reaches p_o (Eq. 10), optionally widened over
 *   near-degenerate occupations (Sec. 2, after Eq. 10).
 *   pt2_energy_correction recanonicalizes the kept space (Sec. 2), recomputes E
 *   there and returns E(full) - E(kept), the scalar part of Eq. 11.
 *
 * Conventions shared by every entry point:
 *   * Arrays are row-major.  Every array argument is a DEVICE pointer owned by
 *     the caller unless the comment says "host".  The library never keeps a
 *     pointer after the call returns and allocates no device memory: scratch
 *     space is the caller's `workspace` of `ws_bytes` bytes (query the size
 *     first).  All device work is enqueued on `stream` (a hipStream_t; NULL is
 *     the default stream).  Entry points that return a host scalar synchronize
 *     that stream before returning.
 *   * Arguments are validated on the host before anything is launched; a bad
 *     argument returns DFPT2_ERR_INVALID_ARG and leaves every output untouched.
 *   * Errors are reported only through the return status; nothing throws
 *     across the ABI.  dfpt2_last_error() gives a message for the calling
 *     thread's last failure.
 *   * Holes are ordered core first, then active.  Virtual energies must be
 *     ascending.  B is laid out [n_h][n_vir][n_aux] (auxiliary index fastest).
 */
#ifndef DFPT2_H
#define DFPT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* dfpt2_stream_t; /* a hipStream_t */

typedef enum {
  DFPT2_OK = 0,
  DFPT2_ERR_INVALID_ARG = -1,   /* null pointer, bad size, s <= 0, p_o outside (0,1], ... */
  DFPT2_ERR_WORKSPACE = -2,     /* ws_bytes smaller than the queried size */
  DFPT2_ERR_HIP = -3,           /* a HIP runtime call or kernel launch failed */
  DFPT2_ERR_NOT_CONVERGED = -4, /* the eigensolver hit its iteration cap */
  DFPT2_ERR_NONFINITE = -5,     /* a non-finite energy or occupation was produced */
  DFPT2_ERR_UNSUPPORTED = -6    /* option combination not implemented */
} dfpt2_status;

typedef enum {
  DFPT2_FP64 = 0,         /* FP64 MFMA for both contractions */
  DFPT2_BF16_SLICED = 1,  /* B and T split into BF16 slices; exact FP32 chunk sums, FP64 across chunks */
  DFPT2_FP8_SLICED = 2,   /* FP8 e4m3 slices with per-block power-of-two scales.  Measured and
                             offered beside the others, but OUTSIDE the 1e-6 Eh energy contract of
                             the mixed paths: products of differently scaled 32-element blocks meet
                             in one FP32 accumulator, so the sums are not exact; the relative energy
                             error is about 1e-8 .. 3e-7 at 4 slices (bounded by 8 x 2^-(5 slices - 1)),
                             i.e. up to ~1e-2 Eh on the 1e6 - 1e8 Eh energies of large inputs */
  DFPT2_INT8_SLICED = 3   /* B and T as balanced base-256 INT8 digits per row; exact INT32 level sums on
                             the INT8 MFMA (n_aux <= 26208 at 5 digits) */
} dfpt2_precision;

typedef struct dfpt2_opts {
  int64_t n_core;   /* correlated core holes (doubly occupied) */
  int64_t n_act;    /* active holes; their density is gamma_act */
  int64_t n_vir;    /* virtual orbitals */
  int64_t n_aux;    /* auxiliary (density-fitting) functions */
  double  s;        /* DSRG flow parameter s (Eh^-2), > 0 */
  int32_t precision;          /* dfpt2_precision */
  int32_t slices_gemm1;       /* slices per operand of V = B B^T; 0 = precision default
                               (BF16, FP8: 4, range 2..4; INT8: 5 digits, range 3..5) */
  int32_t slices_gemm2;       /* slices per operand of the density product: 0 = precision default
                               (BF16: 4 BF16 slices; INT8: 5 INT8 digits; FP64, FP8: FP64 density),
                               1 = FP64 density, 2..4 BF16 slices (BF16), 2..5 digits (INT8) */
  int32_t density_convention; /* 0: spin-summed Gamma^(2)_vv (Eq. A9); 1: per spin (half) */
  int64_t pair_batch;         /* unordered pairs per batch; 0 = library default */
} dfpt2_opts;

/* Message for the calling thread's last failing call ("" if none).  Host string,
 * owned by the library, valid until the next call on the same thread. */
const char* dfpt2_last_error(void);
const char* dfpt2_status_string(int status);
/* Library version string (host, static). */
const char* dfpt2_version(void);

/* Workspace (bytes) needed by dfpt2_build_vv_density for these options.
 * bytes: host out. */
int dfpt2_workspace_size(const dfpt2_opts* opts, size_t* bytes);

/*
 * The DF-DSRG-PT2 pass: energy and virtual 1-RDM (App. A Eqs. A7, A9; Eq. 7).
 *   opts        host pointer to the options
 *   eps_hole    [n_h]            semicanonical hole energies (core, then active)
 *   eps_vir     [n_vir]          semicanonical virtual energies, ascending
 *   gamma_act   [n_act*n_act]    spin-summed active 1-RDM, symmetric; NULL iff n_act == 0
 *   B           [n_h][n_vir][n_aux] FP64 three-index integrals
 *   pair_mask   [n_h*n_h] uint8, symmetric, 1 = compute the pair; NULL = all pairs.
 *               A masked pair contributes nothing to E and D.  Masks are honoured
 *               for core-core pairs; pairs with an active hole are always computed.
 *   D_vv        [n_vir*n_vir] out, symmetric
 *   e_pt2       [2] out, the energy as a double-double (hi, lo)
 *   pair_energy [n_h*n_h] out or NULL: <Vr_ij, 2T_ij - T_ij^T> of each core-core
 *               ordered pair (symmetric); 0 for masked pairs, NaN for pairs with an
 *               active hole
 *   pair_tnorm  [n_h*n_h] out or NULL: ||T_ij||_F (float), symmetric
 *   workspace   device scratch of ws_bytes bytes (see dfpt2_workspace_size)
 * Errors: INVALID_ARG, WORKSPACE, HIP, NONFINITE (energy not finite), UNSUPPORTED.
 */
int dfpt2_build_vv_density(const dfpt2_opts* opts,
                           const double* eps_hole, const double* eps_vir,
                           const double* gamma_act, const double* B,
                           const uint8_t* pair_mask,
                           double* D_vv, double* e_pt2,
                           double* pair_energy, float* pair_tnorm,
                           void* workspace, size_t ws_bytes, dfpt2_stream_t stream);

/*
 * dfpt2_build_vv_density for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as dfpt2_build_vv_density minus the
 * workspace: the pass runs in the library's static device scratch of
 * DFPT2_STATIC_SCRATCH_BYTES per GPU (reserved when the library first uses that
 * GPU, held until the process ends).  The call allocates nothing (leave the
 * stage timers off: enabled, they create HIP events); a pass whose workspace
 * (dfpt2_workspace_size) exceeds the scratch returns DFPT2_ERR_WORKSPACE and
 * launches nothing -- a smaller pair_batch shrinks the need.  The scratch is
 * shared by every call on one GPU and keeps the last call's contents (the pass
 * initializes what it reads): calls that overlap on one GPU (other host threads
 * or streams) race and must be serialized by the caller.  `stream` must belong
 * to the current device.
 */
#define DFPT2_STATIC_SCRATCH_BYTES (64ull << 20)
int dfpt2_build_vv_density_noalloc(const dfpt2_opts* opts,
                                   const double* eps_hole, const double* eps_vir,
                                   const double* gamma_act, const double* B,
                                   const uint8_t* pair_mask,
                                   double* D_vv, double* e_pt2,
                                   double* pair_energy, float* pair_tnorm,
                                   dfpt2_stream_t stream);

/* Workspace (bytes) for fno_truncate / dfpt2_eigh_sym at dimension n.  bytes: host out. */
int fno_truncate_workspace_size(int64_t n_vir, size_t* bytes);

/*
 * Natural orbitals and truncation (Eqs. 8 and 10; near-degeneracy rule of Sec. 2).
 *   D_vv          [n_vir*n_vir] symmetric input (not modified)
 *   p_o           cumulative-occupation threshold in (0, 1]
 *   degen_rel_tol 0 disables the near-degeneracy widening; > 0 keeps adding NOs p
 *                 beyond the cut while n_last - n_p < degen_rel_tol * n_last, with
 *                 n_last the smallest occupation the threshold kept (anchored reading)
 *   occ           [n_vir] out, occupation numbers in descending order
 *   no_vecs       [n_vir*n_vir] out, column k is the NO of occ[k], oriented so that
 *                 its largest-magnitude component is positive
 *   n_kept        host out, N'
 *   margins       host out [2] or NULL: (p_o - c(N'-1), c(N') - p_o), c = cumulative
 *                 occupation fraction
 * Errors: INVALID_ARG, WORKSPACE, HIP, NOT_CONVERGED, NONFINITE.
 */
int fno_truncate(const double* D_vv, int64_t n_vir, double p_o, double degen_rel_tol,
                 double* occ, double* no_vecs, int64_t* n_kept, double* margins,
                 void* workspace, size_t ws_bytes, dfpt2_stream_t stream);

/* Truncation rules for fno_truncate_rule. */
typedef enum {
  DFPT2_TRUNC_CUMULATIVE = 0, /* param = p_o in (0, 1]: smallest N' whose cumulative occupation
                                 reaches p_o of the total (Eq. 10); the rule of fno_truncate */
  DFPT2_TRUNC_FRACTION = 1,   /* param = p_v in (0, 1]: N' = ceil(p_v n_vir), a fixed fraction of
                                 the virtuals (Eq. 9) */
  DFPT2_TRUNC_CUTOFF = 2,     /* param = n_kappa: keep every NO whose occupation is >= n_kappa
                                 (the occupation cutoff of Sec. 2); N' may be 0 */
  DFPT2_TRUNC_FIXED = 3       /* param = N', an integer in [1, n_vir]: the same N' at every
                                 geometry of a scan (Sec. 2 on the PES discontinuity) */
} dfpt2_trunc_rule;

/*
 * Natural orbitals and truncation by any rule of dfpt2_trunc_rule, then the same
 * optional near-degeneracy widening as fno_truncate.  Arguments as for
 * fno_truncate, plus rule and param.  margins (host out [2] or NULL): for the
 * cumulative rule as in fno_truncate; for the cutoff rule (n[N'-1] - n_kappa,
 * n_kappa - n[N']); for the other rules the occupations either side of the cut
 * (n[N'-1], n[N']); +inf where a neighbour does not exist.
 * Errors: INVALID_ARG (unknown rule or parameter out of range), WORKSPACE, HIP,
 * NOT_CONVERGED, NONFINITE.
 */
int fno_truncate_rule(const double* D_vv, int64_t n_vir, int rule, double param, double degen_rel_tol,
                      double* occ, double* no_vecs, int64_t* n_kept, double* margins,
                      void* workspace, size_t ws_bytes, dfpt2_stream_t stream);

/* Workspace (bytes) for dfpt2_add_active_particle_density.  bytes: host out. */
int dfpt2_active_particle_workspace_size(const dfpt2_opts* opts, size_t* bytes);

/*
 * Adds to D_vv the Eq. A9 terms whose amplitudes carry one virtual and one active
 * particle index (the multireference amplitudes t^{ex}_{ij} of Eq. A7 with x active),
 * at zero density cumulants and without singles:
 *     t^{ev}_{mn} tc^{fu}_{mn} eta^u_v + 1/2 S(t^{ey}_{mu} tc^{fx}_{mv}) Gamma^u_v eta^x_y
 *   + 1/4 t^{ez}_{ux} tc^{fw}_{vy} Gamma^u_v Gamma^x_y eta^w_z,      eta = 2 - Gamma_act
 * (the active-active term with the exchange combination tc on its second amplitude).
 *   opts       as for dfpt2_build_vv_density (s, sizes, density_convention)
 *   eps_hole   [n_core + n_act] (the active energies are those of the active particles too)
 *   eps_vir, gamma_act, B   as for dfpt2_build_vv_density
 *   B_act      [n_h][n_act][n_aux] density-fitted integrals B^Q_ix of hole i and active
 *              particle x (symmetric in the active-active block, as such integrals are)
 *   D_vv       [n_vir][n_vir] in/out: the terms are added, symmetrized
 * Does nothing when n_act = 0.  FP64 throughout.  Asynchronous on the stream.
 * Errors: INVALID_ARG, WORKSPACE, HIP.
 */
int dfpt2_add_active_particle_density(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir,
                                      const double* gamma_act, const double* B, const double* B_act, double* D_vv,
                                      void* workspace, size_t ws_bytes, dfpt2_stream_t stream);

/* Workspace (bytes) for dfpt2_add_cumulant_singles_density, with (with_lambda != 0)
 * or without a cumulant.  bytes: host out. */
int dfpt2_cumulant_singles_workspace_size(const dfpt2_opts* opts, int with_lambda, size_t* bytes);

/*
 * Adds to D_vv the Eq. A9 terms with the first-order singles and with the two-body
 * density cumulant lambda of the reference:
 *     2 t_e^m t_f^m + t_e^u t_f^v gamma_u^v + (t_e^u t_fv^xy + t_ey^uv t_f^x) lambda_uv^xy
 *   + t_ee'^uv t_fe'^xy lambda_uv^xy + P(t_ey^mv t_fu^mx) lambda_uv^xy
 *   + 1/2 t_ez^uv t_fw^xy eta_w^z lambda_uv^xy + 1/2 P(t_ey^wv t_fu^zx) gamma_w^z lambda_uv^xy
 * (t_ab^ij the amplitude of a+_a a+_b a_j a_i; m core, u..z active, e, f, e' virtual;
 * eta = 2 - gamma; P(t_ap^ij t_cd^kq) = 2 t_ap^ij t_cd^kq - t_ap^ij t_cd^qk - t_ap^ji t_cd^kq
 * - t_aq^ji t_cd^pk), with the singles of Eq. A6 in the semicanonical model (f_ai = 0):
 *     t_e^i = 1/2 sum_ux (eps_x - eps_u) gamma_x^u (2 t_ex^iu - t_ex^ui) (1 - e^{-s D^2}) / D,
 *     D = eps_i - eps_e.
 * The three-body-cumulant term is left out, as in the method (Sec. 2).  Together with
 * dfpt2_build_vv_density and dfpt2_add_active_particle_density this is every term of
 * Eq. A9 but that one.
 *   opts        as for dfpt2_add_active_particle_density
 *   eps_hole, eps_vir, gamma_act, B, B_act   as for dfpt2_add_active_particle_density
 *   lambda_act  [n_act^4] spin-free cumulant lambda_uv^xy at [((u n_act + v) n_act + x) n_act + y],
 *               symmetric under (u v)(x y) -> (v u)(y x) and (u v) <-> (x y); NULL adds only the
 *               singles terms
 *   D_vv        [n_vir][n_vir] in/out: the terms are added, symmetrized
 *   t1          [n_h][n_vir] out or NULL: the singles t_e^i (row i)
 * Does nothing when n_act = 0 (no source for singles, no cumulant).  FP64 throughout.
 * Asynchronous on the stream.  Errors: INVALID_ARG, WORKSPACE, HIP.
 */
int dfpt2_add_cumulant_singles_density(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir,
                                       const double* gamma_act, const double* lambda_act, const double* B,
                                       const double* B_act, double* D_vv, double* t1, void* workspace,
                                       size_t ws_bytes, dfpt2_stream_t stream);

/* Workspace (bytes) for naf_compress (sizes from opts).  bytes: host out. */
int naf_compress_workspace_size(const dfpt2_opts* opts, size_t* bytes);

/*
 * Natural auxiliary functions (the auxiliary-basis compression the paper's
 * conclusions propose for this pass; Kallay's NAFs): with J[(i,a), P] = B^P_ia,
 * W = J^T J = U diag(sigma) U^T (sigma descending), keep the n_naf functions
 * with sigma_k > eps sigma_0 (a threshold relative to the largest eigenvalue;
 * eps <= 0 keeps all: then V = B B^T is reproduced to rounding) and form
 * B~^k_ia = sum_P B^P_ia U_Pk.
 *   opts    sizes only (n_core + n_act holes, n_vir, n_aux <= 16384)
 *   B       [n_h][n_vir][n_aux] as for dfpt2_build_vv_density
 *   B_naf   [n_h][n_vir][n_aux] capacity, out [n_h][n_vir][n_naf]: pass it with
 *           n_aux = n_naf to dfpt2_build_vv_density / pt2_energy_correction
 *   sigma   [n_aux] out, eigenvalues of W, descending
 *   n_naf   host out
 * Synchronizes the stream.  Errors: INVALID_ARG (also when eps removes every
 * function), WORKSPACE, HIP, NOT_CONVERGED, NONFINITE.
 */
int naf_compress(const dfpt2_opts* opts, const double* B, double eps, double* B_naf, double* sigma,
                 int64_t* n_naf, void* workspace, size_t ws_bytes, dfpt2_stream_t stream);

/*
 * Density-fitted particle-particle ladder, the N_C^2 N_V^4 part of the two-body
 * contraction of the high-level step (Eq. 6) whose cost the FNO truncation cuts
 * by (N_V'/N_V)^4 (Sec. 2):
 *     R^p_ab = sum_cd (ac|bd) T^p_cd,   (ac|bd) = sum_Q B^Q_ac B^Q_bd,
 * for n_amp amplitude matrices T^p (one per hole pair), FP64 throughout.  With X
 * (the kept NOs as columns, e.g. from fno_truncate) the inputs are first
 * transformed, B'^Q = X^T B^Q X and T'^p = X^T T^p X, and R is the ladder in the
 * truncated space.
 *   B_vv   [n_vir][n_vir][n_aux] density-fitted virtual-virtual integrals; must be
 *          symmetric in the two virtual indices (B^Q_ac = B^Q_ca), as such
 *          integrals are: the library reads (ac|bd) as (ac|db)
 *   T      [n_amp][n_vir][n_vir]
 *   X      [n_vir][ldx] or NULL: the first n_kept columns are the kept NOs (fno_truncate's
 *          no_vecs with ldx = n_vir); NULL = full space (n_kept = 0 or n_vir, ldx ignored)
 *   R      [n_amp][m][m] out, m = n_kept with X, else n_vir
 * Limits: n_vir <= 2048, n_amp <= 65535.  Workspace (pp_ladder_workspace_size,
 * n_kept = 0 for the full space): one block of (ac|bd) of up to ~16 GB plus the
 * transformed inputs.  Asynchronous on the stream.
 * Errors: INVALID_ARG, WORKSPACE, HIP.
 */
int pp_ladder_workspace_size(int64_t n_vir, int64_t n_aux, int64_t n_amp, int64_t n_kept, size_t* bytes);
int pp_ladder(int64_t n_vir, int64_t n_aux, int64_t n_amp, const double* B_vv, const double* T, const double* X,
              int64_t ldx, int64_t n_kept, double* R, void* workspace, size_t ws_bytes, dfpt2_stream_t stream);

/* Symmetric FP64 eigensolver used by fno_truncate (Eq. 8) and the
 * recanonicalization: A [n*n] symmetric (not modified); w [n] out ascending;
 * Z [n*n] out, column k is the eigenvector of w[k]. */
int dfpt2_eigh_sym(const double* A, int64_t n, double* w, double* Z,
                   void* workspace, size_t ws_bytes, dfpt2_stream_t stream);

/* Workspace (bytes) for pt2_energy_correction.  bytes: host out. */
int pt2_correction_workspace_size(const dfpt2_opts* opts, int64_t n_kept, size_t* bytes);

/*
 * Additive PT2 correction (Eq. 11, scalar part) for a truncated virtual space.
 *   opts, eps_hole, eps_vir, gamma_act, B   as for dfpt2_build_vv_density
 *   no_vecs     [n_vir*n_vir] NOs (columns, descending occupation) from fno_truncate
 *   n_kept      N', 1 <= N' <= n_vir; the first N' columns span the kept space
 *   e_full      [2] the full-space energy (double-double) from dfpt2_build_vv_density
 *   e_kept      [2] out, E_PT2 in the recanonicalized kept basis
 *   correction  [2] out, e_full - e_kept
 * The kept space is recanonicalized: F' = V_k^T diag(eps_vir) V_k = W diag(eps~) W^T,
 * U = V_k W, B~_i = U^T B_i, and the pass is repeated with (eps~, B~) in the arithmetic
 * opts->precision names.  It need not be the build's: after a BF16 build, INT8 digits
 * (exact integer sums) hold the correction within 1e-6 Eh up to 120 + 12 holes, 2000
 * virtuals and 6000 auxiliary functions, where a BF16 kept-space pass is off by ~2e-6 Eh.
 * Errors: INVALID_ARG, WORKSPACE, HIP, NOT_CONVERGED, NONFINITE, UNSUPPORTED.
 */
int pt2_energy_correction(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir,
                          const double* gamma_act, const double* B, const double* no_vecs,
                          int64_t n_kept, const double* e_full, double* e_kept,
                          double* correction, void* workspace, size_t ws_bytes,
                          dfpt2_stream_t stream);

/*
 * Learned pair screening (not part of the paper's method).  A small network
 * predicts ||t_ij||_F of every unordered core pair before the pass and the
 * mask drops pairs predicted below a threshold; the unscreened pass is the
 * reference it is judged against.  Pair order everywhere: unordered core pairs
 * i <= j, row-major (n_up = n_core (n_core + 1) / 2 entries).
 *
 * Pair quantities (q_iQ = ||B^Q_i.||_2 over virtuals):
 *   U_ij = sum_Q q_iQ q_jQ >= ||V_ij||_F (rigorous), W_ij = (sum_Q q_iQ^2 q_jQ^2)^(1/2),
 *   g_ij = max |1 - e^{-s D^2}| / |D| over the pair's denominators D (Eq. A7),
 *   ||t_ij||_F <= g_ij U_ij.
 * Features (float, [n_up][5]):
 *   (e_i, e_j, log(U/W), 0.1 (log W_ij - (log W_ii + log W_jj)/2), 0.1 log(g W)).
 * log_scale (double, [n_up][2]) = (log(g_ij W_ij), log(g_ij U_ij)).
 * Network: 5 -> 64 (tanh) -> 64 (tanh) -> 1, FP32 parameters packed as
 *   [W1 64x5 row-major, b1 64, W2 64x64, b2 64, w3 64, b3 1] (pairscreen_num_params()).
 * The network output is y = log ||t_ij||_F - log(g_ij W_ij).
 */
int pairscreen_num_params(void);
/* Workspace for pairscreen_features.  bytes: host out. */
int pairscreen_workspace_size(const dfpt2_opts* opts, size_t* bytes);
/* eps_hole [n_h], eps_vir [n_vir] ascending, B [n_h][n_vir][n_aux]; feats, log_scale out. */
int pairscreen_features(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir,
                        const double* B, float* feats, double* log_scale,
                        void* workspace, size_t ws_bytes, dfpt2_stream_t stream);
/* Forward pass for n samples: W [num_params], feats [n][5] -> pred [n];
 * act_cache [n][128] out (hidden activations for the backward pass) or NULL. */
int pairscreen_mlp_forward(const float* W, const float* feats, int64_t n, float* pred, float* act_cache,
                           dfpt2_stream_t stream);
/* Gradient of sum_n dpred_n pred_n: dW [num_params] out.  Workspace from
 * pairscreen_backward_workspace_size(n). */
int pairscreen_backward_workspace_size(int64_t n, size_t* bytes);
int pairscreen_mlp_backward(const float* W, const float* feats, const float* act_cache, const float* dpred,
                            int64_t n, float* dW, void* workspace, size_t ws_bytes, dfpt2_stream_t stream);
/* One Adam update (bias-corrected, step >= 1) of W with gradient dW and moments m, v. */
int pairscreen_adam_step(float* W, const float* dW, float* m, float* v, int64_t n_params, float lr, float b1,
                         float b2, float eps, int64_t step, dfpt2_stream_t stream);
/* Full-batch training: `steps` iterations of forward, mean squared error against
 * y [n], backward and Adam (b1 0.9, b2 0.999, eps 1e-8, steps numbered from
 * step0 + 1); losses [steps] out (device).  Synchronizes the stream. */
int pairscreen_train_workspace_size(int64_t n, size_t* bytes);
int pairscreen_train(float* W, float* m, float* v, const float* feats, const float* y, int64_t n, int64_t steps,
                     int64_t step0, float lr, float* losses, void* workspace, size_t ws_bytes,
                     dfpt2_stream_t stream);
/* Training targets y [n_up] = log ||t_ij||_F - log(g_ij W_ij) from the pass's pair_tnorm [n_h][n_h]. */
int pairscreen_targets(const float* pair_tnorm, const double* log_scale, int64_t n_core, int64_t n_h, float* y,
                       dfpt2_stream_t stream);
/* Pair mask [n_h][n_h] for dfpt2_build_vv_density: 1 everywhere except core pairs with
 *   mode 0 (network): log(g W) + pred + margin < log(threshold)
 *   mode 1 (rigorous bound): log(g U) < log(threshold).
 * n_dropped: host out (unordered pairs dropped) or NULL (then no synchronization).
 * workspace: >= 64 bytes of device scratch. */
int pairscreen_build_mask(const float* pred, const double* log_scale, int64_t n_core, int64_t n_h,
                          double threshold, double margin, int mode, uint8_t* mask, int64_t* n_dropped,
                          void* workspace, size_t ws_bytes, dfpt2_stream_t stream);

/*
 * Stage timers for measurement (not part of the method).  When enabled, every
 * entry point brackets its kernel launches with HIP events on the stream it was
 * given and, at its next stream synchronization, adds the elapsed GPU time to
 * the stage counters below.  Counters, and the enabled flag, are per host thread
 * (thread-local): a thread enables and reads its own, and only the calls it makes
 * are timed, so the library keeps no state shared between threads.
 * dfpt2_profile_enable(1) also resets the calling thread's counters.
 *   ms        host out [DFPT2_NSTAGE], accumulated milliseconds per stage
 *   launches  host out [DFPT2_NSTAGE], number of timed launches per stage
 */
enum {
  DFPT2_STAGE_PAIR = 0,       /* pair product V = B_i B_j^T of the core pairs (with the fused
                                 regularizer/energy epilogue where the product and the epilogue
                                 share a kernel) */
  DFPT2_STAGE_DENSITY = 1,    /* density kernel (D_vv accumulation) of the core pairs */
  DFPT2_STAGE_SPLIT = 2,      /* operand splitting into BF16/FP8 slices */
  DFPT2_STAGE_REDUCE = 3,     /* pair lists, reductions, finalization */
  DFPT2_STAGE_ACTIVE = 4,     /* pairs with an active hole in the D_vv pass: their product, epilogue,
                                 rotation to the natural active orbitals, energy, amplitude split
                                 and density */
  DFPT2_STAGE_EIGH = 5,       /* symmetric eigensolver */
  DFPT2_STAGE_TRANSFORM = 6,  /* recanonicalization GEMMs and B transform */
  DFPT2_STAGE_KEPT_PAIR = 7,  /* the kept-space energy's pair kernels (product and epilogue),
                                 core and active holes */
  DFPT2_STAGE_SCREEN = 8,     /* pair features, MLP, mask compaction */
  DFPT2_STAGE_SPLIT_T = 9,    /* amplitude splitting into BF16 slices for the density */
  DFPT2_STAGE_LADDER_TRANSFORM = 10, /* particle-particle ladder: inputs to the kept NO basis */
  DFPT2_STAGE_LADDER = 11,    /* particle-particle ladder: integral and contraction GEMMs */
  DFPT2_STAGE_PAIR_EPILOGUE = 12, /* the D_vv pass's regularizer/energy epilogue, where it runs as
                                     a kernel of its own */
  DFPT2_NSTAGE = 13
};
int dfpt2_profile_enable(int on);
int dfpt2_profile_read(double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* DFPT2_H */
