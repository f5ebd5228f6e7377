/*
 * hisq.h -- C ABI of the MI355X (gfx950) multi-right-hand-side HISQ Dslash and even-odd CG.
 *
 * Operator (Kaczmarek et al., "HISQ inverter on Intel Xeon Phi and NVIDIA GPUs", Section 1,
 * Eq. 3; several right-hand sides at once as in Eq. 4):
 *
 *   w(x) = sum_{mu=0..3} [ X(x,mu) v(x+mu) - X(x-mu,mu)^dag v(x-mu)
 *                        + N(x,mu) v(x+3mu) - N(x-3mu,mu)^dag v(x-3mu) ]
 *
 * on a periodic lattice of extents dims = {Lx, Ly, Lz, Lt} (each even, >= 4).  Staggered phases
 * and boundary signs are folded into the links X (fat) and N (Naik) by the caller.  D only
 * couples sites of opposite parity (parity = (x+y+z+t) mod 2), D = [[0, D_eo], [D_oe, 0]], and
 * the solver works on the even-site normal operator M = m^2 - D_eo D_oe (Hermitian positive
 * definite because D_eo = -D_oe^dag).
 *
 * Layouts (all little-endian, no padding):
 *   links  : [V][4][3][3] complex128 (re, im interleaved), sites in lexicographic order
 *            lex = x + Lx*(y + Ly*(z + Lz*t)), direction mu = 0..3 is x, y, z, t, each 3x3
 *            matrix row-major.  V = Lx*Ly*Lz*Lt.
 *   vectors: [n][3][V/2] complex (complex128 for HISQ_F64, complex64 otherwise) on the sites of
 *            one parity: right-hand side major, then colour, then site; the site index within a
 *            parity is lex >> 1.  Right-hand side i of a bundle is therefore a pointer offset of
 *            i*3*(V/2) complex elements.  Vector pointers must be multiples of their complex
 *            element size (8 bytes for complex64, 16 for complex128; HISQ_ERR_ARG otherwise).
 *
 * Ownership and streams: every vector pointer is device memory owned by the caller.  The
 * context copies the links on hisq_load_links (the caller may free its buffers afterwards) and
 * owns its workspace.  Work is enqueued on the context's HIP stream; hisq_dslash_mrhs,
 * hisq_apply_m and hisq_dot_mrhs return without synchronising, hisq_cg_mrhs and the network
 * training/evaluation calls synchronise before returning.  A context is not thread-safe.
 *
 * Errors: every int-returning call returns HISQ_OK (0) or a negative code and never throws;
 * hisq_last_error() gives the message of the context's last failing call.
 */
#ifndef HISQ_H
#define HISQ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HISQ_OK = 0,
  HISQ_ERR_ARG = -1,       /* bad argument: dims, null pointer, n out of range, bad enum      */
  HISQ_ERR_STATE = -2,     /* call out of order, e.g. no links loaded / no network initialised */
  HISQ_ERR_HIP = -3,       /* HIP runtime failure; message holds the hipError string          */
  HISQ_ERR_OOM = -4,       /* device allocation failed                                        */
  HISQ_ERR_NOCONV = -5,    /* a right-hand side missed tol; x and the stats are still valid   */
  HISQ_ERR_NONFINITE = -6, /* non-finite input or breakdown of the iteration                  */
  HISQ_ERR_IO = -7         /* file could not be read or written                               */
};

/* Precision of a Dslash application: vectors complex128 + FP64 links (HISQ_F64); vectors
 * complex64 + FP32 links (HISQ_F32); vectors complex64 + FP16 link storage, FP32 arithmetic
 * (HISQ_F16). */
enum { HISQ_F64 = 0, HISQ_F32 = 1, HISQ_F16 = 2 };

/* Bit mask of link copies hisq_load_links builds. */
enum { HISQ_LINKS_F64 = 1, HISQ_LINKS_F32 = 2, HISQ_LINKS_F16 = 4, HISQ_LINKS_ALL = 7 };

/* Solver kinds of hisq_cg_mrhs. */
enum { HISQ_CG_F64 = 0, HISQ_CG_MIXED = 1, HISQ_FCG_NN = 2 };

#define HISQ_MAX_RHS 64

typedef struct hisq_ctx hisq_ctx;

/* Create a context for a lattice of extents dims on HIP device `device`, enqueueing on
 * `hip_stream` (a hipStream_t; NULL = the null stream).  Returns HISQ_ERR_ARG for odd extents or
 * extents below 4, HISQ_ERR_HIP if the device cannot be selected. */
int hisq_create(hisq_ctx **ctx, const int dims[4], int device, void *hip_stream);

/* Free the context, its link copies and its workspace.  NULL is accepted. */
int hisq_destroy(hisq_ctx *ctx);

/* Message of the last failing call on this context ("" if none); NULL ctx gives the message of
 * the last failing hisq_create.  The pointer stays valid until the next call on the context. */
const char *hisq_last_error(const hisq_ctx *ctx);

/* Change the stream later calls enqueue on. */
int hisq_set_stream(hisq_ctx *ctx, void *hip_stream);

/* Copy the fat links X and Naik links N (Section 1, Eq. 3) into the context.
 *   fat, naik : [V][4][3][3] complex128, host or device memory (detected), read only.
 *   copies    : HISQ_LINKS_* mask of device copies to build (FP64 is needed by HISQ_F64 calls
 *               and by the FP64 parts of every solver).
 *   naik_recon: reals stored per Naik link in the FP32 and FP16 copies (Section 1 names Naik
 *               reconstructions from 9 or 13/14 reals, Section 2 uses 14; the FP64 copy always
 *               keeps 18):
 *               18: all 18 reals;
 *               14: rows 0 and 1 of N plus one complex z, row 2 = z * conj(row0 x row1); exact
 *                   for N = c * U with U in U(3);
 *               13: rows 0 and 1 plus one real z (the same with z real); exact for N = c * U
 *                   with c real and U in SU(3) (z = 1 / c);
 *                9: N = c * U with c real and U in SU(3): u01, u02, u10, arg u00, arg u20 and c;
 *                   |u00|, |u20| come from the unit norms of row 0 and column 0 and the four
 *                   other entries from unitarity and det U = 1.
 *               The call fails with HISQ_ERR_ARG if the given Naik links are not of the form the
 *               format needs (relative reconstruction error above 1e-10).  The 13- and 9-real
 *               formats run in the register-tile and 64-site LDS forms of the Dslash (not the
 *               32-site or direction-pipelined forms, lds_links 4-6).
 * Non-finite link entries give HISQ_ERR_NONFINITE.  Replaces earlier links. */
int hisq_load_links(hisq_ctx *ctx, const double *fat, const double *naik, int copies, int naik_recon);

/* Multi-rhs half Dslash (Section 1, Eq. 3 and Eq. 4): out = D_{out_parity, 1-out_parity} in.
 *   out_parity: 1 gives D_oe (even -> odd), 0 gives D_eo (odd -> even).
 *   prec      : HISQ_F64 / HISQ_F32 / HISQ_F16 (see above; the matching link copy must exist).
 *   n         : number of right-hand sides, 1..HISQ_MAX_RHS.
 *   in        : device [n][3][V/2] complex on parity 1-out_parity.
 *   out       : device [n][3][V/2] complex on out_parity; must not alias in.
 * The links are read once per site for all n right-hand sides.  Each output is bit-identical to
 * the output of n separate single-rhs calls.  Asynchronous on the context stream. */
int hisq_dslash_mrhs(hisq_ctx *ctx, int out_parity, int prec, int n, const void *in, void *out);

/* Even-site normal operator out = m^2 in - D_eo (D_oe in) for n right-hand sides (the operator
 * of the even-odd CG).  in/out: device [n][3][V/2] complex on even sites, not aliased.  If
 * pq_out is not NULL it receives (device, n doubles) Re<in, out> per right-hand side,
 * accumulated in FP64.  Asynchronous. */
int hisq_apply_m(hisq_ctx *ctx, int prec, double mass, int n, const void *in, void *out, double *pq_out);

/* Per-rhs inner products dots[i] = <a_i, b_i> = sum conj(a) b over the 3*V/2 components of one
 * parity, accumulated in FP64 (deterministic fixed-order tree).  a, b: device [n][3][V/2]
 * complex of precision prec (HISQ_F64: complex128, else complex64).  dots: device, 2*n doubles
 * (re, im).  Asynchronous. */
int hisq_dot_mrhs(hisq_ctx *ctx, int prec, int n, const void *a, const void *b, double *dots);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): hisq_dot_mrhs with the same arguments, kernels and
 * bit-identical results, which allocates nothing.  Its per-block partials go to a static device
 * buffer of the library (8 MiB, 2^20 doubles, one per GPU, held until the process ends) instead
 * of the context workspace.  It needs 2 * n * ceil(3 * (V/2) / 1024) <= 2^20 doubles (e.g. every
 * n <= 64 up to 48^3 x 24 sites, n <= 85 at 64^3 x 16) and returns HISQ_ERR_ARG beyond that.
 * Every call on a GPU shares that GPU's buffer: calls that overlap in time on one GPU (other
 * streams or contexts) race and must be serialised by the caller; each call writes all the
 * partials it reads, so nothing carries over between calls.  Asynchronous. */
int hisq_dot_mrhs_noalloc(hisq_ctx *ctx, int prec, int n, const void *a, const void *b, double *dots);

/* Launch configuration of the multi-rhs half Dslash.  Section 2 blocks the rhs in registers,
 * blocks sites x rhs in 2-d thread blocks, combines both, and picks the best launch
 * configuration for the GPU, the lattice size and n by automatic tuning.  The library does the
 * same: each (precision, n, plain or fused-M form) is tuned on first use (a few ms of scratch
 * launches) unless the environment sets HISQ_AUTOTUNE=0 (then a fixed heuristic is used) or a
 * configuration is forced.  Every configuration gives bit-identical Dslash output. */
typedef struct {
  int rhs_per_thread;    /* register tile: 1, 2, 4, 8 or 16 (FP64 and the fused-M form: <= 8)  */
  int sites_per_block;   /* 256: one rhs tile per 256-thread workgroup; 64: the 4 waves of a     */
                         /*      workgroup take 4 rhs tiles of the same 64 sites; 32: the       */
                         /*      32-site LDS form (lds_links 1 or 2 = 4 or 8 waves, rhs_per_    */
                         /*      thread 1 or 2, the two halves of a wave on different rhs), for */
                         /*      the plain half Dslash only: hisq_set_launch leaves the fused-M */
                         /*      configuration unchanged for it                                 */
  int nontemporal_links; /* 1: link loads carry the non-temporal cache hint                     */
  int lds_links;         /* 1, 2, 3: a workgroup of 64 sites x 4, 8, 16 waves stages its sites'  */
                         /*    links in LDS and its waves loop over the rhs tiles (requires      */
                         /*    sites_per_block = 64, rhs_per_thread <= 4 (<= 2 for 16 waves);    */
                         /*    FP64 links take a CU's LDS alone, FP32/FP16 links fit twice);     */
                         /* 4, 5, 6: the same with the links staged one direction at a time in  */
                         /*    two LDS buffers, the next direction loading while the current one */
                         /*    is applied; 16 waves x 1 rhs tile (4), 16 x 2 (5), 8 x 2 (6), so  */
                         /*    n <= 16, 32, 16 rhs tiles; rhs_per_thread <= 2; not FP64          */
  int xcd_map;           /* LDS form only: 0 = each XCD takes a contiguous range of sites; 1 =    */
                         /*    each XCD takes Lz/8 z slices for all t (needs (Lx/2)*Ly % 64 == 0 */
                         /*    and Lz % 8 == 0); 2 = each XCD takes 1/8 of the 64-site blocks of */
                         /*    every (z, t) plane, z-major (needs (Lx/2)*Ly % 512 == 0); 3 = the */
                         /*    same blocks walked in z tiles of 4 slices, t within a tile (also  */
                         /*    needs Lz % 4 == 0)                                                */
} hisq_launch;

/* Force the configuration for (prec, n), both forms (the fused-M form clamps rhs_per_thread to
 * its limit); cfg = NULL restores automatic tuning.  HISQ_ERR_ARG for an invalid configuration. */
int hisq_set_launch(hisq_ctx *ctx, int prec, int n, const hisq_launch *cfg);

/* The configuration the next call with (prec, n, fused_m) uses (the heuristic if not tuned yet). */
int hisq_get_launch(hisq_ctx *ctx, int prec, int n, int fused_m, hisq_launch *cfg);

/* Tune (prec, n, fused_m) now: time every valid configuration on scratch vectors and keep the
 * fastest.  best and ms_out (mean ms per launch) may be NULL.  Synchronises the stream. */
int hisq_autotune(hisq_ctx *ctx, int prec, int n, int fused_m, hisq_launch *best, double *ms_out);

/* Save the tuned configurations of this context (its lattice and link formats) to a text file,
 * keeping the file's entries for other lattices; load the entries that match this context's
 * lattice and loaded link formats (call after hisq_load_links; *n_loaded may be NULL).
 * Line format: lx ly lz lt prec recon n fused rt spb nt lds xm ms.  Loading the links again
 * clears tuned (not forced) choices. */
int hisq_save_tuning(hisq_ctx *ctx, const char *path);
int hisq_load_tuning(hisq_ctx *ctx, const char *path, int *n_loaded);

typedef struct {
  int kind;           /* HISQ_CG_F64, HISQ_CG_MIXED or HISQ_FCG_NN                              */
  double tol;         /* stop rhs i when ||b_i - M x_i|| / ||b_i|| <= tol, checked in FP64         */
  int max_iter;       /* iteration cap per right-hand side                                       */
  int reliable_every; /* MIXED/FCG: FP64 true-residual replacement interval in iterations (50)   */
  int link_prec;      /* MIXED/FCG inner operator: HISQ_F32 or HISQ_F16                            */
  int use_x0;         /* 1: x holds the initial guess on entry; 0: start from x = 0                */
  int check_every;    /* host poll interval of the per-rhs residuals, iterations (0 = default 8)  */
  int no_compaction;  /* F64/MIXED: 1 keeps every rhs in its bundle slot to the end; 0 (default)  */
                      /*    repacks the bundle to its live rhs as rhs finish (see hisq_cg_mrhs)  */
} hisq_cg_params;

typedef struct {
  int *iters;          /* [n] iterations done for each rhs (caller-allocated, may be NULL)      */
  double *true_resid;  /* [n] final FP64 ||b - Mx|| / ||b|| (caller-allocated, may be NULL)     */
  int *converged;      /* [n] 1 if rhs i met tol (caller-allocated, may be NULL)                */
  int *fell_back;      /* [n] FCG: 1 if rhs i switched to the mixed solver (may be NULL)         */
  int total_iters;     /* iterations of the bundle loop                                          */
  int reliable_updates;/* FP64 residual replacements done                                        */
  long long dslash_site_rhs; /* sum over half-Dslash launches of (sites x active rhs)           */
  double seconds;      /* wall time of the solve                                                 */
  size_t peak_bytes;   /* most device memory the context held during the solve: link copies,     */
                       /*    workspace, tuning scratch and network state (caller buffers excluded) */
  int link_switch_iter;/* MIXED with FP16 links: iteration at which the inner operator moved to   */
                       /*    the FP32 links (-1: never); see hisq_cg_mrhs                        */
  int compactions;     /* F64/MIXED: times the bundle was repacked to its live rhs (see below)   */
} hisq_cg_stats;

/* Solve M x_i = b_i (M = m^2 - D_eo D_oe on even sites) for n right-hand sides at once; each
 * rhs has its own CG scalars and stops individually (Section 2: the remaining linear algebra
 * is kept separate per rhs so converged rhs can stop).  HISQ_CG_F64 and HISQ_CG_MIXED repack the
 * bundle once a quarter of its slots have finished: finished rhs leave (their solution is written
 * to x), the live ones move to the front, and every later launch works on the smaller bundle
 * with the launch configuration tuned or stored for its size, else with the one of the size
 * before the repack (no autotuning inside the solve); p->no_compaction = 1 turns this off.  A rhs's
 * result does not depend on the repacking or on the other rhs of the bundle.
 *   b : device [n][3][V/2] complex128, even sites.   x : device [n][3][V/2] complex128.
 *   HISQ_CG_F64   : FP64 throughout.
 *   HISQ_CG_MIXED : FP32 Dslash/BLAS body (links p->link_prec), FP64 solution accumulation, FP64
 *                   reductions, FP64 true-residual replacement every p->reliable_every iterations.
 *                   With FP16 links the inner operator moves to the FP32 links (when loaded)
 *                   once the FP16 error dominates: two replacements in a row where the true
 *                   residual exceeds the iterated one by more than 2x in norm while the relative
 *                   residual is still above 1e-5, a stalled true residual, or a falling
 *                   convergence rate (the mean log true residual of the live rhs falls, over the
 *                   last 8 replacements, at less than 0.9 times the best such rate of the solve,
 *                   while it is still 100x above tol).
 *   HISQ_FCG_NN   : flexible CG preconditioned by the network of hisq_nn_init/hisq_nn_train
 *                   (Notay's FCG with truncation 1, complex step sizes; FP32 body with
 *                   p->link_prec links, FP64 reliable updates); a rhs whose preconditioned step
 *                   breaks down, or whose true residual stops falling (6 replacements in a row
 *                   without a 10 % drop), is finished by MIXED from its current x.
 * Synchronises.  Returns HISQ_ERR_NOCONV if some rhs missed tol within max_iter.  With the
 * environment variable HISQ_CG_TRACE=1, F64/MIXED print one stderr line per residual replacement
 * of bundle slot 0 (iteration, link copy, true relative residual, true/iterated ratio).  The
 * F64/MIXED iteration sums the per-rhs alpha partials inside the r pass for V/2 up to ~150 k
 * sites and the beta partials inside the p/x pass for V/2 up to ~350 k (32^3 x 8, V/2 = 131 k:
 * both, four launches per iteration); HISQ_CG_FUSED_REDUCTIONS=0 keeps those sums as launches of
 * their own, with the same bits. */
int hisq_cg_mrhs(hisq_ctx *ctx, double mass, int n, const void *b, void *x,
                 const hisq_cg_params *p, hisq_cg_stats *stats);

/* ---- learned gauge-covariant preconditioner ------------------------------------------------
 * A linear network z = P r on the even sites, for the flexible CG (HISQ_FCG_NN).  Layer l mixes
 * the C = 8 complex channels per site and colour (C x C complex matrix W_l; the first layer lifts
 * the one input channel with W_in[C], the output is read out with W_out[C]) and applies a
 * per-channel gauge-covariant one-hop stencil over the fat links X of Eq. 3:
 *   S(a, phi)_c(x) = a[0,c] phi_c(x) + sum_mu (a[1+mu,c] X(x,mu) phi_c(x+mu)
 *                                            + a[5+mu,c] X(x-mu,mu)^dag phi_c(x-mu)).
 * Parameters (complex; as reals, re/im interleaved), in this order: W_in[C]; for l = 1..L:
 * W_l[C][C] ([out][in], only for l >= 2) then a_l[9][C]; W_out[C].  Hop index: 0 self, 1+mu
 * forward, 5+mu backward.  Activations are stored in BF16 (default; channel mixing on bf16 MFMA)
 * or FP32, arithmetic FP32, master weights FP32.  Needs the FP32 or FP16 link copy. */

/* Create the network (replaces an existing one): layers 1..8, channels must be 8; weights start
 * near P = identity with a small pseudo-random perturbation drawn from seed. */
int hisq_nn_init(hisq_ctx *ctx, int layers, int channels, unsigned long long seed);
/* Number of complex parameters (>= 1), or a negative error code. */
int hisq_nn_num_params(hisq_ctx *ctx);
/* Copy the parameters out of / into the context (host arrays of 2 * hisq_nn_num_params reals).
 * Setting resets the optimiser state. */
int hisq_nn_get_params(hisq_ctx *ctx, double *out, int n_reals);
int hisq_nn_set_params(hisq_ctx *ctx, const double *in, int n_reals);
/* Activation storage: 1 = BF16 (default), 0 = FP32. */
int hisq_nn_set_precision(hisq_ctx *ctx, int bf16_storage);
/* Form of the preconditioner built from the network N (N r = sum_c W_out[c] psi_L[c] on the
 * full lattice):
 *   HISQ_NN_FORM_DIRECT (default): P r = N r restricted to the even sites;
 *   HISQ_NN_FORM_GRAM:             P r = N^dag N r, Hermitian positive semi-definite for any
 *                                  weights (the property CG-type solvers assume of a
 *                                  preconditioner); each application costs two network passes.
 * The form applies to hisq_nn_apply, the loss, training and HISQ_FCG_NN, and is saved. */
enum { HISQ_NN_FORM_DIRECT = 0, HISQ_NN_FORM_GRAM = 1 };
int hisq_nn_set_form(hisq_ctx *ctx, int form);

/* Training loss for pairs (r_j, y_j = M^-1 r_j) over a minibatch of B pairs:
 *   HISQ_NN_LOSS_SOLUTION (default): (1/B) sum_j ||P r_j - y_j||^2 / ||y_j||^2
 *   HISQ_NN_LOSS_RESIDUAL:           (1/B) sum_j ||M (P r_j - y_j)||^2 / ||r_j||^2
 *                                    = (1/B) sum_j ||M P r_j - r_j||^2 / ||r_j||^2,
 * the second with M = m^2 - D_eo D_oe at `mass` (FP32 links, or FP16 if only those exist). */
enum { HISQ_NN_LOSS_SOLUTION = 0, HISQ_NN_LOSS_RESIDUAL = 1 };
int hisq_nn_set_loss(hisq_ctx *ctx, int kind, double mass);
/* z = P r for n vectors: r, z device [n][3][V/2] on even sites, complex128 (prec_io = HISQ_F64)
 * or complex64 (HISQ_F32).  Asynchronous. */
int hisq_nn_apply(hisq_ctx *ctx, int n, int prec_io, const void *r, void *z);
/* Loss (see hisq_nn_set_loss) and its gradient with respect to the parameters (Wirtinger:
 * dL/dRe + i dL/dIm, 2 * num_params reals, host) for n pairs r, y (device complex128
 * [n][3][V/2]).  loss and grad may be NULL.  Synchronises. */
int hisq_nn_loss_grad(hisq_ctx *ctx, int n, const void *r, const void *y, double *loss, double *grad);
/* Train on n_pairs pairs (device complex128 [n_pairs][3][V/2] each) with Adam (Kingma and Ba:
 * lr, beta1 0.9, beta2 0.999, eps 1e-8, on the real and imaginary parts of the parameters as
 * separate coordinates, FP32 master weights), minibatches of `batch` consecutive pairs visited
 * in a seeded random order (n_pairs / batch whole minibatches; the remaining pairs are not used;
 * batch <= HISQ_MAX_RHS), for `epochs` passes.  loss_history (host, epochs doubles, may be
 * NULL) receives the mean minibatch loss of each epoch.  Synchronises. */
int hisq_nn_train(hisq_ctx *ctx, int n_pairs, const void *r, const void *y, int epochs, int batch,
                  double lr, unsigned long long seed, double *loss_history);
/* Training pairs from plain FP64 CG trajectories: solve M x_i = b_i (n rhs, device complex128
 * [n][3][V/2]) to tol and keep x_k after iterations 0, snap_every, 2 snap_every, ... (at most
 * n_snap snapshots); return r_k = b - M x_k in r_out and y_k = x* - x_k = M^-1 r_k in y_out (both
 * device complex128 [n_snap][n][3][V/2], snapshot-major).  *n_pairs = snapshots taken * n. */
int hisq_nn_harvest(hisq_ctx *ctx, double mass, int n, const void *b, double tol, int n_snap,
                    int snap_every, void *r_out, void *y_out, int *n_pairs);

/* Save / load the network (binary: int32 header {magic 0x51534948, version 2, layers, channels,
 * form}, then the parameters as float64 reals; version 1 files, without the form, load as the
 * direct form). */
int hisq_nn_save(hisq_ctx *ctx, const char *path);
int hisq_nn_load(hisq_ctx *ctx, const char *path);

/* ---- stochastic trace (Section 1, Eq. 2) -----------------------------------------------------
 * The observables of Eq. 1 are traces of products of M^-1, estimated with many random vectors.
 * These two calls give the basic one, Tr M^-1 over the 3*V/2 components of the even sites:
 *   estimate = (1/N) sum_k eta_k^dag M^-1 eta_k,  std_error = sample std / sqrt(N),
 * with counter-based Z2 noise: component c = (k*3 + colour)*(V/2) + site of the noise stream is
 * -1 if the top bit of the c-th SplitMix64 output for `seed` is set, else +1 (SplitMix64: output
 * c = mix(seed + (c+1)*0x9E3779B97F4A7C15), Steele, Lea and Flood 2014). */

/* Noise vectors k0 .. k0+n-1 into out (device [n][3][V/2] complex128, real +-1).  Asynchronous. */
int hisq_z2_noise(hisq_ctx *ctx, unsigned long long seed, long long k0, int n, void *out);

/* Estimate Tr M^-1 from n_vec noise vectors 0 .. n_vec-1, solved in bundles of `bundle` rhs by
 * hisq_cg_mrhs with params p (use_x0 is ignored).  samples (host, n_vec doubles) may be NULL;
 * estimate (host) is required; std_error (host) may be NULL.  The context owns the bundle
 * buffers.  Synchronises.  Returns HISQ_ERR_NOCONV, with the estimate still written, if some
 * solve missed tol. */
int hisq_trace_minv(hisq_ctx *ctx, double mass, int n_vec, int bundle, unsigned long long seed,
                    const hisq_cg_params *p, double *samples, double *estimate, double *std_error);

/* The chiral condensate (1/V) Tr (m + D)^-1 of the whole-lattice operator, the trace of Eq. 2
 * without derivative insertions: the diagonal blocks of (m + D)^-1 are m M_ee^-1 and m M_oo^-1,
 * and M_oo has the spectrum of M_ee, so it is (2 m / V) Tr M_ee^-1, estimated as hisq_trace_minv
 * does (same noise vectors, bundles and solver; V the number of sites, taste factors left to the
 * caller).  estimate (host) is required, std_error (host) may be NULL.  Synchronises; returns
 * HISQ_ERR_NOCONV, with the estimate still written, if some solve missed tol. */
int hisq_chiral_condensate(hisq_ctx *ctx, double mass, int n_vec, int bundle, unsigned long long seed,
                           const hisq_cg_params *p, double *estimate, double *std_error);

#ifdef __cplusplus
}
#endif

#endif /* HISQ_H */
