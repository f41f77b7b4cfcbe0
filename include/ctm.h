/*
 * ctm.h -- C ABI of the MI355X CTMRG library (libctm.so).
 *
 * The library runs the corner transfer matrix renormalization group (CTMRG)
 * contraction of an infinite tensor product state (iTPS) on one AMD Instinct
 * MI355X (gfx950), as described in Sec. 2.2 and Fig. 2 of Motoyama et al.,
 * "TeNeS: Tensor Network Solver for Quantum Lattice Systems" (arXiv:2112.13184):
 * the ket and bra site tensors form a double-layer network of bond dimension
 * D^2; each site gets four corner matrices C (chi x chi) and four edge tensors
 * T (chi x chi x D^2), fixed by directional moves (absorb a column, build the
 * enlarged corners, compute QR-free projectors from a partial / randomized SVD
 * of the 2x2 cluster, renormalise).  The converged environment gives one-site
 * and nearest-neighbour expectation values (Sec. 5.3).
 *
 * Conventions (all arrays row-major, C order, FP64 unless stated):
 *   site tensor     A[l][u][r][d][p] (D^4 d values); classical network
 *                   (layers = 1): a[l][u][r][d] (D^4 values, d must be 1)
 *   site index      i = x + Lx * y, +y points up (r = (0,1) is the upper
 *                   neighbour, Sec. 5.3)
 *   pair index      ket * D + bra for a double-layer bond (Db = D^2);
 *                   Db = D for a classical network
 *   environment     per site, clockwise C1 T1 C2 T2 C3 T3 C4 T4 (C1 upper
 *                   left, T1 above).  Corner C_k[next][prev], edge
 *                   T_k[prev][next][pair]; next / prev name the clockwise
 *                   neighbour.  Stored zero padded to chi on every chi leg.
 *   directions      CTM_LEFT moves absorb columns into C1 T4 C4, CTM_RIGHT
 *                   into C3 T2 C2, CTM_UP into C2 T1 C1, CTM_DOWN into C4 T3 C3.
 *   operators       one-site op[out][in] (d x d); two-site
 *                   op[(out_i, out_j)][(in_i, in_j)] (d^2 x d^2), the element
 *                   order of the paper's operator input (Sec. 5.2).
 *
 * Errors: every call returns a ctm_status.  Invalid arguments give
 * CTM_EINVAL and leave the state unchanged; device failures CTM_EDEVICE;
 * NaN / Inf or a cut without any singular value above zero CTM_ENUMERIC.
 * ctm_last_error() describes the last failure on a context.  A context is
 * single threaded; a queue may be called from any thread.
 *
 * Ownership: host inputs are copied; device inputs are read during the call
 * only; outputs go to caller buffers.  The context owns all device memory it
 * allocates and frees it in ctm_free().
 */
#ifndef CTM_H
#define CTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CTM_OK = 0,
  CTM_EINVAL = -1,     /* bad argument or shape                                  */
  CTM_ENOMEM = -2,     /* device allocation failed                               */
  CTM_EDEVICE = -3,    /* HIP / rocSOLVER failure                                */
  CTM_ENUMERIC = -4,   /* NaN / Inf, or a cut with no singular value above zero  */
  CTM_ETOOBIG = -5,    /* request larger than the queue's memory budget          */
  CTM_EAGAIN = -6,     /* result not ready yet                                   */
  CTM_ECANCELED = -7   /* request cancelled                                      */
} ctm_status;

/* Arithmetic of the contraction GEMMs (enlarged corners, sketch products,
 * renormalisation).  QR, SVD, projector scaling, normalisation, convergence
 * and expectation values always run in FP64.  Reduced precisions round the
 * operands of each GEMM to nearest even and accumulate in FP32.
 * CTM_F16_SPLIT writes each operand as hi + lo (two FP16 numbers with a
 * power-of-two scale) and sums the three products hi*hi, hi*lo, lo*hi. */
typedef enum { CTM_F64 = 0, CTM_F32 = 1, CTM_BF16 = 2, CTM_F16_SPLIT = 3 } ctm_precision;

typedef enum { CTM_LEFT = 0, CTM_RIGHT = 1, CTM_UP = 2, CTM_DOWN = 3 } ctm_dir;

typedef struct {
  int Lx, Ly;              /* unit cell                                            */
  int d;                   /* physical dimension (1 for layers = 1)                */
  int D;                   /* virtual bond dimension of the site tensors           */
  int chi;                 /* environment bond dimension                           */
  int layers;              /* 2 = ket/bra iTPS (bra = ket, real), 1 = classical    */
  ctm_precision prec;      /* precision of the contraction GEMMs                   */
  double svd_rel_cutoff;   /* singular values <= cutoff * sigma_0 are dropped;
                              0 selects the default 1e-12                          */
  int rsvd_oversample;     /* p of the randomized SVD (k = chi + p); < 0 selects
                              the exact FP64 SVD of the explicitly formed cluster
                              matrix (small problems only)                         */
  int rsvd_power_iters;    /* q, number of power iterations                        */
  uint64_t seed;           /* key of the counter-based sketch generator            */
  void* stream;            /* hipStream_t to run on, or NULL for a private stream  */
  int projector_path;      /* CTM_PATH_AUTO, or CTM_PATH_HOUSEHOLDER to run every
                              truncating cut through Householder QR and the
                              library SVD (the path a cut takes when k > 320 or
                              its Cholesky QR breaks down)                          */
} ctm_config;

enum { CTM_PATH_AUTO = 0, CTM_PATH_HOUSEHOLDER = 1 };

typedef struct ctm_ctx ctm_ctx;

/* Sec. 2.2 (the iTPS of Sec. 2.1 and its double layer, Fig. 2): set up a
 * context for the given site tensors.  tensors holds Lx*Ly site tensors back
 * to back (site order i = x + Lx*y), in host memory (tensors_on_device = 0)
 * or device memory (1, read on cfg->stream, after the work enqueued on that
 * stream before the call, and not referenced afterwards).  boundary (Db values, host)
 * is the vector on every outer leg of the initial environment, or NULL for
 * the ket/bra identity (layers = 2) / all ones (layers = 1).  The initial
 * environment has C = [[1]] and T[0][0][:] = boundary (all chi legs of
 * dimension 1).  On success *out owns the new context. */
ctm_status ctm_init(const ctm_config* cfg, const double* tensors, int tensors_on_device,
                    const double* boundary, ctm_ctx** out);

/* Sec. 2.2: one directional move over every column (row) of the unit cell. */
ctm_status ctm_move(ctm_ctx* ctx, ctm_dir dir);

/* Sec. 2.2 (iterative determination of C and T) with the convergence
 * criterion of the ctm parameters (Sec. 5.2), read as follows.
 * Up to max_sweeps sweeps (left, right, up, down).  After every sweep the
 * singular values of every corner, normalised to sum 1, are compared with
 * those of the previous sweep; the run stops when the largest L1 change
 * (delta) is below tol.  Any out pointer may be NULL.  Not converging is not
 * an error (*converged = 0). */
ctm_status ctm_sweep(ctm_ctx* ctx, int max_sweeps, double tol, int* sweeps_done,
                     double* delta, int* converged);

/* Sec. 2.2: the QR-free projectors of one cut, from the partial
 * (randomized) SVD of the cluster matrix, which is applied only through
 * products with the four enlarged corners.
 * Projectors of one cut of a move, computed from the current environment and
 * not applied.  (x, y) are the column and cut row in the frame of the move
 * (the frame in which the move is a left move: the lattice rotated by 0, 2, 1,
 * 3 quarter turns counter-clockwise for left, right, up, down).  With
 * n = chi * Db, Pt (n x chi, host) renormalises the side above the cut and
 * P (chi x n, host) the side below; both are zero padded.  *k_eff is the
 * number of non-zero projector columns.  May be NULL. */
ctm_status ctm_projectors(ctm_ctx* ctx, ctm_dir dir, int x, int y, double* P, double* Pt,
                          int* k_eff);

/* Sec. 2.2, Fig. 2(c): a corner matrix with its two edge tensors and the
 * site absorbed.
 * Enlarged corner of role `corner` (0..3 = C1..C4) around `site`, as the
 * n x n matrix E[(c_next, o_next)][(c_prev, o_prev)] (host buffer): the
 * corner, its two edge tensors and the site seen from that corner, with ket
 * and bra contracted one after the other.  For testing. */
ctm_status ctm_enlarged_corner(ctm_ctx* ctx, int corner, int site, double* E);

/* Sec. 5.3: <op> at `site` from the 3x3 patch of the environment. */
ctm_status ctm_expect_1site(ctm_ctx* ctx, int site, const double* op, double* val);

/* Sec. 5.3: <op> on the bond from `site` to its neighbour at +x (dir = 0) or
 * +y (dir = 1), from the 3x4 / 4x3 patch.  op is d^2 x d^2 (see above). */
ctm_status ctm_expect_2site(ctm_ctx* ctx, int site, int dir, const double* op, double* val);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ctm_expect_2site with every transient of the contraction placed in one
 * fixed device array of CTM_NOALLOC_SCRATCH_BYTES that the library holds on
 * each device for the life of the process (set up by ctm_init), instead of
 * the context's workspace, which ctm_expect_2site grows on first use.  The
 * call itself allocates nothing (no hipMalloc, no allocating library call);
 * the context must exist (ctm_init allocates).  CTM_ETOOBIG, state unchanged,
 * if the contraction needs more than the array (the transients of a bond
 * grow as chi^2 D^4 (4 + 2 d) doubles: D = 3, chi = 40 fits, D = 4, chi = 64
 * does not); CTM_EDEVICE if the array's address could not be obtained on the
 * context's device.  All calls on one GPU share the array and it keeps the
 * last call's contents (nothing in it needs to start at zero): calls that
 * overlap on one GPU race, so serialise them. */
#define CTM_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
ctm_status ctm_expect_2site_noalloc(ctm_ctx* ctx, int site, int dir, const double* op, double* val);

/* Reduced density matrices behind the two calls above (host, ket index first:
 * rho[p][p'] and rho[(p_s, p_t)][(p_s', p_t')]), normalised to trace 1. */
ctm_status ctm_rho_1site(ctm_ctx* ctx, int site, double* rho);
ctm_status ctm_rho_2site(ctm_ctx* ctx, int site, int dir, double* rho);

/* Sec. 5.3, Eq. (8): the correlation function C(r) = <A(r0) B(r0 + r e)> for
 * r = 0..rmax, r0 = `site`, e = (1, 0) (dir = 0) or (0, 1) (dir = 1); A and B
 * are one-site operators (d x d, [out][in], host).  C[0] is the one-site
 * value of the product A B.  For r >= 1: the left boundary of r0, its column
 * with A, r - 1 plain columns, the column of r0 + r e with B and its right
 * boundary, over the same network without operators (the columns' edge
 * tensors are those of the sites passed).  C: rmax + 1 doubles (host). */
ctm_status ctm_correlation(ctm_ctx* ctx, int site, int dir, const double* opA, const double* opB, int rmax,
                           double* C);

/* Sec. 5.3 (correlation length): the nev eigenvalues of largest modulus of
 * the transfer matrix of one period of the unit cell, along +x (dir = 0) in
 * row `line` (0 <= line < Ly) or along +y (dir = 1) in column `line`
 * (0 <= line < Lx): the product of the columns T1 (site) T3 of the period's
 * sites acting on a left boundary (chi x D^2 x chi).  Computed on the device
 * by explicitly restarted Arnoldi with full reorthogonalisation (Krylov
 * dimension min(60, chi^2 D^2), Ritz residuals below 1e-12 |lambda_0|).
 * re / im (nev doubles each, host): the eigenvalues sorted by modulus,
 * descending.  e (nev - 1 doubles, may be NULL): e_k = -log|lambda_k /
 * lambda_0| / period, per lattice spacing.  xi (may be NULL): 1 / e_1, the
 * correlation length.  1 <= nev <= 16. */
ctm_status ctm_transfer_spectrum(ctm_ctx* ctx, int dir, int line, int nev, double* re, double* im, double* e,
                                 double* xi);

/* Sec. 5.3, Eq. (9): finite-chi extrapolation of the correlation length from
 * runs at n >= 2 values of chi: the least-squares line
 * e_1(chi) = 1/xi(inf) - k (e_2(chi) - e_1(chi)).  inv_xi: 1/xi(inf); k: its slope. */
ctm_status ctm_xi_extrapolate(int n, const double* e1, const double* e2, double* inv_xi, double* k);

/* The single-layer network of Fig. 2(b) contracted with the environment of
 * Fig. 2(c), for a classical network (layers = 1): Z(b) / Z(a) on the 3x3 patch of `site`,
 * with b (D^4, host) in place of the site tensor (e.g. a magnetisation). */
ctm_status ctm_impurity(ctm_ctx* ctx, int site, const double* b, double* val);

/* The contraction of the whole network of Fig. 2 (the norm of the iTPS, or
 * the partition function of a classical network) per site, 1x1 cell:
 * ln kappa, the log of the partition function (norm) per site, as
 * ln Z(3x3) + ln Z(corners) - ln Z(2x3) - ln Z(3x2). */
ctm_status ctm_log_kappa(ctm_ctx* ctx, double* ln_kappa);

/* The environment of Fig. 2(c) (corner matrices and edge tensors of one
 * site), read or replaced, so that a converged environment can be kept and
 * reused, as the paper's saved tensors are (Sec. 5.3).
 * Environment of one site as host FP64: C1..C4 (chi*chi each) then T1..T4
 * (chi*chi*Db each), zero padded; bytes must be >= ctm_env_bytes().  dims
 * (16 ints, may be NULL) gets the actual leg dimensions: C_k (next, prev) for
 * k = 1..4, then T_k (prev, next). */
size_t ctm_env_bytes(const ctm_ctx* ctx);
ctm_status ctm_get_env(ctm_ctx* ctx, int site, double* buf, size_t bytes, int* dims);
/* Replace the environment of one site (same layout; entries beyond dims must
 * be zero).  dims may be NULL: then every chi leg is taken as chi. */
ctm_status ctm_set_env(ctm_ctx* ctx, int site, const double* buf, size_t bytes, const int* dims);

/* Number of moves done since ctm_init (keys the sketch of each cut). */
ctm_status ctm_move_count(const ctm_ctx* ctx, int64_t* moves);

/* Projector cuts computed since ctm_init (moves and ctm_projectors), by path:
 * counts[0] identity (the cut bond is no larger than chi), counts[1] the
 * batched randomized SVD (Cholesky QR + Jacobi), counts[2] the fallback
 * (Householder QR and LAPACK-style SVD, or the dense SVD when
 * rsvd_oversample < 0) taken when the Cholesky QR of a panel breaks down,
 * the Jacobi SVD of a cut does not converge, k > 320, or projector_path is
 * CTM_PATH_HOUSEHOLDER.  All paths compute the same projectors (Sec. 2.2). */
ctm_status ctm_cut_stats(const ctm_ctx* ctx, int64_t counts[3]);

/* Per-phase GPU timing with HIP events recorded on the context's stream
 * around the launches of the timed phases, while enabled: on = 1 times every
 * phase, on = 2 the sketch GEMMs only, on = 0 stops.  Each pair of events
 * leaves a short idle gap (about 10 us) on the stream; the four sketch
 * products of one application of M (or M^T) share one pair, so their ms
 * include the split-K reductions between them.  Phases:
 *   0 other contraction GEMMs (edge-corner products, projector formation
 *                     P~ = G G V', the edge renormalisation, dense-mode M)
 *   1 sketch GEMMs    (the randomized SVD's products of an n x n enlarged
 *                     corner with an n x k panel: (10 + 8q) per cut)
 *   2 absorption      (single-layer ket and bra contractions of the site)
 *   3 factorisations  (QR, SVD and projector scaling, FP64)
 *   4 other           (small GEMMs, FP64 in every precision; normalisation,
 *                     permutations, spectra)
 * flops counts the algorithmic floating-point operations of the launches
 * (2 M N K per GEMM, 4 chi^2 D^6 d per absorption; 0 for phases 3 and 4).
 * ctm_timing_read() synchronises the stream. */
#define CTM_NPHASE 5
typedef struct {
  int64_t launches[CTM_NPHASE];
  double ms[CTM_NPHASE];
  double flops[CTM_NPHASE];
} ctm_timing;
ctm_status ctm_timing_enable(ctm_ctx* ctx, int on);   /* 0, 1 or 2; also clears the counters */
ctm_status ctm_timing_read(ctm_ctx* ctx, ctm_timing* out);

/* Device memory a context with this configuration allocates (resident state
 * plus workspaces), in bytes; 0 for an invalid configuration. */
size_t ctm_footprint_bytes(const ctm_config* cfg);

/* Text of the last error on ctx (valid until the next call on ctx); a static
 * message for ctx == NULL. */
const char* ctm_last_error(const ctm_ctx* ctx);

void ctm_free(ctm_ctx* ctx);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of independent CTMRG solves on one GPU       */
/* (a Hamiltonian parameter scan, say).  Each request is a CTMRG run of the  */
/* given site tensors to convergence (Sec. 2.2) followed by the expectation  */
/* values of Sec. 5.3: energy per site and the requested observables.        */
/* ------------------------------------------------------------------------ */
typedef struct ctm_queue ctm_queue;

#define CTM_MAX_OBS 8       /* observables of each kind per request            */
#define CTM_MAX_SITES 16    /* largest unit cell                               */

typedef struct {
  ctm_config cfg;            /* stream is ignored: each group runs on its own stream */
  const double* tensors;     /* Lx*Ly site tensors (layout as for ctm_init); host
                                memory, or device memory if tensors_on_device     */
  int tensors_on_device;     /* device tensors are copied at submit, on the queue's
                                stream (after the work enqueued on it before)      */
  const double* bond_op;     /* d^2 x d^2 operator on every +x and +y bond (the
                                Hamiltonian term, Sec. 5.2 element order)          */
  const double* onsite_op;   /* d x d Hamiltonian term on every site, or NULL     */
  int n_obs;                 /* one-site observables to measure, 0..CTM_MAX_OBS   */
  const double* obs_ops;     /* n_obs operators of d x d, back to back ([out][in]) */
  int n_obs2;                /* two-site observables, 0..CTM_MAX_OBS              */
  const double* obs2_ops;    /* n_obs2 operators of d^2 x d^2, back to back       */
  double tol;                /* stop when delta < tol (see ctm_sweep)             */
  int max_sweeps;
  uint64_t tag;              /* returned unchanged                                */
} ctm_request;

typedef struct {
  ctm_status status;         /* CTM_OK, CTM_ENUMERIC (this solve only), CTM_ECANCELED,
                                CTM_EDEVICE / CTM_ENOMEM                           */
  int converged, sweeps;
  double delta;
  double energy_per_site;    /* (1/N) sum_s <h_{s,s+x}> + <h_{s,s+y}> + <h_s>     */
  double obs[CTM_MAX_OBS][CTM_MAX_SITES];      /* <O_k> at site i (i < Lx*Ly)     */
  double obs2[CTM_MAX_OBS][CTM_MAX_SITES][2];  /* <O2_k> on the bond from site i to
                                                  i + x [0] and to i + y [1]      */
  uint64_t tag;
  int64_t t_submit_ns, t_admit_ns, t_done_ns;   /* steady clock; t_done is the time
                                                   this solve's result was published */
} ctm_result;

/* A queue of CTMRG solves run concurrently on the current device.
 *
 * Admission: up to max_active groups run at once, each on a worker thread
 * with its own context and HIP stream; a pending request is admitted (first
 * fit in arrival order; a request passed over by 8 later admissions stops
 * further skipping) when the summed footprints (ctm_footprint_bytes) of the
 * running groups plus its own stay within hbm_budget_bytes.  Later pending
 * requests of the same shape (every ctm_config field but seed and stream)
 * join it, up to 8, while the group's footprint fits: the group's solves are
 * replicas of one context, whose launches cover the cuts of all its live
 * replicas.
 * Per solve: sweeps until delta < tol, max_sweeps, cancellation (checked
 * between sweeps) or a numerical failure of that solve alone (NaN / Inf, or
 * a cut without singular values: CTM_ENUMERIC); then its observables are
 * evaluated and its result published at once.  Its slot in the group is then
 * free: at the next sweep boundary the oldest pending request of the same
 * shape takes it (no further memory), so a group keeps running while such
 * requests arrive.  The group's memory returns to the budget when its last
 * solve is published.  A request's result does not depend on the other
 * requests it ran with (same seed, same result, bitwise).
 * stream: hipStream_t (e.g. the caller's torch stream) on which device-side
 * request tensors are read at submit, or NULL for the null stream. */
ctm_status ctm_queue_create(size_t hbm_budget_bytes, int max_active, void* stream, ctm_queue** out);
/* Copies the request (inputs and operators) and returns at once; *ticket
 * identifies it.  CTM_ETOOBIG if its footprint exceeds the budget, CTM_EINVAL
 * for a bad shape, NULL pointers or too many observables, CTM_ENUMERIC for
 * NaN / Inf in the site tensors. */
ctm_status ctm_queue_submit(ctm_queue* q, const ctm_request* req, uint64_t* ticket);
/* CTM_EAGAIN while pending or running; otherwise the final status, with the
 * result filled in. */
ctm_status ctm_queue_poll(ctm_queue* q, uint64_t ticket, ctm_result* res);
/* Waits up to timeout_ms (< 0: forever); CTM_EAGAIN on timeout. */
ctm_status ctm_queue_wait(ctm_queue* q, uint64_t ticket, int timeout_ms, ctm_result* res);
/* A pending request ends at once (CTM_ECANCELED); a running one at its next
 * sweep boundary. */
ctm_status ctm_queue_cancel(ctm_queue* q, uint64_t ticket);
/* Cancels pending requests, waits for running ones, frees everything. */
void ctm_queue_destroy(ctm_queue* q);

/* Sec. 2.3, Eq. (4) with the CTMRG environment (the full update): one
 * first-order Trotter step of the site tensors held by the context, in the
 * simple update's bond order (horizontal bonds of sites 0..N-1, then the
 * vertical ones), H [N][2][d^2][d^2] (host) as for ctm_su_set_hamiltonians.
 * Each bond: QR of both tensors into [other legs][(bond, p)] = X a; the bond
 * environment N[(rho_i, rho_j)][(rho_i', rho_j')] from the context's current
 * environment with X_i, X_j in place of the sites, made symmetric and
 * positive semidefinite; the gate applied to a_i a_j; start from its
 * truncated SVD; als_iters rounds of alternating least squares (each factor
 * by the pseudo-inverse of its normal matrix, eigenvalues <= 1e-12 of the
 * largest dropped); the new tensors X a with the sign of each bond index
 * fixed (first entry of the left tensor within 1e-8 of its largest modulus
 * positive) and each divided by its largest |entry|; then env_sweeps CTMRG
 * sweeps from the current environment.  Needs an FP64 iTPS context (layers
 * = 2) with Lx, Ly >= 2 and d <= D^2; converge the environment first. */
ctm_status ctm_fu_step(ctm_ctx* ctx, const double* H, double tau, int als_iters, int env_sweeps);
/* The context's current site tensors, [N][D^4 d] (host). */
ctm_status ctm_get_tensors(ctm_ctx* ctx, double* tensors);

/* ------------------------------------------------------------------------
 * Simple-update imaginary-time evolution and the mean-field environment.
 *
 * Sec. 2.3, Eqs. (1)-(3): exp(-T H)|Psi_0> as N_tau first-order
 * Suzuki-Trotter steps of two-site gates exp(-tau H_ij); after each gate the
 * bond is truncated back to D (Eq. (4)) with the rest of the network replaced
 * by the mean-field environment, i.e. the simple update.  Sec. 2.2 (MFE
 * paragraph): local density matrices contracted with bond weights on the open
 * bonds, O(D^4) for a site and O(D^5) for a bond.
 *
 * State of one problem (Vidal form; all arrays C order, FP64):
 *   gamma   [N][D][D][D][D][d]  site tensors G_s[l][u][r][d][p], N = Lx*Ly,
 *                               site s = x + Lx*y, +y up
 *   lambda  [N][2][D]           bond weights: [s][0] on the bond between s
 *                               and its right neighbour, [s][1] between s
 *                               and its upper neighbour.  Leg l of s carries
 *                               the [.][0] weight of its left neighbour, u
 *                               its own [s][1], r its own [s][0], d the
 *                               [.][1] weight of its lower neighbour.
 *   H       [N][2][d*d][d*d]    bond Hamiltonian of the same bonds,
 *                               H[(out_i, out_j)][(in_i, in_j)], i = s and j
 *                               its right (0) or upper (1) neighbour.
 * A batch holds `batch` independent problems back to back (same shape; each
 * its own tensors, Hamiltonians and tau), all evolved by one call.
 * The iTPS a state stands for has A_s = G_s with sqrt(weight) on every leg
 * (ctm_su_get_itps), which ctm_init / ctm_queue_submit take as site tensors.
 *
 * One Trotter step updates the horizontal bonds of sites 0..N-1, then the
 * vertical bonds of sites 0..N-1.  Bond update (i, j): absorb the weights of
 * the other legs, contract the shared bond with its weights, apply the gate,
 * keep the D largest singular triplets of the two-site matrix ((other legs of
 * i, p_i) x (other legs of j, p_j)); the new weights are those singular
 * values divided by their 2-norm; the new tensors are the singular vectors
 * with the absorbed weights divided out again (a weight <= 1e-13 counts as
 * zero); the sign of each kept pair makes the first entry of its left vector
 * within 1e-8 of the largest modulus positive.
 * Limits: Lx, Ly >= 2, Lx*Ly <= 16, 1 <= D <= 8, 1 <= d <= 4,
 * min(D^3, D d) d <= 64, and the two reduced bond tensors must fit one
 * workgroup's LDS (D = 8, d = 2 fits in real arithmetic, D = 6, d = 2 in
 * complex); batch <= 65535.
 * ------------------------------------------------------------------------ */
typedef struct {
  int Lx, Ly;      /* unit cell, both >= 2                                     */
  int d;           /* physical dimension                                        */
  int D;           /* bond dimension kept by the truncation                     */
  int batch;       /* independent problems evolved together                     */
  void* stream;    /* hipStream_t, or NULL for a private stream                 */
  int complex_tensors;  /* 1: complex site tensors, Hamiltonians, gates and
                           density matrices, stored as (re, im) pairs of
                           doubles (every such array twice as long); the bra
                           is conj(ket); weights and energies stay real.
                           The phase of each kept pair makes the first
                           near-largest entry of its left vector real and
                           positive.  0: real (FP64).                       */
} ctm_su_config;

typedef struct ctm_su ctm_su;

/* Copies gamma [batch][N][D^4 d] and lambda [batch][N][2][D] (host) to the
 * device.  CTM_EINVAL, before any device call, for a shape outside the
 * limits, a non-finite tensor entry or a weight that is negative or not
 * finite. */
ctm_status ctm_su_create(const ctm_su_config* cfg, const double* gamma, const double* lambda, ctm_su** out);
/* Eq. (3): H [batch][N][2][d^2][d^2] and tau [batch] (host, finite,
 * tau >= 0); the gates exp(-tau H) are formed on the device (scaling and
 * squaring of a Taylor polynomial).  Must precede ctm_su_run. */
ctm_status ctm_su_set_hamiltonians(ctm_su* su, const double* H, const double* tau);
/* nsteps Trotter steps of every problem.  CTM_ENUMERIC if a bond of some
 * problem lost all its singular values (zero or non-finite state). */
ctm_status ctm_su_run(ctm_su* su, int nsteps);
/* Device time of the last ctm_su_run (HIP events around its launches), its
 * launch count and the bond updates it made (any pointer may be NULL). */
ctm_status ctm_su_stats(const ctm_su* su, double* gpu_ms, long* launches, long* bond_updates);
/* Copies the state to host arrays of the ctm_su_create layout (either may be NULL). */
ctm_status ctm_su_get(ctm_su* su, double* gamma, double* lambda);
/* A_s = G_s times sqrt(weight) on each leg, [batch][N][D^4 d], into host
 * memory (on_device = 0) or device memory (1). */
ctm_status ctm_su_get_itps(ctm_su* su, double* tensors, int on_device);
/* Sec. 2.2, MFE: unit-trace density matrices, rho1 [batch][N][d][d]
 * (ket index first) of every site (weights squared on its four legs) and rho2
 * [batch][N][2][d^2][d^2] of every bond, rho2[(p_i, p_j)][(p_i', p_j')] (the
 * 1 x 2 cluster with weights on its six open legs).  Either may be NULL. */
ctm_status ctm_su_mfe(ctm_su* su, double* rho1, double* rho2);
/* MFE energy per site of every problem: energy[b] = (1/N) sum_s
 * (<H[s][0]> + <H[s][1]> + <onsite_b>), onsite [batch][d][d] or NULL;
 * bond_energy [batch][N][2] (may be NULL) receives each bond's <H>. */
ctm_status ctm_su_mfe_energy(ctm_su* su, const double* onsite, double* energy, double* bond_energy);
const char* ctm_su_last_error(const ctm_su* su);
void ctm_su_free(ctm_su* su);

#ifdef __cplusplus
}
#endif
#endif /* CTM_H */
