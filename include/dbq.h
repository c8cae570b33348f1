/*
 * dbq.h -- C ABI of the MI355X deflated-BiCGStab library for Wilson and twisted-mass
 * fermion systems A x = b with many right-hand sides.
 *
 * Method: Abdel-Rehim, Morgan and Wilcox, "Deflated BiCGStab for linear equations in QCD
 * problems" (Lattice 2007).  Sec. 1 sets the problem (many right-hand sides, kappa near
 * kappa_c, gamma5 A gamma5 = A^dagger), Sec. 2 the D-BiCGStab(k) algorithm, Sec. 3 the first
 * right-hand side by GMRES-DR(m,k) and the definition of kappa_c, Sec. 4 the twisted-mass
 * operator and the projection over previous shifts' solutions.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: extents L[4] = {Lx, Ly, Lz, Lt}, all even and >= 2, periodic; V = Lx*Ly*Lz*Lt;
 * lexicographic site index lex = x + Lx*(y + Ly*(z + Lz*t)); n = 12*V.
 * Spinor fields (caller layout): complex128 (interleaved re, im doubles), [nrhs][V][4 spin][3 colour],
 * so element index 12*lex + 3*spin + colour inside one right-hand side.
 * Gauge field (caller layout): complex128 [4 mu][V][3][3]; links[mu][x] = U_mu(x), the SU(3)
 * matrix on the link x -> x + mu.  Rows must be unitary with determinant 1 for the single-precision
 * path (it stores two rows and rebuilds the third as conj(row0 x row1)).
 * Operator: A(mu) = I - kappa*H + i*mu*gamma5,
 *   (H psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu)],
 *   chiral gamma basis with gamma5 = diag(1, 1, -1, -1); the dagger is A(mu)^dagger = gamma5 A(-mu) gamma5.
 * Memory: every large array (fields, vectors, bases) is a DEVICE pointer owned by the caller;
 * scalar outputs (theta, stats, norms) are HOST pointers.  The library owns only the workspace
 * inside a dbq_ctx (allocated lazily, reused across calls, freed by dbq_destroy).
 * Streams: all work is ordered on the context's stream; solver calls synchronise that stream
 * before returning, wilson_apply and link_force do not.
 * Errors: every call returns a dbq_status and never throws; dbq_last_error() gives the message.
 * Invalid arguments (odd or zero extents, k >= m, nrhs < 1, null pointers) return DBQ_EINVAL
 * without launching anything.
 * Tolerances: tol means ||b - A x||_2 / ||b||_2 <= tol, judged on an FP64 residual recomputed
 * from the final x.  max_mv caps matrix-vector products per right-hand side.
 */
#ifndef DBQ_H
#define DBQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dbq_ctx dbq_ctx;

typedef enum {
  DBQ_OK = 0,
  DBQ_NOT_CONVERGED = 1, /* the paper's "F": x holds the best iterate, stats are valid */
  DBQ_EINVAL = -1,
  DBQ_EBREAKDOWN = -2,   /* BiCGStab broke down more than 10 times */
  DBQ_ESINGULAR = -3,    /* projected k x k matrix numerically singular (cond > 1e12) */
  DBQ_EHIP = -4,
  DBQ_ENOMEM = -5
} dbq_status;

typedef enum {
  DBQ_FP64 = 0,  /* FP64 vectors, FP64 18-real links */
  DBQ_MIXED = 1  /* FP32 vectors and 12-real links inside BiCGStab, FP64 reliable updates */
} dbq_prec;

/* Operator of a call.  schur selects the system the iteration runs on (Sec. 3 and Sec. 4 solve
 * the even-odd preconditioned one):
 *   0: the full operator A(mu) on all V sites;
 *   1: the even-odd reduced operator, the Schur complement on the even sites
 *        Ahat(mu) = D - kappa^2 H_eo D^{-1} H_oe,   D = I + i*mu*gamma5,
 *      (H_eo: the hops from odd to even sites), dagger gamma5 Ahat(-mu) gamma5.  Vectors keep the
 *      caller layout of all V sites: a solver is still handed b and returns x of A x = b (it
 *      solves Ahat x_e = b_e + kappa H_eo D^{-1} b_o and sets x_o = D^{-1} (b_o + kappa H_oe x_e));
 *      deflation vectors are even-site vectors stored as full vectors with zero odd sites;
 *      wilson_apply writes Ahat in_e to the even sites of out and zero to the odd ones.  One
 *      application of Ahat is one matrix-vector product.  Not accepted by link_force. */
typedef struct {
  int32_t L[4];
  const void* links; /* device, complex128 [4][V][3][3] */
  double kappa;
  double mu;         /* twisted mass; 0 for plain Wilson */
  int32_t schur;     /* 0: A; 1: the even-odd reduced operator (see above) */
  int32_t pad;       /* must be 0 */
} dbq_operator;

typedef struct {
  int64_t matvecs;          /* operator applications charged to this right-hand side */
  int64_t iterations;       /* BiCGStab iterations (GMRES-DR: cycles) */
  int64_t restarts;         /* BiCGStab breakdown restarts */
  int64_t reliable_updates; /* FP64 residual recomputations (mixed precision) */
  double rel_true_resid;    /* ||b - A x|| / ||b|| in FP64 at exit */
  double seconds;           /* wall time of the call (shared by all rhs of a call) */
  int32_t status;           /* dbq_status of this right-hand side */
  int32_t fp64_continued;   /* mixed precision: 1 if the FP32 iteration stalled, diverged or
                               overflowed and the FP64 solver finished this rhs, else 0 */
} dbq_stats;

/* Context: hip_stream is a hipStream_t (NULL = the null stream).  The stream must live as long
 * as the context.  Returns DBQ_OK and a context in *out. */
int dbq_create(dbq_ctx** out, void* hip_stream);
int dbq_destroy(dbq_ctx* ctx);
const char* dbq_last_error(const dbq_ctx* ctx);
/* Change the stream later calls are ordered on. */
int dbq_set_stream(dbq_ctx* ctx, void* hip_stream);

/* Geometry tables of the site order used inside the library.  Sec. 3 solves the even-odd
 * preconditioned system; here even-odd is the storage order of the full operator, blocked into
 * 4-d tiles of T0 x T1 x T2 x T3 sites (powers of two dividing the extents, reported by
 * dbq_site_tile):
 *   eo = parity*V/2 + tile*(T0*T1*T2*T3/2) + (in-tile lex >> 1),   parity = (x+y+z+t) mod 2,
 * tile = lexicographic index of (x/T0, y/T1, z/T2, t/T3) over the tile grid, in-tile lex =
 * (x mod T0) + T0*((y mod T1) + T1*((z mod T2) + T2*(t mod T3))).
 * lex_of_eo: DEVICE int32 [V]; nbr: DEVICE int32 [8][V] with nbr[2*mu][eo] = eo index of x+mu and
 * nbr[2*mu+1][eo] = eo index of x-mu.  dbq_geometry_host fills HOST arrays with the same values
 * from the same index arithmetic on the CPU.  Extents must be even and >= 2 (DBQ_EINVAL). */
int dbq_geometry(dbq_ctx* ctx, const int32_t L[4], int32_t* lex_of_eo, int32_t* nbr);
int dbq_geometry_host(const int32_t L[4], int32_t* lex_of_eo, int32_t* nbr);
/* Tile extents T[4] (host array) of the internal site order for extents L: per direction the
 * largest power of two dividing L_mu, at most 4 (a tile holds at most 4^4 = 256 sites).  Host
 * only; DBQ_EINVAL for odd or < 2 extents. */
int dbq_site_tile(const int32_t L[4], int32_t* T);

/* Processing order of the LDS-staged FP32 Dslash over (tile, rhs chunk) pairs, for inspection
 * (host only).  A launch with nchunks chunks of right-hand sides runs ntiles * nchunks blocks,
 * ntiles = prod_mu L_mu / T_mu (tiles of dbq_site_tile, numbered lexicographically); logical
 * block b (blocks reach the eight XCDs in contiguous ranges of b) processes tile[b] and chunk[b].
 * order 0: tiles in lexicographic order, the chunks of one tile adjacent; order 1: the tile grid
 * cut in halves along x, y and z into eight regions taken one after the other, tiles
 * lexicographic inside a region, chunks adjacent; order 2: the regions of order 1, inside a
 * region every tile for one chunk before the next chunk; order 3: the tile grid cut in halves
 * along z and quarters along t (t quarter b = [floor(b NT_t / 4), floor((b + 1) NT_t / 4))) into
 * eight regions taken one after the other (z half fastest), each with the whole x and y extent,
 * tiles lexicographic inside a region, chunks adjacent.  tile, chunk: HOST int32
 * [ntiles * nchunks].  DBQ_EINVAL for odd extents, nchunks < 1 or another order. */
int dbq_tile_schedule_host(const int32_t L[4], int32_t nchunks, int32_t order, int32_t* tile,
                           int32_t* chunk);

/* Streaming probe of the practical HBM ceiling: kind 0 copies bytes from src to dst, kind 1 reads
 * src (writing one float per block to dst, 2048 floats), kind 2 fills dst;
 * hand-written float4 kernels, launched reps times after one warm-up on the context stream,
 * timed with HIP events.  src, dst: DEVICE, bytes a multiple of 16.  *ms (HOST) = average
 * milliseconds per launch; bytes moved per launch: 2 x bytes (copy) or bytes (read, fill).
 * Synchronises the stream. */
int dbq_stream_probe(dbq_ctx* ctx, const void* src, void* dst, int64_t bytes, int32_t kind,
                     int32_t reps, double* ms);

/* out = A(mu) in (dagger = 0) or A(mu)^dagger in (dagger = 1) for nrhs right-hand sides
 * (Sec. 1 operator; the matrix-vector product every solver in the paper is costed in); with
 * op->schur = 1, out_e = Ahat in_e (or its dagger) and out_o = 0.
 * in, out: DEVICE complex128 [nrhs][V][12], must not overlap.  prec = DBQ_MIXED computes in
 * FP32 with 12-real links and returns the FP32 result widened to complex128. */
int wilson_apply(dbq_ctx* ctx, const dbq_operator* op, const void* in, void* out,
                 int32_t nrhs, int32_t dagger, int32_t prec);

/* wilson_apply for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same operator, but the packed
 * links and vectors live in one static device array of 64 MiB per GPU (each GPU that the library
 * runs on holds it until the process ends; its device address is looked up in dbq_create), and
 * the call allocates nothing.  Full operator only (op->schur = 0); a fixed launch shape (FP64:
 * one thread per site; DBQ_MIXED: the LDS tile kernel with every rhs per block), so no tuning.
 * in, out: DEVICE complex128 [nrhs][V][12] as for wilson_apply (the caller owns them).  The
 * scratch must hold the packed links and both packed vectors: V * (576 + 384 nrhs) bytes in FP64,
 * V * (192 + 192 nrhs) in DBQ_MIXED (each part rounded up to 256 bytes); larger inputs return
 * DBQ_EINVAL before any launch.  Every call on a GPU uses that GPU's one array: calls that overlap
 * on one GPU (several streams or threads) race; calls ordered on one stream do not.  Not
 * synchronising. */
int wilson_apply_noalloc(dbq_ctx* ctx, const dbq_operator* op, const void* in, void* out,
                         int32_t nrhs, int32_t dagger, int32_t prec);

/* First right-hand side by GMRES-DR(m,k) (Sec. 1 and Sec. 3): restarted GMRES whose restart
 * keeps the k harmonic Ritz vectors of smallest |theta|; convergence is tested once per cycle,
 * so matvecs = m + (m-k)(cycles-1) when x0 = 0.
 * b: DEVICE complex128 [V][12]; x: DEVICE complex128 [V][12], in: initial guess, out: solution.
 * V_out: DEVICE complex128 column-major n x k (column j at V_out + j*n), orthonormal, spanning the
 * final cycle's harmonic Ritz vectors; theta: HOST double [2*k] (re, im) sorted by |theta|;
 * k_out: HOST, the number of columns returned (k, or k-1 when the k-th and (k+1)-th values are a
 * complex-conjugate pair, which would make the left-right projection singular).
 * Returns DBQ_NOT_CONVERGED when max_mv is reached first; V_out and theta are still written.
 * With op->schur = 1 the Krylov space and V_out are those of Ahat (even sites; odd sites of V_out
 * are zero), tol is relative to ||b|| of the full system, and x is the full solution.
 * Requires 2 <= k < m <= 128. */
int gmresdr_first_rhs(dbq_ctx* ctx, const dbq_operator* op, const void* b, void* x,
                      int32_t m, int32_t k, double tol, int64_t max_mv,
                      void* V_out, double* theta, int32_t* k_out, dbq_stats* stats);

/* D-BiCGStab(k) (Sec. 2) for a batch of nops operators (lattices of possibly different size),
 * operator i with nrhs[i] right-hand sides:
 *   r0 = b - A x0;  solve (U^H A V) y = U^H r0 with U = gamma5 V;  x0 += V y;  BiCGStab from x0.
 * With dagger = 1 the system is A^dagger x = b and the roles swap (right vectors gamma5 V, left V).
 * V[i]: DEVICE complex128 column-major n_i x k[i] (k[i] = 0: no deflation, plain BiCGStab).
 * B[i]: DEVICE complex128 [nrhs[i]][V_i][12]; X[i]: same shape, in: x0, out: solution.
 * per_rhs: HOST array of sum(nrhs) stats, in operator order.  prec: dbq_prec.
 * DBQ_MIXED runs the BiCGStab recursion in FP32 and, whenever its residual norm has fallen 1000x
 * (or after 500 iterations without that), computes b - A x in FP64 and restarts the recursion
 * from it (rhat = p = r); a right-hand side on which the FP32 recursion stalls, diverges or
 * overflows is finished by the FP64 solver (per_rhs[j].fp64_continued = 1).
 * With schur = 1 (the same for every operator of the call) V[i] holds eigenvectors of Ahat as
 * full vectors with zero odd sites (as gmresdr_first_rhs returns them), the iteration runs on
 * Ahat, and X[i] receives the full solution; rel_true_resid is ||bhat - Ahat x_e|| / ||b||, which
 * equals ||b - A x|| / ||b|| up to the rounding of the odd-site reconstruction.
 * Returns the worst status over all right-hand sides (an error status if any, else
 * DBQ_NOT_CONVERGED if any did not converge). */
int dbicgstab_solve(dbq_ctx* ctx, const dbq_operator* ops, int32_t nops,
                    const void* const* V, const int32_t* k, const void* const* B,
                    void* const* X, const int32_t* nrhs, double tol, int64_t max_mv,
                    int32_t prec, int32_t dagger, dbq_stats* per_rhs);

/* Minimal-residual projection over previous shifts' solutions (Sec. 4): for each rhs j,
 * d = argmin ||r0 - A_new Q_j d|| with r0 = b_j - A_new x0_j, then x0_j += Q_j d.  The paper writes
 * the normal equations Q^H A^H A Q d = Q^H A^H r0; this solves the same least-squares problem
 * through a QR factorisation of W = A_new Q_j (classical Gram-Schmidt twice) so cond(W) is not
 * squared.  Q: DEVICE complex128 [nrhs][nq][V][12]; B, X0: DEVICE complex128 [nrhs][V][12] (X0
 * in/out); rnorm_before_after: HOST double [2*nrhs] = ||r0||, ||r_new|| per rhs.
 * Costs (1 if x0 != 0) + nq matrix-vector products per rhs.  1 <= nq <= 32.
 * With op_new->schur = 1 the projection is done on the reduced system of op_new (r0 = bhat -
 * Ahat x0_e over the even parts of Q) and X0 receives the full vector with its odd sites
 * reconstructed; the norms are those of the reduced residuals. */
int project_shifts(dbq_ctx* ctx, const dbq_operator* op_new, const void* Q, int32_t nq,
                   const void* B, void* X0, int32_t nrhs, double* rnorm_before_after);

/* GMRES(m)-Proj(k), the comparison method of Sec. 1 and Sec. 3 for later right-hand sides: a
 * minimal-residual projection over the right eigenvectors V (x += V d, d = argmin ||r - A V d||)
 * alternating with cycles of GMRES(m) from the current residual, until ||r|| <= tol ||b|| (tested
 * after each projection and each cycle) or max_mv products.  FP64, the right-hand sides one after
 * another.  V: DEVICE complex128 column-major n x k as gmresdr_first_rhs returns it (k = 0: plain
 * restarted GMRES(m)); B, X: DEVICE complex128 [nrhs][V][12] (X in: x0, out: solution);
 * per_rhs: HOST stats (matvecs excludes the k products of the setup W = A V; iterations = GMRES
 * cycles).  Requires 2 <= m <= 128, 0 <= k <= 128.  Accepts op->schur = 1 like dbicgstab_solve. */
int gmres_proj_solve(dbq_ctx* ctx, const dbq_operator* op, const void* V, int32_t k,
                     const void* B, void* X, int32_t nrhs, int32_t m, double tol, int64_t max_mv,
                     dbq_stats* per_rhs);

/* Gradient of L = sum_j Re(eta_j^H A^{-1} b_j) with respect to the links, given the solutions
 * x_j = A^{-1} b_j and the adjoint solutions lambda_j = A^{-H} eta_j (dL = -Re(lambda^H dA x)):
 *   G_mu(y) = kappa * sum_j sum_spin [ lambda(y) ((1-gamma_mu) x(y+mu))^H + x(y) ((1+gamma_mu) lambda(y+mu))^H ].
 * lambda, x: DEVICE complex128 [nrhs][V][12].
 * kind 0: F = DEVICE double [4][V][8], F[mu][y][a] = Re(i tr[T_a U_mu(y) G_mu(y)^H]), T_a = Gell-Mann/2,
 *         the derivative along U -> exp(i theta T_a) U.
 * kind 1: F = DEVICE complex128 [4][V][3][3] = G itself (dL = Re sum conj(G) dU).
 * op->schur must be 0: solves on the reduced system return the full x and lambda, whose gradient
 * is the one of the full operator (pass them with schur = 0). */
int link_force(dbq_ctx* ctx, const dbq_operator* op, const void* lambda, const void* x,
               int32_t nrhs, int32_t kind, void* F);

/* kappa_c (Sec. 3: the kappa at which the real part of A's smallest eigenvalue vanishes), i.e.
 * 1 / max Re lambda(H), from a thick-restarted Arnoldi iteration on H (restart keeps the k Ritz
 * vectors of largest real part).  lambda: HOST double [2] = rightmost eigenvalue of H;
 * resid: HOST, ||H v - lambda v|| / ||v|| of its Ritz vector.  Requires 2 <= k < m <= 128. */
int kappa_critical(dbq_ctx* ctx, const int32_t L[4], const void* links, int32_t m, int32_t k,
                   double tol, int64_t max_mv, double* kappa_c, double* lambda, double* resid);

/* kappa_critical, also returning the nritz (1 <= nritz <= k) Ritz values of largest real part of
 * the final cycle in decreasing real part, ritz: HOST double [2 * nritz] (re, im), the first one
 * being lambda.  Beyond the first, whose residual resid bounds, these are Ritz values of the same
 * Krylov space, not converged eigenvalues: they show how far the rightmost one stands from the
 * next ones (Sec. 3 defines kappa_c by the rightmost).  DBQ_EINVAL for nritz outside 0..k or a
 * null ritz with nritz > 0; otherwise as kappa_critical. */
int kappa_critical_ritz(dbq_ctx* ctx, const int32_t L[4], const void* links, int32_t m, int32_t k,
                        double tol, int64_t max_mv, double* kappa_c, double* lambda, double* resid,
                        int32_t nritz, double* ritz);

/* Instrumentation: with timing on (dbq_set_timing with on = N >= 1), every N-th launch of each
 * class -- the Dslash launches of the full operator inside the library and the FP32 BiCGStab
 * update steps (x += alpha p + omega s, r = s - omega t, p = r + beta (p - omega v) with ||r||^2) -- is
 * bracketed with HIP events on the context stream (a pair of events adds a few microseconds to
 * the stream; an odd N samples alternating epilogues alike); on = 0 turns timing off.
 * dbq_kernel_time returns the accumulated milliseconds, the number of timed launches and their
 * algorithmic HBM bytes for one class (0 = Dslash FP64, 1 = Dslash FP32, 2 = FP32 update step: 8
 * vector passes per active rhs) since the last reset. */
int dbq_set_timing(dbq_ctx* ctx, int32_t on);
int dbq_kernel_time(dbq_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches,
                    double* algorithmic_bytes);
int dbq_reset_timing(dbq_ctx* ctx);

/* Library version string. */
const char* dbq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DBQ_H */
