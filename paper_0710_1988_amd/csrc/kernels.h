// Host-side launchers of the dbq device kernels and the data structures they share.
//
// Internal storage (device, per right-hand side), sites in even-odd order:
//   FP64 spinor : double2 [6][V][2]    element (k, s, j) = component c = 2k + j (c = 3*spin + colour)
//   FP32 spinor : float4  [6][V]       element (j, s) = components 2j and 2j+1 at site s
//   FP64 links  : double2 [4][9][V]    U_mu(s)[a][b] at ((mu*9 + 3a + b)*V + s)
//   FP32 links  : float4  [4][3][V]    rows 0 and 1 of U_mu(s) (12 reals); row 2 = conj(row0 x row1)
// Consecutive threads touch consecutive sites, so every load and store is coalesced; FP32 element
// e of a vector holds the same two components as FP64 elements 2e and 2e+1, and the second half
// of every vector holds spins 2 and 3 (gamma5 = -1) in both precisions.
#pragma once

#include <algorithm>

#include "common.h"

namespace dbq {

// ----------------------------------------------------------------------------- per-rhs solver state
enum : int {
  F_CONV = 1,      // recursive residual below the stopping threshold
  F_RELIABLE = 2,  // mixed precision: residual dropped by delta since the last FP64 update
  F_BREAK = 4,     // rho or <rhat, v> vanished: restart with rhat <- r
  F_OMEGA0 = 8,    // omega = 0 in this iteration (restart after the update)
  F_NAN = 16,      // non-finite reduction
  F_DONE = 32,     // FP64 true residual below the stopping threshold (decided on the device)
  F_STALL = 64,    // FP32 iteration no longer reduces the FP64 residual (decided on the device)
};

struct RhsScal {
  zd rho, rho_prev, alpha, omega, beta;
  zd rho_next;     // <rhat, r> of the iteration in progress (<rhat, s> - omega <rhat, t>)
  zd dot;          // last <rhat, v>
  double rr;       // recursive ||r||^2
  double rr_true;  // last FP64 ||b - A x||^2
  double rr_max;   // largest rr since the last reliable update
  double bb;       // ||b||^2
  double stop2;    // tol^2 * bb
  double delta2;   // reliable-update threshold squared (0: none)
  double rhat2;    // ||rhat||^2
  int active;      // iterate this rhs
  int sel;         // selected for a host-requested operation
  int flags;
  int iters;
  int nrel;        // FP64 residual replacements decided on the device (each one FP64 MVP)
  int since;       // iterations since the last residual replacement (mixed precision)
  int stalls;      // consecutive FP64 checks that found too little progress (mixed precision)
  int reproj;      // mixed precision: deflation projection again at each FP64 residual (host-set)
  double rr_prev;  // FP64 ||r||^2 at the previous check (mixed precision)
};

// Mixed precision gives up on an rhs (F_STALL; the solve continues it in FP64 from its current
// solution) after two FP64 checks at which the FP32 recursion claimed a 10x drop, or had run
// STALL_ITERS iterations without a replacement (which forces a check), while the true residual
// fell by less than 2x.  (500 rather than 250 or 150: the same products on 16^4 and 20^3 x 32,
// 12% less time on the lightest twisted-mass shifts at kappa_c, where a forced check also
// restarts the recursion.)
constexpr int STALL_ITERS = 500;

// End of a BiCGStab iteration for one rhs, from a2 = ||r||^2 of the update step: rr = a2, rho
// takes the value the <t, s> epilogue prepared, and the flags that end the rhs's run of
// iterations (convergence claim, reliable update, breakdown, non-finite values) are raised.
// Called by the update step's finalize, or by the <rhat, v> finalize of the next iteration.
__device__ inline void fin_xr(RhsScal& q, double a2) {
  if (!q.active) return;
  q.iters += 1;
  q.since += 1;
  q.rr = a2;
  if (!isfinite(a2)) {
    q.flags |= F_NAN;
    q.active = 0;
    return;
  }
  const zd rn = q.rho_next;
  if (a2 <= q.stop2) q.flags |= F_CONV;
  if (q.delta2 > 0.0) {
    if (a2 > q.rr_max) q.rr_max = a2;
    // a drop by the reliable-update factor, or a long stretch without one (checked for a
    // stall by the FP64 residual that follows), or growth by 100x over the last FP64
    // residual (checked for divergence)
    if (a2 < q.delta2 * q.rr_max || q.since >= STALL_ITERS || a2 > 1e4 * q.rr_prev)
      q.flags |= F_RELIABLE;
  }
  if (norm2(rn) <= 1e-28 * q.rhat2 * a2) q.flags |= F_BREAK;
  if (q.flags & F_OMEGA0) q.flags |= F_BREAK;
  q.rho_prev = q.rho;
  q.rho = rn;
  if (q.flags & (F_CONV | F_RELIABLE | F_BREAK | F_NAN)) q.active = 0;
  // a convergence claim or a reliable update asks for the FP64 residual of this rhs
  if (q.flags & (F_CONV | F_RELIABLE)) q.sel = 1;
}

// ----------------------------------------------------------------------------- batches
constexpr int MAXLAT = 8;
constexpr int DS_BS = 256;  // Dslash threads per block = sites per block
// running sums per rhs in a Dslash epilogue (the <t, s> one uses all 7: <t, s>, |t|^2,
// <rhat, t>, <rhat, s>); the partials hold 3 per slot, then 4 per slot in a second region
constexpr int DS_NSUM = 7;

struct DsLat {
  Geom g;
  const void* links;
  const void* in;   // [nrhs][.][V]
  void* out;
  const void* aux;  // epilogue input with the layout of `in` (rhat, b) or null
  const void* cen;  // half-lattice kernels: the output parity's own input, or null
  int nrhs;
  int rhs_base;     // global rhs index of this lattice's first rhs
  int nsb;          // site blocks (tiles) per rhs
  int blk_begin;    // first logical block of this lattice
  double kappa, mu;
};

// Optional accounting of the algorithmic bytes of a gated launch, done inside the Dslash by the
// blocks of each lattice's first tile or site block: each processed rhs adds its spinor traffic,
// and the first processed rhs of each lattice adds the lattice's links.
struct DsAcct {
  unsigned long long* bytes;  // device accumulator, or null for no accounting
  unsigned long long* tags;   // device, MAXLAT entries: nonzero once this launch counted the
                              // lattice's links (cleared by the launch's finalize)
  int spinor_passes;          // spinor vectors read or written per processed rhs-site
  int spinor_bytes;           // bytes of one spinor at one site
  int link_bytes;             // bytes of the links of one site
};

struct DsBatch {
  DsLat lat[MAXLAT];
  int nlat;
  int nblocks;     // set by the launcher for the chosen rhs-per-thread
  int nrhs_total;
  int pstride;     // partial-sum slots per rhs
  int nb;          // right-hand sides per thread (1, 2 or 4), set by the launcher
  int rgroup;      // thread rhs-groups sharing a sweep over the site blocks, set by the launcher
  int torder;      // LDS tile kernels: order in which blocks visit the tiles (see tile_of_block)
  DsAcct acct;     // zero unless the caller accounts bytes of a gated launch
  int decide;      // RESID finalize also decides convergence / replacement (device loop)
  int schur;       // the lattices' operator is the even-odd reduced one (half vectors)
  // With xr_part set, the <rhat, v> finalize first ends the previous iteration (fin_xr) from the
  // update step's partials of ||r||^2: for rhs j, ceil(xr_nelem[j] / BL_CHUNK) slots of 3
  // doubles (the third is ||r||^2) from xr_part + 3 j xr_pstride.
  const double* xr_part;
  const int* xr_nelem;
  int xr_pstride;
};

enum Epi : int { EPI_NONE = 0, EPI_RHAT = 1, EPI_TS = 2, EPI_RESID = 3 };

// Vector-set description for BLAS-1 kernels over all right-hand sides of a batch.
struct VecSet {
  const long long* off;  // element offset of rhs j (device)
  const int* nelem;      // elements of rhs j (device)
  const int2* blk;       // per block: (rhs, chunk index) (device)
  int nblocks;
  int nrhs;
  int pstride;           // partial slots per rhs (>= max chunks)
};
constexpr int BL_BS = 256;     // BLAS-1 threads per block
constexpr int BL_EPT = 4;      // elements per thread
constexpr int BL_CHUNK = BL_BS * BL_EPT;

// ----------------------------------------------------------------------------- pack.hip
void launch_geometry(hipStream_t s, const Geom& g, int32_t* lex_of_eo, int32_t* nbr);
void pack_spinor_f64(hipStream_t s, const Geom& g, const void* canon, double2* out, int nrhs);
void unpack_spinor_f64(hipStream_t s, const Geom& g, const double2* in, void* canon, int nrhs);
void pack_spinor_f32(hipStream_t s, const Geom& g, const void* canon, float4* out, int nrhs);
void unpack_spinor_f32(hipStream_t s, const Geom& g, const float4* in, void* canon, int nrhs);
void pack_links_f64(hipStream_t s, const Geom& g, const void* canon, double2* out);
void pack_links_f32(hipStream_t s, const Geom& g, const void* canon, float4* out);
// gamma5 applied to packed FP64 vectors (count vectors of 12V elements), out may equal in
void gamma5_f64(hipStream_t s, const double2* in, double2* out, long long V, int count);

// ----------------------------------------------------------------------------- dslash.hip
// Launches the Dslash kernel alone; a launch with an epilogue must be followed by
// launch_ds_finalize on the batch as updated here (site-block counts and block layout).
// nb = right-hand sides per thread (1, 2, 4), or 0 for the LDS-staged tile kernel (FP32 only).
// rgroup = for nb > 0, how many rhs groups of nb sweep the site blocks together (block order:
// rhs chunk, then site block, then rhs within the chunk); for nb = 0, the rhs one block applies
// the operator to in turn with its links held in registers.  0 means all of them.
// Returns the algorithmic HBM bytes of the launch when every rhs is processed (links once, input
// once, output once, plus the epilogue operand).
double launch_dslash_f64(hipStream_t s, DsBatch& b, int dagger, int epi, RhsScal* sc,
                         double* partials, int nb, int rgroup);
double launch_dslash_f32(hipStream_t s, DsBatch& b, int dagger, int epi, RhsScal* sc,
                         double* partials, int nb, int rgroup);
// Half-lattice kernels of the even-odd reduced operator on half vectors [rhs][.][V/2] (the sites
// of one parity): step 1 computes the odd sites, out = D^{-1} (cen + c H_oe in); step 2 the even
// ones, out = D cen - c H_eo in followed by the epilogue; c = lat.kappa, D = 1 + i t gamma5 with
// t = lat.mu (-mu for the dagger, whose hops are those of H^dagger); cen may be null in step 1.
// gate: 0 = every rhs, 1 = the active ones, 2 = the selected ones (needs sc).  nb = 1 or 2 rhs
// per thread (rgroup as for the full operator), or in FP32 nb = 0 for the LDS-staged tile kernel
// (rgroup rhs per block, 0 = all).
void launch_dslash_half_f64(hipStream_t s, DsBatch& b, int step, int dagger, int epi,
                            RhsScal* sc, double* partials, int nb, int rgroup, int gate);
void launch_dslash_half_f32(hipStream_t s, DsBatch& b, int step, int dagger, int epi,
                            RhsScal* sc, double* partials, int nb, int rgroup, int gate);
// partial-sum slots per rhs that every launch shape of the Dslash needs for a lattice
inline int ds_partial_slots(const Geom& g) {
  return std::max(2 * ((g.Vh + DS_BS - 1) / DS_BS), g.V >> (g.lTh + 1));
}
void launch_ds_finalize(hipStream_t s, const DsBatch& b, int epi, RhsScal* sc,
                        const double* partials);
// spinor vectors moved per processed rhs-site for an epilogue (in, out, and the epilogue operand)
inline int ds_spinor_passes(int epi) { return epi != EPI_NONE ? 3 : 2; }

// ----------------------------------------------------------------------------- bicg.hip
// BI_S: r <- s = r - alpha v.  BI_XR: x += alpha p + omega s, r = s - omega t and the next
// search direction p = r + beta (p - omega v) in one pass (beta from the <t, s> epilogue), with
// ||r||^2 into the partials.
enum BicgOp : int { BI_S = 1, BI_XR = 2 };
// FP64 vectors (double2 elements) or FP32 vectors (float4 elements)
void bicg_step_f64(hipStream_t s, int op, const VecSet& vs, double2* x, double2* r,
                   const double2* rhat, double2* p, const double2* v, const double2* t,
                   RhsScal* sc, double* partials);
// BI_XR launches only the update (its inner products into partials): bicg_fin_xr follows.
// acct (timing only, may be null): the XR step adds its algorithmic bytes (8 vector passes per
// active rhs: x, p, s, t, v read, x, r, p written) to *acct.
void bicg_fin_xr(hipStream_t s, const VecSet& vs, RhsScal* sc, const double* partials);
void bicg_step_f32(hipStream_t s, int op, const VecSet& vs, float4* x, float4* r,
                   const float4* rhat, float4* p, const float4* v, const float4* t,
                   RhsScal* sc, double* partials, unsigned long long* acct = nullptr);
// AX_INIT (rhs with active != 0): working r = r64 (copy or narrowed), rhat = p = r, x32 = 0
// (mixed); AX_RESTART (sel != 0): rhat = p = r; AX_REPLACE (sel != 0): r = rhat = p = r64, the
// FP64 residual (narrowed in FP32).  Each sets rho = ||r||^2 through its finalize.
enum BicgAux : int { AX_INIT = 0, AX_RESTART = 1, AX_REPLACE = 2 };
void bicg_aux_f64(hipStream_t s, int op, const VecSet& vs, const double2* r64, double2* r,
                  double2* rhat, double2* p, double2* v, RhsScal* sc, double* partials);
void bicg_aux_f32(hipStream_t s, int op, const VecSet& vs32, const VecSet& vs64,
                  const double2* r64, float4* r, float4* rhat, float4* p, float4* v, float4* x32,
                  RhsScal* sc, double* partials);
// x64 += widen(x32), x32 = 0 for rhs with sel != 0
// Y[:, j] = 0 (k entries) for every rhs j < nrhs whose sel is clear, or with reproj_only whose
// reproj is clear as well (sc points at the first)
void mask_unselected_f64(hipStream_t s, double2* Y, int k, int nrhs, const RhsScal* sc,
                         bool reproj_only);
void bicg_xacc(hipStream_t s, const VecSet& vs32, const VecSet& vs64, double2* x64, float4* x32,
               const RhsScal* sc);

// ----------------------------------------------------------------------------- blas.hip (FP64)
// Tall-skinny products over vectors of n elements (double2):
//   C[i + j*na] = sum_e conj(A_i[e]) * sg(e) * B_j[e]   (sg = -1 for components 6..11 when g5)
// A_i at A + i*lda, B_j at B + j*ldb.  V = sites (for the gamma5 sign: element e of a vector is
// component e / V).
void gram_f64(hipStream_t s, const double2* A, long long lda, int na, const double2* B,
              long long ldb, int nb, long long n, long long V, int g5, double2* C, double* work,
              size_t work_elems);
size_t gram_work_elems(long long n, int na, int nb);
// Y_j (+)= sum_i A_i * (sg) * M[i + j*ldm] for j < nb; beta = 0 overwrites Y, 1 accumulates,
// -1 subtracts (Y_j -= sum ...).  Y_j at Y + j*ldy.
void combine_f64(hipStream_t s, const double2* A, long long lda, int na, const double2* M, int ldm,
                 double2* Y, long long ldy, int nb, long long n, long long V, int g5, int beta);
// C = A^H [B_0, B_1] (na x 2) for the Arnoldi step (no gamma5)
void gram2_f64(hipStream_t s, const double2* A, long long lda, int na, const double2* B,
               long long ldb, long long n, double2* C, double* work, size_t work_elems);
// Arnoldi step with delayed reorthogonalisation: from G = [Q, z_j]^H [z_j, w] ((j+1) x 2, or
// (j+1) x 1 with last) correct Hessenberg column j-1, write column j (rows 0..j) and the
// coefficients m0, m1 (j+1 each) and c1 of the second sweep; start = 1 for a vector that is
// already orthonormal.  j <= 128.
void arn_coef_f64(hipStream_t s, const double2* G, int j, int start, int last, double2* H, int ldh,
                  double2* m0, double2* m1, double* c1);
// In place: col j = sum_{i<=j} Q_i m0[i]; if m1, col j+1 = c1 col(j+1) - sum_{i<=j} Q_i m1[i]
void arn_combine_f64(hipStream_t s, double2* Q, long long ld, int j, long long n, const double2* m0,
                     const double2* m1, const double* c1);
// y = alpha * x (complex scalar from device memory, optional reciprocal of a real norm)
void scale_f64(hipStream_t s, const double2* x, double2* y, long long n, const double* inv_norm_of);
// ||x||^2 per vector (count vectors of n elements, stride ld) into out[count] (device)
void norm2_f64(hipStream_t s, const double2* x, long long ld, int count, long long n, double* out,
               double* work, size_t work_elems);
// y = x (count vectors)
void copy_f64(hipStream_t s, const double2* x, double2* y, long long n);
// y = a - b
void sub_f64(hipStream_t s, const double2* a, const double2* b, double2* y, long long n);
// M[0..count-1][col] = h1 + h2, M[diag_row][col] = sqrt(*nrm2)  (Arnoldi / Gram-Schmidt column)
void write_col_f64(hipStream_t s, double2* M, int ld, int col, int count, const double2* h1,
                   const double2* h2, const double* nrm2, int diag_row);
// c = sqrt(*nrm2) e_1 (length len)
void set_e1_f64(hipStream_t s, double2* c, int len, const double* nrm2);
// deterministic pseudo-random vector (splitmix64 hash of the element index)
void fill_hash_f64(hipStream_t s, double2* x, long long n, unsigned long long seed);
// x = 0 with a kernel (safe inside captured graphs)
void zero_f64(hipStream_t s, double2* x, long long n);

// ----------------------------------------------------------------------------- dense.hip
// Small dense FP64 linear algebra on one workgroup.
// LU with partial pivoting of M (k x k, column-major) and solve M Y = C (k x nrhs); Y overwrites C.
// Writes the 1-norm condition number to cond (device double).
void dense_lu_solve(hipStream_t s, const double2* M, int k, double2* C, int nrhs, double2* work,
                    double* cond);
// GMRES-DR / Arnoldi cycle end, see dense.hip for the meaning of the modes.
struct CycleArgs {
  const double2* Hbar;  // (m+1) x m column-major, ld = m+1
  const double2* c;     // m+1
  int m, k;
  int mode;             // 0: GMRES-DR restart, 1: GMRES-DR final vectors, 2: Ritz (largest Re),
                        // 3: least squares only (GMRES(m) cycle; rho = c - Hbar d into cnew)
  double tol_abs;       // convergence threshold on ||rho|| (modes 0, 1)
  double2* d;           // out: m least-squares coefficients (modes 0, 1)
  double2* P;           // out: (m+1) x (k+1) column-major restart / output basis
  double2* Hnew;        // out: (k+1) x k, ld = m+1 (written into the first k columns)
  double2* cnew;        // out: m+1 (mode 3: rho)
  double2* theta;       // out: m eigenvalues sorted
  double* info;         // out: [0] ||rho||, [1] k_out, [2] converged flag, [3] ritz residual of
                        //      theta[0] (mode 2), [4] eigen-solver failure flag
  double2* work;        // scratch, dense_cycle_work(m) elements
};
size_t dense_cycle_work(int m);
void dense_cycle(hipStream_t s, const CycleArgs& a);
// small triangular solve / matvec helpers used by project_shifts
void dense_trsolve_upper(hipStream_t s, const double2* R, int ldr, int n, double2* z, int nrhs,
                         int ldz);

// ----------------------------------------------------------------------------- force.hip
void launch_link_force(hipStream_t s, const Geom& g, const void* links, double kappa,
                       const void* lambda, const void* x, int nrhs, int kind, void* F);

}  // namespace dbq
