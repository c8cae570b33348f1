// Small dense FP64 complex linear algebra on one workgroup (one wavefront): the k x k solve of
// the deflation step (Sec. 2), and the end of a GMRES-DR / Arnoldi cycle -- least squares on the
// (m+1) x m Hessenberg-like matrix, the harmonic Ritz (or Ritz) eigenproblem, selection of k
// vectors, and the restart basis.  The matrices have at most 129 x 128 entries.
//
// Every phase works on a copy in LDS where it fits: one shared area of 97 x 96 complex entries
// (145.5 KiB), reused phase by phase, holds the (m+1) x m least-squares matrix (m <= 96), then the
// m x m matrix of the eigenproblem (m <= 96) together with its Schur vectors (m <= 67), then the
// restart basis and Hbar times it.  Larger problems use the same code on the global scratch area
// (resident in L2).  The 64 lanes share every step: vectors that one lane would otherwise walk
// serially (pivot search, triangular solves, eigenvectors of the triangular factor) are held one
// entry per lane in registers and move by shuffles, and a Givens rotation of the QR iteration
// updates its two rows, its two columns and the Schur vectors in one phase (one barrier).
#include <cfloat>

#include "kernels.h"

namespace dbq {

namespace {

constexpr int NT = 64;         // one wavefront
constexpr int CY_BS = 256;     // the cycle kernel: four wavefronts (all in the QR iteration)
constexpr int LDS_CAP = 9312;  // double2 entries of the shared area (97 x 96)

__device__ __forceinline__ double cabs_(zd a) { return hypot(a.re, a.im); }
__device__ __forceinline__ zd ld2(const double2* p, int i) {
  const double2 v = p[i];
  return zd{v.x, v.y};
}
__device__ __forceinline__ void st2(double2* p, int i, zd a) { p[i] = make_double2(a.re, a.im); }
__device__ __forceinline__ double wsum(double v) { return wave_sum(v); }
__device__ __forceinline__ double nrm1(zd a) { return fabs(a.re) + fabs(a.im); }

// Orders the LDS (and global) accesses of the lanes of one wavefront: the phases that run on one
// wave while the others wait use it instead of a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A vector of up to 128 entries held across the wavefront: entry i in lane i % 64, in member a
// for i < 64 and b above.  Index arguments are uniform over the wave.
struct WVec {
  zd a, b;
};
__device__ __forceinline__ zd wv_get(const WVec& x, int i) {
  const zd v = i < 64 ? x.a : x.b;
  return zd{__shfl(v.re, i & 63, 64), __shfl(v.im, i & 63, 64)};
}
__device__ __forceinline__ void wv_set(WVec& x, int i, zd v) {
  if (int(threadIdx.x & 63) == (i & 63)) {
    if (i < 64) x.a = v;
    else x.b = v;
  }
}
__device__ __forceinline__ WVec wv_load(const double2* p, int n) {
  const int t = threadIdx.x & 63;
  WVec x;
  x.a = t < n ? ld2(p, t) : zd{0.0, 0.0};
  x.b = t + 64 < n ? ld2(p, t + 64) : zd{0.0, 0.0};
  return x;
}

// ----------------------------------------------------------------------------- reflections
// Householder reflector H = I - f w w^H with H x = alpha e_1, alpha = -phase(x_0) |x|: from x_0
// and |x|^2, w equals x except w_0 = x_0 - alpha.
__device__ __forceinline__ void reflector(zd x0, double nx2, zd& w0, double& f) {
  const double ax0 = cabs_(x0), nx = sqrt(nx2);
  const zd ph = ax0 > 0 ? zd{x0.re / ax0, x0.im / ax0} : zd{1.0, 0.0};
  const zd alpha{-ph.re * nx, -ph.im * nx};
  w0 = x0 - alpha;
  f = 2.0 / (nx2 - ax0 * ax0 + norm2(w0));
}

// col[0..len) <- H col with w = (w0, v[1], ..., v[len-1])
__device__ __forceinline__ void reflect_col(double2* col, const double2* v, zd w0, int len,
                                            double f) {
  zd s = cmulc(w0, ld2(col, 0));
#pragma unroll 4
  for (int i = 1; i < len; ++i) s = s + cmulc(ld2(v, i), ld2(col, i));
  s = f * s;
  st2(col, 0, ld2(col, 0) - w0 * s);
#pragma unroll 4
  for (int i = 1; i < len; ++i) st2(col, i, ld2(col, i) - ld2(v, i) * s);
}

// ----------------------------------------------------------------------------- least squares
// Householder QR of QR ((m+1) x m, ld m+1) with g (m+1 entries) transformed alongside: on exit the
// upper triangle of QR is R and g = Q^H g.  v: scratch of m+1 entries.
__device__ __forceinline__ void ls_qr(double2* QR, double2* g, int m, double2* v) {
  const int t = threadIdx.x, m1 = m + 1;
  for (int j = 0; j < m; ++j) {
    const int len = m1 - j;
    double p = 0;
    for (int i = t; i < len; i += NT) {
      const double2 x = QR[(j + i) + j * m1];
      p += x.x * x.x + x.y * x.y;
      v[i] = x;
    }
    const double nx2 = wsum(p);
    wave_sync();
    if (nx2 == 0.0) continue;
    zd w0;
    double f;
    reflector(ld2(v, 0), nx2, w0, f);
    for (int c = j + t; c <= m; c += NT)
      reflect_col(c < m ? QR + c * m1 + j : g + j, v, w0, len, f);
    wave_sync();
  }
}

// R d = g for upper-triangular R (m x m, ld ldr); d across the wave (0 where R_ii = 0)
__device__ __forceinline__ WVec back_subst(const double2* R, int ldr, const double2* g, int m) {
  const int t = threadIdx.x;
  WVec b = wv_load(g, m);
  for (int j = m - 1; j >= 0; --j) {
    const zd rjj = ld2(R, j + j * ldr);
    const zd dj = (rjj.re != 0.0 || rjj.im != 0.0) ? cdiv(wv_get(b, j), rjj) : zd{0.0, 0.0};
    wv_set(b, j, dj);
    if (t < j) b.a = b.a - ld2(R, t + j * ldr) * dj;
    if (t + 64 < j) b.b = b.b - ld2(R, t + 64 + j * ldr) * dj;
  }
  return b;
}

// ----------------------------------------------------------------------------- LU
// In-place LU with partial pivoting of A (n x n, ld ld); piv[j] = row swapped with j (LDS).
// Returns false if a pivot column is exactly zero (that step is skipped).
__device__ __forceinline__ bool lu_wave(double2* A, int n, int ld, int* piv) {
  const int t = threadIdx.x;
  bool ok = true;
  for (int j = 0; j < n; ++j) {
    double best = -1.0;
    int bi = n;
    for (int i = j + t; i < n; i += NT) {
      const double a = cabs_(ld2(A, i + j * ld));
      if (a > best) {
        best = a;
        bi = i;
      }
    }
    // the largest modulus, the first row among equal ones
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const int p = bi;
    if (t == 0) piv[j] = p;
    if (best == 0.0) ok = false;
    if (p != j)
      for (int c = t; c < n; c += NT) {
        const zd a = ld2(A, j + c * ld), b = ld2(A, p + c * ld);
        st2(A, j + c * ld, b);
        st2(A, p + c * ld, a);
      }
    wave_sync();
    const zd d = ld2(A, j + j * ld);
    if (d.re != 0.0 || d.im != 0.0) {
      for (int i = j + 1 + t; i < n; i += NT)
        st2(A, i + j * ld, cdiv(ld2(A, i + j * ld), d));
      wave_sync();
      const int r = n - j - 1;
      for (int idx = t; idx < r * r; idx += NT) {
        const int i = j + 1 + idx % r, c = j + 1 + idx / r;
        st2(A, i + c * ld,
            ld2(A, i + c * ld) - ld2(A, i + j * ld) * ld2(A, j + c * ld));
      }
    }
    wave_sync();
  }
  return ok;
}

// (LU) x = b with the factors of lu_wave; b and x across the wave
__device__ __forceinline__ void lu_solve_wave(const double2* A, int n, int ld, const int* piv,
                                              WVec& b) {
  const int t = threadIdx.x;
  for (int j = 0; j < n; ++j) {
    const int p = piv[j];
    if (p != j) {
      const zd bj = wv_get(b, j), bp = wv_get(b, p);
      wv_set(b, j, bp);
      wv_set(b, p, bj);
    }
  }
  for (int j = 0; j < n; ++j) {  // L y = b (unit diagonal)
    const zd bj = wv_get(b, j);
    if (t > j && t < n) b.a = b.a - ld2(A, t + j * ld) * bj;
    if (t + 64 > j && t + 64 < n) b.b = b.b - ld2(A, t + 64 + j * ld) * bj;
  }
  for (int j = n - 1; j >= 0; --j) {  // U x = y
    const zd xj = cdiv(wv_get(b, j), ld2(A, j + j * ld));
    wv_set(b, j, xj);
    if (t < j) b.a = b.a - ld2(A, t + j * ld) * xj;
    if (t + 64 < j) b.b = b.b - ld2(A, t + 64 + j * ld) * xj;
  }
}

// ----------------------------------------------------------------------------- k x k solve
// (LU) x = b for lane t's own column, held lane-interleaved (entry i at X[i * 64 + t], so a wave's
// accesses hit consecutive LDS slots); the factors are read by all lanes at once
__device__ __forceinline__ void lu_solve_own(const double2* A, int n, const int* piv, double2* X,
                                             int t) {
  for (int j = 0; j < n; ++j) {
    const int p = piv[j];
    if (p != j) {
      const zd a = ld2(X, j * 64 + t), b = ld2(X, p * 64 + t);
      st2(X, j * 64 + t, b);
      st2(X, p * 64 + t, a);
    }
  }
  for (int i = 0; i < n; ++i) {  // L y = b (unit diagonal)
    zd s = ld2(X, i * 64 + t);
    for (int j = 0; j < i; ++j) s = s - ld2(A, i + j * n) * ld2(X, j * 64 + t);
    st2(X, i * 64 + t, s);
  }
  for (int i = n - 1; i >= 0; --i) {  // U x = y
    zd s = ld2(X, i * 64 + t);
    for (int j = i + 1; j < n; ++j) s = s - ld2(A, i + j * n) * ld2(X, j * 64 + t);
    st2(X, i * 64 + t, cdiv(s, ld2(A, i + i * n)));
  }
}

// M^{-1} C and the 1-norm condition number of M.  With X (k x 64 LDS slots) every lane solves
// its own columns (inverse columns, then columns of C); otherwise the wave solves one column at a
// time with the vector spread over its lanes.
__device__ __forceinline__ void lu_solve_body(const double2* __restrict__ M, int k,
                                              double2* __restrict__ C, int nrhs, double2* LU,
                                              double2* X, double* cond, int* piv) {
  const int t = threadIdx.x;
  for (int i = t; i < k * k; i += NT) LU[i] = M[i];
  // 1-norm of M: largest column sum
  double n1 = 0;
  for (int j = t; j < k; j += NT) {
    double s = 0;
    for (int i = 0; i < k; ++i) s += cabs_(ld2(M, i + j * k));
    n1 = fmax(n1, s);
  }
  for (int o = 32; o > 0; o >>= 1) n1 = fmax(n1, __shfl_xor(n1, o, 64));
  wave_sync();
  if (!lu_wave(LU, k, k, piv)) {
    if (t == 0) *cond = INFINITY;
    return;
  }
  // 1-norm of M^{-1}, one column at a time
  double ninv = 0;
  if (X) {
    for (int c0 = 0; c0 < k; c0 += 64) {
      const int j = c0 + t;
      if (j < k) {
        for (int i = 0; i < k; ++i) X[i * 64 + t] = make_double2(i == j ? 1.0 : 0.0, 0.0);
        lu_solve_own(LU, k, piv, X, t);
        double s = 0;
        for (int i = 0; i < k; ++i) s += cabs_(ld2(X, i * 64 + t));
        ninv = fmax(ninv, s);
      }
    }
    for (int o = 32; o > 0; o >>= 1) ninv = fmax(ninv, __shfl_xor(ninv, o, 64));
  } else {
    for (int j = 0; j < k; ++j) {
      WVec e{zd{t == j ? 1.0 : 0.0, 0.0}, zd{t + 64 == j ? 1.0 : 0.0, 0.0}};
      lu_solve_wave(LU, k, k, piv, e);
      const double s = wsum((t < k ? cabs_(e.a) : 0.0) + (t + 64 < k ? cabs_(e.b) : 0.0));
      ninv = fmax(ninv, s);
    }
  }
  if (t == 0) {
    const double c = n1 * ninv;
    *cond = isfinite(c) ? c : INFINITY;
  }
  // Y = M^{-1} C (solved with the factors for accuracy)
  if (X) {
    for (int c0 = 0; c0 < nrhs; c0 += 64) {
      const int j = c0 + t;
      if (j < nrhs) {
        double2* cj = C + j * k;
        for (int i = 0; i < k; ++i) X[i * 64 + t] = cj[i];
        lu_solve_own(LU, k, piv, X, t);
        for (int i = 0; i < k; ++i) cj[i] = X[i * 64 + t];
      }
    }
  } else {
    for (int j = 0; j < nrhs; ++j) {
      double2* cj = C + j * k;
      WVec b = wv_load(cj, k);
      lu_solve_wave(LU, k, k, piv, b);
      if (t < k) st2(cj, t, b.a);
      if (t + 64 < k) st2(cj, t + 64, b.b);
    }
  }
}

__global__ __launch_bounds__(NT) void k_lu_solve(const double2* __restrict__ M, int k,
                                                 double2* __restrict__ C, int nrhs,
                                                 double2* __restrict__ work, double* cond) {
  __shared__ double2 sh[LDS_CAP];
  __shared__ int piv[128];
  if (k * k + 64 * k <= LDS_CAP) lu_solve_body(M, k, C, nrhs, sh, sh + k * k, cond, piv);
  else if (k * k <= LDS_CAP) lu_solve_body(M, k, C, nrhs, sh, nullptr, cond, piv);
  else lu_solve_body(M, k, C, nrhs, work, nullptr, cond, piv);
}

// ----------------------------------------------------------------------------- eigenproblem
// Householder reduction of G (n x n, ld n) to upper Hessenberg form.  Reflector j (acting on rows
// and columns j+1..j+hl[j]) is kept below the subdiagonal of column j, its first entry in w0s[j],
// its factor in fs[j] (0: identity) and its length in hl[j], for form_q; the caller zeroes that
// part afterwards.  Column j's nonzeros below the diagonal end at some row `last` (after a thick
// restart the matrix is Hessenberg but for a dense leading block, whose fill moves down one row
// per reduced column), so the reflector and both applications are restricted to rows and columns
// j+1..last: the terms left out are products with exact zeros.
__device__ __forceinline__ void hessenberg(double2* G, int n, int ld, double2* v, double2* w0s, double* fs,
                                           int* hl) {
  const int t = threadIdx.x;
  for (int j = 0; j + 2 < n; ++j) {
    int lastl = j + 1;
    for (int r = j + 2 + t; r < n; r += NT) {
      const double2 x = G[r + j * ld];
      if (x.x != 0.0 || x.y != 0.0) lastl = r;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lastl = max(lastl, __shfl_xor(lastl, o, 64));
    const int len = lastl - j;
    double p = 0;
    for (int i = t; i < len; i += NT) {
      const double2 x = G[(j + 1 + i) + j * ld];
      p += x.x * x.x + x.y * x.y;
      v[i] = x;
    }
    const double nx2 = wsum(p);
    wave_sync();
    zd w0{0.0, 0.0};
    double f = 0.0;
    if (nx2 != 0.0) reflector(ld2(v, 0), nx2, w0, f);
    if (t == 0) {
      w0s[j] = make_double2(w0.re, w0.im);
      fs[j] = f;
      hl[j] = len;
    }
    if (nx2 == 0.0) continue;
    // left: rows j+1..j+len, columns j..n-1
    for (int c = j + t; c < n; c += NT) reflect_col(G + c * ld + j + 1, v, w0, len, f);
    wave_sync();
    // right: all rows, columns j+1..j+len
    for (int r = t; r < n; r += NT) {
      double2* row = G + r + (j + 1) * ld;
      zd s = ld2(row, 0) * w0;
#pragma unroll 4
      for (int i = 1; i < len; ++i) s = s + ld2(row, i * ld) * ld2(v, i);
      s = f * s;
      st2(row, 0, ld2(row, 0) - s * conj(w0));
#pragma unroll 4
      for (int i = 1; i < len; ++i)
        st2(row, i * ld, ld2(row, i * ld) - s * conj(ld2(v, i)));
    }
    wave_sync();
    for (int i = 1 + t; i < len; i += NT) G[(j + 1 + i) + j * ld] = v[i];
    wave_sync();
  }
}

// Q = H_0 H_1 ... H_{n-3} (so that G_in = Q G_out Q^H), accumulated backwards (Q <- H_j Q), one
// column per lane: no lane reads another lane's column, so no barriers.
__device__ __forceinline__ void form_q(const double2* G, int n, int ld, const double2* w0s,
                                       const double* fs, const int* hl, double2* Q) {
  const int t = threadIdx.x;
  for (int c = t; c < n; c += NT) {
    double2* qc = Q + c * ld;
    for (int r = 0; r < n; ++r) qc[r] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    for (int j = min(n - 3, c - 1); j >= 0; --j) {
      const double f = fs[j];
      if (f == 0.0) continue;
      const int len = hl[j];
      const zd w0 = ld2(w0s, j);
      const double2* w = G + j * ld + j + 1;  // w[i], i >= 1
      double2* col = qc + j + 1;
      zd s = cmulc(w0, ld2(col, 0));
#pragma unroll 4
      for (int i = 1; i < len; ++i) s = s + cmulc(ld2(w, i), ld2(col, i));
      s = f * s;
      st2(col, 0, ld2(col, 0) - w0 * s);
#pragma unroll 4
      for (int i = 1; i < len; ++i) st2(col, i, ld2(col, i) - ld2(w, i) * s);
    }
  }
}

// Shifted QR iteration (single Wilkinson shift, Givens bulge chase) on the upper Hessenberg G,
// reducing it to upper triangular Schur form T with G_in = Z T Z^H; Z holds the Hessenberg
// reduction's Q on entry.  All four wavefronts of the block take part: every wave computes each
// rotation from the two entries it annihilates, then, in one phase closed by one barrier, wave 0
// rotates the two rows, wave 1 the two columns, wave 3 the 2 x 2 block where both act, and waves
// 2 and 3 the Schur vectors (zlds, Z in LDS).  Otherwise the sweep's rotations are recorded (rc,
// rs) and applied to the rows of Z after the sweep.  Returns false if it did not converge.
__device__ __forceinline__ bool schur(double2* G, double2* Z, int n, int ld, bool zlds, double* rc,
                                      double2* rs) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double eps = DBL_EPSILON;
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    // the largest l in 1..hi with a negligible subdiagonal entry G[l][l-1] (0 if none)
    int l = 0;
    for (int qb = 0; qb <= hi; qb += 64) {
      const int q = qb + lane;
      bool neg = false;
      if (q >= 1 && q <= hi) {
        const double sd = nrm1(ld2(G, (q - 1) + (q - 1) * ld)) + nrm1(ld2(G, q + q * ld));
        neg = nrm1(ld2(G, q + (q - 1) * ld)) <= eps * (sd > 0 ? sd : 1e-300);
      }
      const unsigned long long mask = __ballot(neg);
      if (mask) l = qb + 63 - __clzll(mask);
    }
    __syncthreads();  // every wave has read the entry before it is zeroed
    if (l > 0 && tid == 0) G[l + (l - 1) * ld] = make_double2(0.0, 0.0);
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (total > 60 * n) return false;
    // shift (every thread computes it)
    zd mu;
    {
      const zd a = ld2(G, (hi - 1) + (hi - 1) * ld), b = ld2(G, (hi - 1) + hi * ld);
      const zd c = ld2(G, hi + (hi - 1) * ld), d = ld2(G, hi + hi * ld);
      if (iter > 0 && iter % 11 == 0) {
        mu = d + zd{fabs(c.re) + fabs(c.im), 0.0};  // exceptional shift
      } else {
        const zd half{0.5 * (a.re - d.re), 0.5 * (a.im - d.im)};
        const zd disc2 = half * half + b * c;
        const double r = cabs_(disc2);
        double sr = sqrt(0.5 * (r + disc2.re)), si = sqrt(fmax(0.0, 0.5 * (r - disc2.re)));
        if (disc2.im < 0) si = -si;
        const zd sq{sr, si};
        const zd mid{0.5 * (a.re + d.re), 0.5 * (a.im + d.im)};
        const zd m1 = mid + sq, m2 = mid - sq;
        mu = (cabs_(m1 - d) <= cabs_(m2 - d)) ? m1 : m2;
      }
    }
    for (int kk = l; kk < hi; ++kk) {
      zd x, y;
      if (kk == l) {
        x = ld2(G, l + l * ld) - mu;
        y = ld2(G, (l + 1) + l * ld);
      } else {
        x = ld2(G, kk + (kk - 1) * ld);
        y = ld2(G, (kk + 1) + (kk - 1) * ld);
      }
      // c = |x| / rho, s = (x / |x|) conj(y) / rho, rho = sqrt(|x|^2 + |y|^2) (entries far from
      // the range limits: no hypot-style scaling)
      const double nx = x.re * x.re + x.im * x.im, ny = y.re * y.re + y.im * y.im;
      double c;
      zd s;
      if (nx + ny == 0.0) {
        c = 1.0;
        s = zd{0.0, 0.0};
      } else if (nx == 0.0) {
        c = 0.0;
        s = zd{1.0, 0.0};
      } else {
        const double irho = rsqrt(nx + ny), iax = rsqrt(nx);
        c = nx * iax * irho;
        const zd ph{x.re * iax, x.im * iax};
        s = ph * conj(y);
        s = zd{s.re * irho, s.im * irho};
      }
      // rows kk, kk+1 over the columns outside {kk, kk+1} from kk-1 (from kk at the start of the
      // sweep, where column l-1 holds zeros), the bulge left in column kk-1 set to exactly zero;
      // columns kk, kk+1 over the rows up to min(kk+2, hi) outside {kk, kk+1}; the 2 x 2 block
      // (rows first, then columns); the Schur vectors
      const int j0 = kk == l ? kk : kk - 1;
      const int rmax = kk + 2 < hi ? kk + 2 : hi;
      if (wv == 0) {
        for (int q = lane; q < n; q += 64)
          if (q >= j0 && q != kk && q != kk + 1) {
            const zd a = ld2(G, kk + q * ld), b = ld2(G, (kk + 1) + q * ld);
            st2(G, kk + q * ld, c * a + s * b);
            st2(G, (kk + 1) + q * ld, q == kk - 1 ? zd{0.0, 0.0} : c * b - conj(s) * a);
          }
      } else if (wv == 1) {
        for (int q = lane; q <= rmax; q += 64)
          if (q != kk && q != kk + 1) {
            const zd a = ld2(G, q + kk * ld), b = ld2(G, q + (kk + 1) * ld);
            st2(G, q + kk * ld, c * a + conj(s) * b);
            st2(G, q + (kk + 1) * ld, c * b - s * a);
          }
      } else {
        if (wv == 3 && lane == 0) {
          const zd a11 = ld2(G, kk + kk * ld), a12 = ld2(G, kk + (kk + 1) * ld);
          const zd a21 = ld2(G, (kk + 1) + kk * ld), a22 = ld2(G, (kk + 1) + (kk + 1) * ld);
          const zd b11 = c * a11 + s * a21, b12 = c * a12 + s * a22;
          const zd b21 = c * a21 - conj(s) * a11, b22 = c * a22 - conj(s) * a12;
          st2(G, kk + kk * ld, c * b11 + conj(s) * b12);
          st2(G, kk + (kk + 1) * ld, c * b12 - s * b11);
          st2(G, (kk + 1) + kk * ld, c * b21 + conj(s) * b22);
          st2(G, (kk + 1) + (kk + 1) * ld, c * b22 - s * b21);
        }
        if (zlds) {
          const int q = (wv - 2) * 64 + lane;
          if (q < n) {
            const zd a = ld2(Z, q + kk * ld), b = ld2(Z, q + (kk + 1) * ld);
            st2(Z, q + kk * ld, c * a + conj(s) * b);
            st2(Z, q + (kk + 1) * ld, c * b - s * a);
          }
        } else if (wv == 2 && lane == 0) {
          rc[kk] = c;
          rs[kk] = make_double2(s.re, s.im);
        }
      }
      __syncthreads();
    }
    if (!zlds) {
      // the sweep's rotations on the rows of Z: column kk is final after rotation kk, column
      // kk+1 carried to the next one; the untouched columns are loaded ahead in groups of 16
      for (int r = tid; r < n; r += blockDim.x) {
        zd za = ld2(Z, r + l * ld);
        for (int kb = l; kb < hi; kb += 16) {
          const int cnt = hi - kb < 16 ? hi - kb : 16;
          zd zb[16];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (u < cnt) zb[u] = ld2(Z, r + (kb + 1 + u) * ld);
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (u < cnt) {
              const double cc = rc[kb + u];
              const zd ss = ld2(rs, kb + u);
              st2(Z, r + (kb + u) * ld, cc * za + conj(ss) * zb[u]);
              za = cc * zb[u] - ss * za;
            }
        }
        st2(Z, r + hi * ld, za);
      }
    }
    ++iter;
    ++total;
  }
  __syncthreads();
  return true;
}

// Eigenvector of the upper-triangular T (n x n) for diagonal position q, y with y_q = 1 and
// y_j = 0 above q, solved backwards column by column across the wave; returns g = Z y normalised
// in out[0..n) (column of ld-strided storage) and writes out[n] = 0 when pad.
__device__ __forceinline__ void tri_eigvec(const double2* T, const double2* Z, int n, int ld, int q,
                                           double tnorm, double2* out, bool pad) {
  const int t = threadIdx.x & 63;
  const zd th = ld2(T, q + q * ld);
  const double small = fmax(DBL_EPSILON * tnorm, 1e-300);
  WVec acc{zd{0.0, 0.0}, zd{0.0, 0.0}};
  WVec y{zd{0.0, 0.0}, zd{0.0, 0.0}};
  wv_set(y, q, zd{1.0, 0.0});
  zd yj{1.0, 0.0};
  for (int j = q; j >= 1; --j) {
    if (t < j) acc.a = acc.a + ld2(T, t + j * ld) * yj;
    if (t + 64 < j) acc.b = acc.b + ld2(T, t + 64 + j * ld) * yj;
    zd d = ld2(T, (j - 1) + (j - 1) * ld) - th;
    if (cabs_(d) < small) d = zd{small, 0.0};
    yj = -cdiv(wv_get(acc, j - 1), d);
    wv_set(y, j - 1, yj);
  }
  zd g[2];
  double nn = 0;
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const int r = slot * 64 + t;
    zd s{0.0, 0.0};
    if (slot * 64 < n)
      for (int j = 0; j <= q; ++j) {
        const zd yv = wv_get(y, j);
        if (r < n) s = s + ld2(Z, r + j * ld) * yv;
      }
    g[slot] = s;
    if (r < n) nn += norm2(s);
  }
  nn = 1.0 / sqrt(wsum(nn));
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const int r = slot * 64 + t;
    if (r < n) st2(out, r, zd{g[slot].re * nn, g[slot].im * nn});
  }
  if (pad && t == 0) out[n] = make_double2(0.0, 0.0);
}

// orthonormalise column q of P (len rows, ld ldp) against columns 0..q-1 (Gram-Schmidt twice);
// h: scratch of q entries
__device__ __forceinline__ void orth_column(double2* P, int ldp, int len, int q, double2* h) {
  const int t = threadIdx.x;
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = t; i < q; i += NT) {
      zd s{0, 0};
      for (int r = 0; r < len; ++r) s = s + cmulc(ld2(P, r + i * ldp), ld2(P, r + q * ldp));
      st2(h, i, s);
    }
    wave_sync();
    for (int r = t; r < len; r += NT) {
      zd w = ld2(P, r + q * ldp);
      for (int i = 0; i < q; ++i) w = w - ld2(P, r + i * ldp) * ld2(h, i);
      st2(P, r + q * ldp, w);
    }
    wave_sync();
  }
  double p = 0;
  for (int r = t; r < len; r += NT) p += norm2(ld2(P, r + q * ldp));
  const double nn = sqrt(wsum(p));
  const double f = nn > 0 ? 1.0 / nn : 0.0;
  for (int r = t; r < len; r += NT) {
    const zd w = ld2(P, r + q * ldp);
    st2(P, r + q * ldp, zd{w.re * f, w.im * f});
  }
  wave_sync();
}

// ----------------------------------------------------------------------------- cycle phases
// least squares min || c - Hbar d || (QR: m1 x m area, g: m1 entries); rho = c - Hbar d into rho
// (LDS), and cnew in mode 3; returns ||rho|| in every lane
__device__ __forceinline__ double phase_ls(const CycleArgs& a, double2* QR, double2* g,
                                           double2* v, double2* rho) {
  const int t = threadIdx.x, m = a.m, m1 = m + 1;
  const double2* H = a.Hbar;
  for (int i = t; i < m1 * m; i += NT) QR[i] = H[i];
  for (int i = t; i < m1; i += NT) g[i] = a.c[i];
  wave_sync();
  ls_qr(QR, g, m, v);
  const WVec d = back_subst(QR, m1, g, m);
  if (t < m) st2(a.d, t, d.a);
  if (t + 64 < m) st2(a.d, t + 64, d.b);
  double p = 0;
  for (int rb = 0; rb < m1; rb += NT) {
    const int r = rb + t;
    zd s = r < m1 ? ld2(a.c, r) : zd{0.0, 0.0};
    for (int j = 0; j < m; ++j) {
      const zd dj = wv_get(d, j);
      if (r < m1) s = s - ld2(H, r + j * m1) * dj;
    }
    if (r < m1) {
      st2(rho, r, s);
      if (a.mode == 3) st2(a.cnew, r, s);
      p += norm2(s);
    }
  }
  wave_sync();
  return sqrt(wsum(p));
}

// harmonic Ritz matrix G = H_m + |h_{m+1,m}|^2 f e_m^T with H_m^H f = e_m (Bm: m x m area that
// G then overwrites), or the Ritz matrix G = H_m (mode 2)
__device__ __forceinline__ void phase_g(const CycleArgs& a, double2* G, int ld, int* piv) {
  const int t = threadIdx.x, m = a.m, m1 = m + 1;
  const double2* H = a.Hbar;
  WVec f{zd{0.0, 0.0}, zd{0.0, 0.0}};
  if (a.mode != 2) {
    for (int i = t; i < m * m; i += NT) {
      const int r = i % m, c = i / m;
      st2(G, r + c * ld, conj(ld2(H, c + r * m1)));
    }
    wave_sync();
    lu_wave(G, m, ld, piv);
    wv_set(f, m - 1, zd{1.0, 0.0});
    lu_solve_wave(G, m, ld, piv, f);
    wave_sync();
  }
  for (int i = t; i < m * m; i += NT) {
    const int r = i % m, c = i / m;
    G[r + c * ld] = H[r + c * m1];
  }
  wave_sync();
  if (a.mode != 2) {
    const double h2 = norm2(ld2(H, m + (m - 1) * m1));
    if (t < m) st2(G, t + (m - 1) * ld, ld2(G, t + (m - 1) * ld) + h2 * f.a);
    if (t + 64 < m)
      st2(G, t + 64 + (m - 1) * ld, ld2(G, t + 64 + (m - 1) * ld) + h2 * f.b);
    wave_sync();
  }
}

// Hessenberg form of G (m x m) and the Q of the reduction in Z (one wave)
__device__ __forceinline__ void phase_hess(const CycleArgs& a, double2* G, double2* Z, int ld, double2* v,
                                           double2* w0s, double* fs, int* hl) {
  const int t = threadIdx.x, m = a.m;
  hessenberg(G, m, ld, v, w0s, fs, hl);
  form_q(G, m, ld, w0s, fs, hl, Z);
  wave_sync();
  for (int c = t; c < m; c += NT)
    for (int r = c + 2; r < m; ++r) G[r + c * ld] = make_double2(0.0, 0.0);
  wave_sync();
}

// eigenvalues of the Schur form T (in G) sorted into a.theta and order[]; returns the number of
// vectors to keep (in every lane) and the largest |entry| of T in tn (one wave)
__device__ __forceinline__ int phase_sort(const CycleArgs& a, const double2* G, int ld, int* order,
                                          int* s_kout, double& tn) {
  const int t = threadIdx.x, m = a.m, k = a.k;
  // sort: |theta| ascending (harmonic) or Re descending (Ritz), ties by (Re, Im, index)
  for (int i = t; i < m; i += NT) {
    const zd ti = ld2(G, i + i * ld);
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const zd tj = ld2(G, j + j * ld);
      bool less;
      if (a.mode != 2) {
        const double ai = cabs_(ti), aj = cabs_(tj);
        less = (aj < ai) || (aj == ai && (tj.re < ti.re || (tj.re == ti.re && (tj.im < ti.im || (tj.im == ti.im && j < i)))));
      } else {
        less = (tj.re > ti.re) || (tj.re == ti.re && (tj.im > ti.im || (tj.im == ti.im && j < i)));
      }
      rank += less ? 1 : 0;
    }
    order[rank] = i;
  }
  wave_sync();
  for (int i = t; i < m; i += NT) a.theta[i] = G[order[i] + order[i] * ld];
  if (t == 0) {
    int kout = k;
    if (a.mode == 1 && k < m) {
      const zd x = ld2(G, order[k - 1] + order[k - 1] * ld);
      const zd y = ld2(G, order[k] + order[k] * ld);
      const double sc = cabs_(x);
      if (fabs(x.im) > 1e-3 * sc && cabs_(x - conj(y)) <= 1e-3 * sc) kout = k - 1;
    }
    *s_kout = kout;
    a.info[1] = kout;
  }
  double mx = 0;
  for (int i = t; i < m * m; i += NT) mx = fmax(mx, cabs_(ld2(G, i % m + (i / m) * ld)));
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  tn = mx;
  wave_sync();
  return *s_kout;
}

// P: orthonormal basis of the ks selected eigenvectors (already in P's columns) padded with a zero
// row, then the extra column (rho in mode 0, e_{m+1} in mode 2); then Hnew = P^H Hbar P_k and
// cnew = P^H rho (mode 0).  P: (m+1) x (k+1) area, T1: (m+1) x k area.
__device__ __forceinline__ void phase_restart(const CycleArgs& a, double2* P, double2* T1, int ks,
                                              const double2* rho, double2* h) {
  const int t = threadIdx.x, m = a.m, m1 = m + 1, k = a.k;
  const double2* H = a.Hbar;
  for (int q = 0; q < ks; ++q) orth_column(P, m1, m1, q, h);
  if (a.mode == 2) {
    if (t == 0) {
      const double hm = cabs_(ld2(H, m + (m - 1) * m1));
      a.info[3] = hm * cabs_(ld2(P, m - 1));
      P[m + k * m1] = make_double2(1.0, 0.0);
    }
    wave_sync();
  } else if (a.mode == 0) {
    for (int r = t; r < m1; r += NT) P[r + k * m1] = rho[r];
    wave_sync();
    orth_column(P, m1, m1, k, h);
  }
  if (a.mode == 1) return;
  for (int i = t; i < m1 * k; i += NT) {
    const int r = i % m1, c = i / m1;
    zd s{0, 0};
    for (int j = 0; j < m; ++j) s = s + ld2(H, r + j * m1) * ld2(P, j + c * m1);
    st2(T1, r + c * m1, s);
  }
  wave_sync();
  for (int i = t; i < (k + 1) * k; i += NT) {
    const int r = i % (k + 1), c = i / (k + 1);
    zd s{0, 0};
    for (int j = 0; j < m1; ++j) s = s + cmulc(ld2(P, j + r * m1), ld2(T1, j + c * m1));
    st2(a.Hnew, r + c * m1, s);
  }
  for (int r = t; r < m1; r += NT) {
    zd s{0, 0};
    if (r <= k && a.mode == 0)
      for (int j = 0; j < m1; ++j) s = s + cmulc(ld2(P, j + r * m1), ld2(rho, j));
    st2(a.cnew, r, s);
  }
}

__global__ __launch_bounds__(CY_BS) void k_cycle(CycleArgs a) {
  const int t = threadIdx.x, wv = t >> 6;
  const int m = a.m, m1 = m + 1, k = a.k;
  // the eigenproblem's matrices (G, its Schur vectors Z) are stored with an odd leading
  // dimension: a lane per column then walks LDS at an odd multiple of 16 bytes, which spreads a
  // wave's accesses over all banks (a stride of m = 64 or 96 entries would hit one bank group)
  const int ld = m | 1;
  // global scratch for what does not fit in LDS
  double2* w = a.work;
  double2* wA = w;                 // (m+1) x m
  double2* wG = wA + m1 * m;       // m x m, ld
  double2* wZ = wG + m * ld;       // m x m, ld
  double2* wT1 = wZ + m * ld;      // (m+1) x m
  __shared__ double2 sh[LDS_CAP];
  __shared__ double2 v[129];
  __shared__ double2 gr[129];      // c transformed by the least squares, then rho
  __shared__ double2 w0s[128];     // Hessenberg reflectors, then the sweep's rotations
  __shared__ double fs[128];
  __shared__ int hl[128];          // Hessenberg reflector lengths
  __shared__ int piv[128];
  __shared__ int order[128];
  __shared__ int s_kout, s_exit;
  __shared__ double s_tn;
  const bool g_lds = m * ld <= LDS_CAP, z_lds = 2 * m * ld <= LDS_CAP;

  // ---- wave 0: least squares, the eigenproblem's matrix and its Hessenberg form
  if (wv == 0) {
    int ex = 0;
    if (a.mode == 0 || a.mode == 1 || a.mode == 3) {
      const double rn = m1 * m <= LDS_CAP ? phase_ls(a, sh, gr, v, gr) : phase_ls(a, wA, gr, v, gr);
      const bool conv = rn <= a.tol_abs;
      if (t == 0) {
        a.info[0] = rn;
        a.info[2] = conv ? 1.0 : 0.0;
      }
      ex = (a.mode == 0 && conv) || a.mode == 3;
    }
    if (t == 0) s_exit = ex;
    if (!ex) {
      if (z_lds) {
        phase_g(a, sh, ld, piv);
        phase_hess(a, sh, sh + m * ld, ld, v, w0s, fs, hl);
      } else if (g_lds) {
        phase_g(a, sh, ld, piv);
        phase_hess(a, sh, wZ, ld, v, w0s, fs, hl);
      } else {
        phase_g(a, wG, ld, piv);
        phase_hess(a, wG, wZ, ld, v, w0s, fs, hl);
      }
    }
  }
  __syncthreads();
  if (s_exit) return;
  // ---- all waves: the QR iteration
  const bool ok = z_lds ? schur(sh, sh + m * ld, m, ld, true, fs, w0s)
                        : (g_lds ? schur(sh, wZ, m, ld, false, fs, w0s)
                                 : schur(wG, wZ, m, ld, false, fs, w0s));
  // ---- wave 0: selection
  if (wv == 0) {
    if (t == 0) a.info[4] = ok ? 0.0 : 1.0;
    double tn;
    g_lds ? phase_sort(a, sh, ld, order, &s_kout, tn) : phase_sort(a, wG, ld, order, &s_kout, tn);
    if (t == 0) s_tn = tn;
    for (int i = t; i < m1 * (k + 1); i += NT) a.P[i] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  // ---- all waves: eigenvectors of the selected values into the columns of P (padded with a
  // zero row), one vector per wave at a time
  const int ks = s_kout;
  const double tn = s_tn;
  for (int q = wv; q < ks; q += CY_BS / 64) {
    const int col = order[q];
    if (z_lds) tri_eigvec(sh, sh + m * ld, m, ld, col, tn, a.P + q * m1, true);
    else if (g_lds) tri_eigvec(sh, wZ, m, ld, col, tn, a.P + q * m1, true);
    else tri_eigvec(wG, wZ, m, ld, col, tn, a.P + q * m1, true);
  }
  __syncthreads();
  if (wv != 0) return;
  // restart basis and Hnew, in LDS where P and Hbar P fit
  if (m1 * (2 * k + 1) <= LDS_CAP) {
    double2* P = sh;
    double2* T1 = sh + m1 * (k + 1);
    for (int i = t; i < m1 * (k + 1); i += NT) P[i] = a.P[i];
    wave_sync();
    phase_restart(a, P, T1, ks, gr, v);
    wave_sync();
    for (int i = t; i < m1 * (k + 1); i += NT) a.P[i] = P[i];
  } else {
    phase_restart(a, a.P, wT1, ks, gr, v);
  }
}

__global__ void k_trsolve(const double2* __restrict__ R, int ldr, int n, double2* __restrict__ z,
                          int nrhs, int ldz) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double2* b = z + j * ldz;
  for (int i = n - 1; i >= 0; --i) {
    zd s = ld2(b, i);
    for (int c = i + 1; c < n; ++c) s = s - ld2(R, i + c * ldr) * ld2(b, c);
    const zd d = ld2(R, i + i * ldr);
    st2(b, i, (d.re != 0.0 || d.im != 0.0) ? cdiv(s, d) : zd{0.0, 0.0});
  }
}

}  // namespace

size_t dense_cycle_work(int m) {
  const size_t m1 = m + 1;
  return 2 * m1 * m + 2 * size_t(m) * size_t(m | 1) + 8;
}

void dense_lu_solve(hipStream_t s, const double2* M, int k, double2* C, int nrhs, double2* work,
                    double* cond) {
  DBQ_CHECK(k >= 1 && k <= 128, "dense_lu_solve: k must be in 1..128");
  hipLaunchKernelGGL(k_lu_solve, dim3(1), dim3(NT), 0, s, M, k, C, nrhs, work, cond);
  DBQ_HIP(hipGetLastError());
}

void dense_cycle(hipStream_t s, const CycleArgs& a) {
  DBQ_CHECK(a.m >= 2 && a.m <= 128 && a.k >= 1 && a.k < a.m, "dense_cycle: bad (m, k)");
  hipLaunchKernelGGL(k_cycle, dim3(1), dim3(CY_BS), 0, s, a);
  DBQ_HIP(hipGetLastError());
}

void dense_trsolve_upper(hipStream_t s, const double2* R, int ldr, int n, double2* z, int nrhs,
                         int ldz) {
  hipLaunchKernelGGL(k_trsolve, dim3((nrhs + 63) / 64), dim3(64), 0, s, R, ldr, n, z, nrhs, ldz);
  DBQ_HIP(hipGetLastError());
}

}  // namespace dbq
