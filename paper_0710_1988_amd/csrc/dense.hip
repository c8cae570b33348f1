// Small dense FP64 complex linear algebra on one workgroup (one wavefront): the k x k solve of
// the deflation step (Sec. 2), and the end of a GMRES-DR / Arnoldi cycle -- least squares on the
// (m+1) x m Hessenberg-like matrix, the harmonic Ritz (or Ritz) eigenproblem, selection of k
// vectors, and the restart basis.  These matrices have at most 129 x 128 entries; the kernels
// keep them in global memory (resident in L2) and run every rotation and reflection with the 64
// lanes of one wavefront working on a row or column at a time.
#include <cfloat>

#include "kernels.h"

namespace dbq {

namespace {

constexpr int NT = 64;  // one wavefront

__device__ __forceinline__ double cabs_(zd a) { return hypot(a.re, a.im); }
__device__ __forceinline__ zd ld2(const double2* p, long long i) {
  const double2 v = p[i];
  return zd{v.x, v.y};
}
__device__ __forceinline__ void st2(double2* p, long long i, zd a) { p[i] = make_double2(a.re, a.im); }

// sum of v over the workgroup (single wavefront), result in every lane
__device__ __forceinline__ double wsum(double v) { return wave_sum(v); }

// ----------------------------------------------------------------------------- LU (column-major)
// In-place LU with partial pivoting of an n x n matrix; piv[j] = row swapped with j.
// Returns false (in every lane) if a pivot is exactly zero.
__device__ bool lu_factor(double2* A, int n, int ld, int* piv) {
  __shared__ int s_p;
  __shared__ int s_ok;
  const int t = threadIdx.x;
  if (t == 0) s_ok = 1;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (t == 0) {
      int p = j;
      double best = -1.0;
      for (int i = j; i < n; ++i) {
        const double a = cabs_(ld2(A, i + (long long)j * ld));
        if (a > best) {
          best = a;
          p = i;
        }
      }
      s_p = p;
      piv[j] = p;
      if (best == 0.0) s_ok = 0;
    }
    __syncthreads();
    const int p = s_p;
    if (p != j)
      for (int c = t; c < n; c += NT) {
        const zd a = ld2(A, j + (long long)c * ld), b = ld2(A, p + (long long)c * ld);
        st2(A, j + (long long)c * ld, b);
        st2(A, p + (long long)c * ld, a);
      }
    __syncthreads();
    const zd d = ld2(A, j + (long long)j * ld);
    if (d.re != 0.0 || d.im != 0.0) {
      for (int i = j + 1 + t; i < n; i += NT) st2(A, i + (long long)j * ld, cdiv(ld2(A, i + (long long)j * ld), d));
      __syncthreads();
      for (int idx = t; idx < (n - j - 1) * (n - j - 1); idx += NT) {
        const int i = j + 1 + idx % (n - j - 1), c = j + 1 + idx / (n - j - 1);
        st2(A, i + (long long)c * ld, ld2(A, i + (long long)c * ld) - ld2(A, i + (long long)j * ld) * ld2(A, j + (long long)c * ld));
      }
    }
    __syncthreads();
  }
  return s_ok != 0;
}

// Solve (LU) x = b for one right-hand side in a single lane (b overwritten).
__device__ void lu_solve_lane(const double2* A, int n, int ld, const int* piv, double2* b, long long ldb_stride) {
  for (int j = 0; j < n; ++j) {
    const int p = piv[j];
    if (p != j) {
      const zd a = ld2(b, j * ldb_stride), c = ld2(b, p * ldb_stride);
      st2(b, j * ldb_stride, c);
      st2(b, p * ldb_stride, a);
    }
  }
  for (int i = 0; i < n; ++i) {  // L y = b (unit diagonal)
    zd s = ld2(b, i * ldb_stride);
    for (int j = 0; j < i; ++j) s = s - ld2(A, i + (long long)j * ld) * ld2(b, j * ldb_stride);
    st2(b, i * ldb_stride, s);
  }
  for (int i = n - 1; i >= 0; --i) {  // U x = y
    zd s = ld2(b, i * ldb_stride);
    for (int j = i + 1; j < n; ++j) s = s - ld2(A, i + (long long)j * ld) * ld2(b, j * ldb_stride);
    st2(b, i * ldb_stride, cdiv(s, ld2(A, i + (long long)i * ld)));
  }
}

// ----------------------------------------------------------------------------- k x k solve
__global__ __launch_bounds__(NT) void k_lu_solve(const double2* __restrict__ M, int k,
                                                 double2* __restrict__ C, int nrhs,
                                                 double2* __restrict__ work, double* cond) {
  const int t = threadIdx.x;
  double2* LU = work;
  double2* inv = work + k * k;
  int* piv = (int*)(work + 2 * k * k);
  __shared__ double s_n1;
  for (int i = t; i < k * k; i += NT) LU[i] = M[i];
  __syncthreads();
  // 1-norm of M
  if (t == 0) {
    double best = 0;
    for (int j = 0; j < k; ++j) {
      double s = 0;
      for (int i = 0; i < k; ++i) s += cabs_(ld2(M, i + (long long)j * k));
      best = fmax(best, s);
    }
    s_n1 = best;
  }
  const bool ok = lu_factor(LU, k, k, piv);
  if (!ok) {
    if (t == 0) *cond = INFINITY;
    return;
  }
  // inverse, one column per lane
  for (int j = t; j < k; j += NT) {
    for (int i = 0; i < k; ++i) inv[i + (long long)j * k] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    lu_solve_lane(LU, k, k, piv, inv + (long long)j * k, 1);
  }
  __syncthreads();
  if (t == 0) {
    double best = 0;
    for (int j = 0; j < k; ++j) {
      double s = 0;
      for (int i = 0; i < k; ++i) s += cabs_(ld2(inv, i + (long long)j * k));
      best = fmax(best, s);
    }
    const double c = s_n1 * best;
    *cond = isfinite(c) ? c : INFINITY;
  }
  // Y = M^{-1} C, one column of C per lane (solve with the factors for accuracy)
  for (int j = t; j < nrhs; j += NT) lu_solve_lane(LU, k, k, piv, C + (long long)j * k, 1);
}

// ----------------------------------------------------------------------------- eigenproblem
// Householder reduction of G (n x n, ld n) to upper Hessenberg form; Q (n x n) accumulates the
// reflections so that G_in = Q G_out Q^H.
__device__ void hessenberg(double2* G, double2* Q, int n) {
  __shared__ double2 v[128];
  __shared__ double s_vn2;
  const int t = threadIdx.x;
  for (int i = t; i < n * n; i += NT) Q[i] = make_double2((i % n) == (i / n) ? 1.0 : 0.0, 0.0);
  __syncthreads();
  for (int j = 0; j + 2 < n; ++j) {
    const int len = n - j - 1;
    double p = 0;
    for (int i = t; i < len; i += NT) {
      const zd x = ld2(G, (j + 1 + i) + (long long)j * n);
      p += norm2(x);
      v[i] = make_double2(x.re, x.im);
    }
    const double nx2 = wsum(p);
    __syncthreads();
    if (nx2 == 0.0) continue;
    if (t == 0) {
      const zd x0{v[0].x, v[0].y};
      const double ax0 = cabs_(x0), nx = sqrt(nx2);
      const zd ph = ax0 > 0 ? zd{x0.re / ax0, x0.im / ax0} : zd{1.0, 0.0};
      const zd alpha{-ph.re * nx, -ph.im * nx};
      const zd v0 = x0 - alpha;
      v[0] = make_double2(v0.re, v0.im);
      s_vn2 = nx2 - ax0 * ax0 + norm2(v0);
    }
    __syncthreads();
    const double f = 2.0 / s_vn2;
    // left: rows j+1.., columns j..n-1
    for (int c = j + t; c < n; c += NT) {
      zd s{0, 0};
      for (int i = 0; i < len; ++i) s = s + cmulc(zd{v[i].x, v[i].y}, ld2(G, (j + 1 + i) + (long long)c * n));
      for (int i = 0; i < len; ++i) {
        const zd vi{v[i].x, v[i].y};
        st2(G, (j + 1 + i) + (long long)c * n, ld2(G, (j + 1 + i) + (long long)c * n) - f * (vi * s));
      }
    }
    __syncthreads();
    // right: all rows, columns j+1..
    for (int r = t; r < n; r += NT) {
      zd s{0, 0};
      for (int i = 0; i < len; ++i) s = s + ld2(G, r + (long long)(j + 1 + i) * n) * zd{v[i].x, v[i].y};
      for (int i = 0; i < len; ++i) {
        const zd vc = conj(zd{v[i].x, v[i].y});
        st2(G, r + (long long)(j + 1 + i) * n, ld2(G, r + (long long)(j + 1 + i) * n) - f * (s * vc));
      }
      zd q{0, 0};
      for (int i = 0; i < len; ++i) q = q + ld2(Q, r + (long long)(j + 1 + i) * n) * zd{v[i].x, v[i].y};
      for (int i = 0; i < len; ++i) {
        const zd vc = conj(zd{v[i].x, v[i].y});
        st2(Q, r + (long long)(j + 1 + i) * n, ld2(Q, r + (long long)(j + 1 + i) * n) - f * (q * vc));
      }
    }
    __syncthreads();
    for (int i = j + 2 + t; i < n; i += NT) G[i + (long long)j * n] = make_double2(0.0, 0.0);
    __syncthreads();
  }
}

__device__ __forceinline__ double nrm1(zd a) { return fabs(a.re) + fabs(a.im); }

// Shifted QR iteration (single Wilkinson shift, Givens bulge chase) on an upper Hessenberg G,
// reducing it to upper triangular Schur form T with G_in = Z T Z^H; Z must hold the
// Hessenberg reduction's Q on entry.  Returns false if it did not converge.
__device__ bool schur(double2* G, double2* Z, int n) {
  __shared__ int s_l, s_hi;
  __shared__ double s_c;
  __shared__ double2 s_s;
  __shared__ int s_done;
  const int t = threadIdx.x;
  const double eps = DBL_EPSILON;
  int iter = 0, total = 0;
  if (t == 0) {
    s_hi = n - 1;
    s_done = 0;
  }
  __syncthreads();
  while (true) {
    if (t == 0) {
      int hi = s_hi;
      int l = hi;
      while (l > 0) {
        const double s = nrm1(ld2(G, (l - 1) + (long long)(l - 1) * n)) + nrm1(ld2(G, l + (long long)l * n));
        const double sub = nrm1(ld2(G, l + (long long)(l - 1) * n));
        if (sub <= eps * (s > 0 ? s : 1e-300)) {
          G[l + (long long)(l - 1) * n] = make_double2(0.0, 0.0);
          break;
        }
        --l;
      }
      s_l = l;
    }
    __syncthreads();
    const int hi = s_hi, l = s_l;
    if (hi <= 0) break;
    if (l == hi) {
      if (t == 0) s_hi = hi - 1;
      iter = 0;
      __syncthreads();
      continue;
    }
    if (total > 60 * n) return false;
    // shift
    zd mu;
    {
      const zd a = ld2(G, (hi - 1) + (long long)(hi - 1) * n), b = ld2(G, (hi - 1) + (long long)hi * n);
      const zd c = ld2(G, hi + (long long)(hi - 1) * n), d = ld2(G, hi + (long long)hi * n);
      if (iter > 0 && iter % 11 == 0) {
        mu = d + zd{fabs(c.re) + fabs(c.im), 0.0};  // exceptional shift
      } else {
        const zd half{0.5 * (a.re - d.re), 0.5 * (a.im - d.im)};
        const zd disc2 = half * half + b * c;
        // principal square root
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
      if (t == 0) {
        zd x, y;
        if (kk == l) {
          x = ld2(G, l + (long long)l * n) - mu;
          y = ld2(G, (l + 1) + (long long)l * n);
        } else {
          x = ld2(G, kk + (long long)(kk - 1) * n);
          y = ld2(G, (kk + 1) + (long long)(kk - 1) * n);
        }
        // c = |x| / rho, s = (x / |x|) conj(y) / rho, rho = sqrt(|x|^2 + |y|^2): two square roots
        // and two reciprocals that do not depend on each other (the entries are far from the
        // range limits, so no hypot-style scaling is needed; this chain is the critical path of
        // every rotation)
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
          const double ax = sqrt(nx);
          const double irho = 1.0 / sqrt(nx + ny);
          const double iax = 1.0 / ax;
          c = ax * irho;
          const zd ph{x.re * iax, x.im * iax};
          s = ph * conj(y);
          s = zd{s.re * irho, s.im * irho};
        }
        s_c = c;
        s_s = make_double2(s.re, s.im);
      }
      __syncthreads();
      const double c = s_c;
      const zd s{s_s.x, s_s.y};
      // rows kk, kk+1 over columns max(kk-1, 0).. n-1
      for (int j = (kk > 0 ? kk - 1 : 0) + t; j < n; j += NT) {
        const zd a = ld2(G, kk + (long long)j * n), b = ld2(G, (kk + 1) + (long long)j * n);
        st2(G, kk + (long long)j * n, c * a + s * b);
        st2(G, (kk + 1) + (long long)j * n, c * b - conj(s) * a);
      }
      __syncthreads();
      // columns kk, kk+1 over rows 0 .. min(kk+2, hi); Z over all rows
      const int rmax = (kk + 2 < hi ? kk + 2 : hi);
      for (int i = t; i < n; i += NT) {
        if (i <= rmax) {
          const zd a = ld2(G, i + (long long)kk * n), b = ld2(G, i + (long long)(kk + 1) * n);
          st2(G, i + (long long)kk * n, c * a + conj(s) * b);
          st2(G, i + (long long)(kk + 1) * n, c * b - s * a);
        }
        const zd a = ld2(Z, i + (long long)kk * n), b = ld2(Z, i + (long long)(kk + 1) * n);
        st2(Z, i + (long long)kk * n, c * a + conj(s) * b);
        st2(Z, i + (long long)(kk + 1) * n, c * b - s * a);
      }
      __syncthreads();
      if (kk > l && t == 0) G[(kk + 1) + (long long)(kk - 1) * n] = make_double2(0.0, 0.0);
      __syncthreads();
    }
    ++iter;
    ++total;
  }
  return true;
}

// Eigenvector of upper-triangular T for diagonal position q, in Schur coordinates (y, length n,
// y_j = 0 for j > q), then g = Z y.  Runs in one lane.
__device__ void tri_eigvec(const double2* T, const double2* Z, int n, int q, double tnorm,
                           double2* y, double2* g) {
  const zd th = ld2(T, q + (long long)q * n);
  const double small = fmax(DBL_EPSILON * tnorm, 1e-300);
  for (int j = 0; j < n; ++j) y[j] = make_double2(j == q ? 1.0 : 0.0, 0.0);
  for (int i = q - 1; i >= 0; --i) {
    zd s{0, 0};
    for (int j = i + 1; j <= q; ++j) s = s + ld2(T, i + (long long)j * n) * ld2(y, j);
    zd d = ld2(T, i + (long long)i * n) - th;
    if (cabs_(d) < small) d = zd{small, 0.0};
    st2(y, i, -cdiv(s, d));
  }
  double nn = 0;
  for (int r = 0; r < n; ++r) {
    zd s{0, 0};
    for (int j = 0; j <= q; ++j) s = s + ld2(Z, r + (long long)j * n) * ld2(y, j);
    st2(g, r, s);
    nn += norm2(s);
  }
  nn = 1.0 / sqrt(nn);
  for (int r = 0; r < n; ++r) {
    const zd s = ld2(g, r);
    st2(g, r, zd{s.re * nn, s.im * nn});
  }
}

// orthonormalise column q of P (length len, ld ldp) against columns 0..q-1 (Gram-Schmidt twice);
// returns the norm before normalisation (all lanes)
__device__ double orth_column(double2* P, int ldp, int len, int q, double2* h) {
  const int t = threadIdx.x;
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = t; i < q; i += NT) {
      zd s{0, 0};
      for (int r = 0; r < len; ++r) s = s + cmulc(ld2(P, r + (long long)i * ldp), ld2(P, r + (long long)q * ldp));
      st2(h, i, s);
    }
    __syncthreads();
    for (int r = t; r < len; r += NT) {
      zd w = ld2(P, r + (long long)q * ldp);
      for (int i = 0; i < q; ++i) w = w - ld2(P, r + (long long)i * ldp) * ld2(h, i);
      st2(P, r + (long long)q * ldp, w);
    }
    __syncthreads();
  }
  double p = 0;
  for (int r = t; r < len; r += NT) p += norm2(ld2(P, r + (long long)q * ldp));
  const double nn = sqrt(wsum(p));
  const double f = nn > 0 ? 1.0 / nn : 0.0;
  for (int r = t; r < len; r += NT) {
    const zd w = ld2(P, r + (long long)q * ldp);
    st2(P, r + (long long)q * ldp, zd{w.re * f, w.im * f});
  }
  __syncthreads();
  return nn;
}

__global__ __launch_bounds__(NT) void k_cycle(CycleArgs a) {
  const int t = threadIdx.x;
  const int m = a.m, m1 = m + 1, k = a.k;
  double2* w = a.work;
  double2* QR = w;                 // (m+1) x m
  double2* gv = QR + m1 * m;       // m+1
  double2* rho = gv + m1;          // m+1
  double2* G = rho + m1;           // m x m
  double2* Z = G + m * m;          // m x m
  double2* Bm = Z + m * m;         // m x m
  double2* f = Bm + m * m;         // m
  double2* Y = f + m;              // m x m eigenvector scratch
  double2* Gv = Y + m * m;         // m x m selected eigenvectors
  double2* T1 = Gv + m * m;        // (m+1) x m
  double2* hh = T1 + m1 * m;       // m+1
  int* piv = (int*)(hh + m1);      // m ints
  __shared__ int order[128];
  __shared__ int s_kout;
  __shared__ int s_conv;
  const double2* H = a.Hbar;

  if (a.mode == 0 || a.mode == 1 || a.mode == 3) {
    // ---- least squares min || c - Hbar d || by Householder QR
    for (int i = t; i < m1 * m; i += NT) QR[i] = H[i];
    for (int i = t; i < m1; i += NT) gv[i] = a.c[i];
    __syncthreads();
    __shared__ double2 v[129];
    __shared__ double s_vn2;
    for (int j = 0; j < m; ++j) {
      const int len = m1 - j;
      double p = 0;
      for (int i = t; i < len; i += NT) {
        const zd x = ld2(QR, (j + i) + (long long)j * m1);
        p += norm2(x);
        v[i] = make_double2(x.re, x.im);
      }
      const double nx2 = wsum(p);
      __syncthreads();
      if (nx2 == 0.0) continue;
      if (t == 0) {
        const zd x0{v[0].x, v[0].y};
        const double ax0 = cabs_(x0), nx = sqrt(nx2);
        const zd ph = ax0 > 0 ? zd{x0.re / ax0, x0.im / ax0} : zd{1.0, 0.0};
        const zd alpha{-ph.re * nx, -ph.im * nx};
        const zd v0 = x0 - alpha;
        v[0] = make_double2(v0.re, v0.im);
        s_vn2 = nx2 - ax0 * ax0 + norm2(v0);
      }
      __syncthreads();
      const double fct = 2.0 / s_vn2;
      for (int c = j + t; c <= m; c += NT) {  // columns j..m-1 of QR, plus gv as column m
        double2* col = (c < m) ? QR + (long long)c * m1 : gv;
        zd s{0, 0};
        for (int i = 0; i < len; ++i) s = s + cmulc(zd{v[i].x, v[i].y}, ld2(col, j + i));
        for (int i = 0; i < len; ++i) st2(col, j + i, ld2(col, j + i) - fct * (zd{v[i].x, v[i].y} * s));
      }
      __syncthreads();
    }
    // back substitution R d = gv[0..m-1]
    if (t == 0) {
      for (int i = m - 1; i >= 0; --i) {
        zd s = ld2(gv, i);
        for (int j = i + 1; j < m; ++j) s = s - ld2(QR, i + (long long)j * m1) * ld2(a.d, j);
        const zd rii = ld2(QR, i + (long long)i * m1);
        st2(a.d, i, (rii.re != 0.0 || rii.im != 0.0) ? cdiv(s, rii) : zd{0.0, 0.0});
      }
    }
    __syncthreads();
    // rho = c - Hbar d with the original Hbar
    double p = 0;
    for (int r = t; r < m1; r += NT) {
      zd s = ld2(a.c, r);
      for (int j = 0; j < m; ++j) s = s - ld2(H, r + (long long)j * m1) * ld2(a.d, j);
      st2(rho, r, s);
      if (a.mode == 3) st2(a.cnew, r, s);
      p += norm2(s);
    }
    const double rn = sqrt(wsum(p));
    if (t == 0) {
      a.info[0] = rn;
      a.info[2] = (rn <= a.tol_abs) ? 1.0 : 0.0;
      s_conv = (rn <= a.tol_abs) ? 1 : 0;
    }
    __syncthreads();
    if ((a.mode == 0 && s_conv) || a.mode == 3) return;
  }

  // ---- eigenproblem matrix G (m x m)
  for (int i = t; i < m * m; i += NT) {
    const int r = i % m, c = i / m;
    G[i] = H[r + (long long)c * m1];
  }
  __syncthreads();
  if (a.mode != 2) {
    // harmonic Ritz: G = H_m + |h_{m+1,m}|^2 f e_m^T with H_m^H f = e_m
    for (int i = t; i < m * m; i += NT) {
      const int r = i % m, c = i / m;
      const zd hv = ld2(H, c + (long long)r * m1);
      st2(Bm, i, conj(hv));
    }
    __syncthreads();
    lu_factor(Bm, m, m, piv);
    __syncthreads();
    if (t == 0) {
      for (int i = 0; i < m; ++i) f[i] = make_double2(i == m - 1 ? 1.0 : 0.0, 0.0);
      lu_solve_lane(Bm, m, m, piv, f, 1);
    }
    __syncthreads();
    const double h2 = norm2(ld2(H, m + (long long)(m - 1) * m1));
    for (int r = t; r < m; r += NT) st2(G, r + (long long)(m - 1) * m, ld2(G, r + (long long)(m - 1) * m) + h2 * ld2(f, r));
    __syncthreads();
  }
  // The Hessenberg reduction and the QR iteration touch the whole matrix after every Givens
  // rotation: for m <= 64 they run on a copy in LDS (two 64 x 64 complex matrices, 128 KiB)
  // instead of through the caches.
  constexpr int LDS_M = 64;
  __shared__ double2 sGZ[2 * LDS_M * LDS_M];
  const bool in_lds = m <= LDS_M;
  double2* Gw = in_lds ? sGZ : G;
  double2* Zw = in_lds ? sGZ + m * m : Z;
  if (in_lds) {
    for (int i = t; i < m * m; i += NT) Gw[i] = G[i];
    __syncthreads();
  }
  hessenberg(Gw, Zw, m);
  __syncthreads();
  const bool ok = schur(Gw, Zw, m);
  __syncthreads();
  if (in_lds) {
    for (int i = t; i < m * m; i += NT) {
      G[i] = Gw[i];
      Z[i] = Zw[i];
    }
    __syncthreads();
  }
  if (t == 0) a.info[4] = ok ? 0.0 : 1.0;
  // ---- sort eigenvalues: |theta| ascending (harmonic) or Re descending (Ritz)
  for (int i = t; i < m; i += NT) {
    const zd ti = ld2(G, i + (long long)i * m);
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const zd tj = ld2(G, j + (long long)j * m);
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
  __syncthreads();
  for (int i = t; i < m; i += NT) a.theta[i] = G[order[i] + (long long)order[i] * m];
  if (t == 0) {
    int kout = k;
    if (a.mode == 1 && k < m) {
      const zd x = ld2(G, order[k - 1] + (long long)order[k - 1] * m);
      const zd y = ld2(G, order[k] + (long long)order[k] * m);
      const double sc = cabs_(x);
      if (fabs(x.im) > 1e-3 * sc && cabs_(x - conj(y)) <= 1e-3 * sc) kout = k - 1;
    }
    s_kout = kout;
    a.info[1] = kout;
  }
  __syncthreads();
  const int ks = s_kout;
  // ---- eigenvectors of the selected values
  double tn = 0;
  for (int i = t; i < m * m; i += NT) tn = fmax(tn, cabs_(ld2(G, i)));
  for (int o = 32; o > 0; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o, 64));
  for (int q = t; q < ks; q += NT) tri_eigvec(G, Z, m, order[q], tn, Y + (long long)q * m, Gv + (long long)q * m);
  __syncthreads();
  // ---- P: orthonormal basis of the selected vectors padded with a zero row, then the extra column
  for (int i = t; i < m1 * (k + 1); i += NT) a.P[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int i = t; i < m * ks; i += NT) {
    const int r = i % m, c = i / m;
    a.P[r + (long long)c * m1] = Gv[r + (long long)c * m];
  }
  __syncthreads();
  for (int q = 0; q < ks; ++q) orth_column(a.P, m1, m1, q, hh);
  if (a.mode == 2) {
    // Ritz residual of the first (rightmost) pair: |h_{m+1,m}| |e_m^T g|
    if (t == 0) {
      const double hm = cabs_(ld2(H, m + (long long)(m - 1) * m1));
      a.info[3] = hm * cabs_(ld2(a.P, (m - 1)));
      a.P[m + (long long)k * m1] = make_double2(1.0, 0.0);
    }
    __syncthreads();
  } else if (a.mode == 0) {
    for (int r = t; r < m1; r += NT) a.P[r + (long long)k * m1] = rho[r];
    __syncthreads();
    orth_column(a.P, m1, m1, k, hh);
  }
  if (a.mode == 1) return;
  // ---- Hnew = P^H Hbar P_k  ((k+1) x k), cnew = P^H rho
  for (int i = t; i < m1 * k; i += NT) {
    const int r = i % m1, c = i / m1;
    zd s{0, 0};
    for (int j = 0; j < m; ++j) s = s + ld2(H, r + (long long)j * m1) * ld2(a.P, j + (long long)c * m1);
    st2(T1, r + (long long)c * m1, s);
  }
  __syncthreads();
  for (int i = t; i < (k + 1) * k; i += NT) {
    const int r = i % (k + 1), c = i / (k + 1);
    zd s{0, 0};
    for (int j = 0; j < m1; ++j) s = s + cmulc(ld2(a.P, j + (long long)r * m1), ld2(T1, j + (long long)c * m1));
    st2(a.Hnew, r + (long long)c * m1, s);
  }
  for (int r = t; r < m1; r += NT) {
    zd s{0, 0};
    if (r <= k && a.mode == 0)
      for (int j = 0; j < m1; ++j) s = s + cmulc(ld2(a.P, j + (long long)r * m1), ld2(rho, j));
    st2(a.cnew, r, s);
  }
}

__global__ void k_trsolve(const double2* __restrict__ R, int ldr, int n, double2* __restrict__ z,
                          int nrhs, int ldz) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double2* b = z + (long long)j * ldz;
  for (int i = n - 1; i >= 0; --i) {
    zd s = ld2(b, i);
    for (int c = i + 1; c < n; ++c) s = s - ld2(R, i + (long long)c * ldr) * ld2(b, c);
    const zd d = ld2(R, i + (long long)i * ldr);
    st2(b, i, (d.re != 0.0 || d.im != 0.0) ? cdiv(s, d) : zd{0.0, 0.0});
  }
}

}  // namespace

size_t dense_cycle_work(int m) {
  const size_t m1 = m + 1;
  return m1 * m * 2 + 3 * m1 + 6 * size_t(m) * m + m + m1 + (size_t(m) + 3) / 4 + 8;
}

void dense_lu_solve(hipStream_t s, const double2* M, int k, double2* C, int nrhs, double2* work,
                    double* cond) {
  hipLaunchKernelGGL(k_lu_solve, dim3(1), dim3(NT), 0, s, M, k, C, nrhs, work, cond);
  DBQ_HIP(hipGetLastError());
}

void dense_cycle(hipStream_t s, const CycleArgs& a) {
  DBQ_CHECK(a.m >= 2 && a.m <= 128 && a.k >= 1 && a.k < a.m, "dense_cycle: bad (m, k)");
  hipLaunchKernelGGL(k_cycle, dim3(1), dim3(NT), 0, s, a);
  DBQ_HIP(hipGetLastError());
}

void dense_trsolve_upper(hipStream_t s, const double2* R, int ldr, int n, double2* z, int nrhs,
                         int ldz) {
  hipLaunchKernelGGL(k_trsolve, dim3((nrhs + 63) / 64), dim3(64), 0, s, R, ldr, n, z, nrhs, ldz);
  DBQ_HIP(hipGetLastError());
}

}  // namespace dbq
