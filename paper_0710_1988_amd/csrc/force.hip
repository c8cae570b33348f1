// Link gradient of L = sum_j Re(eta_j^H A^{-1} b_j) for the differentiable solve: with x = A^{-1} b
// and lambda = A^{-H} eta, dL = -Re(lambda^H dA x) and dA = -kappa dH.  Only two terms of H carry
// U_mu(y) (the forward hop out of y and the backward hop out of y+mu), which gives
//   G_mu(y) = kappa sum_spin [ lambda(y) ((1-gamma_mu) x(y+mu))^H + x(y) ((1+gamma_mu) lambda(y+mu))^H ].
// One thread per link, working directly on the caller's lexicographic complex128 layout.
#include "kernels.h"

namespace dbq {

namespace {

// (1 + S gamma_mu) psi in the chiral basis gamma_mu = [[0, B], [B^dagger, 0]]:
// upper = psi_up + S B psi_dn = h, lower = S B^dagger h
template <int MU>
__device__ __forceinline__ void proj_full(double S, const zd (&p)[12], zd (&o)[12]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const zd p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    zd h0, h1;
    if (MU == 0) {
      h0 = p0 - S * ti(p3);
      h1 = p1 - S * ti(p2);
      o[6 + c] = S * ti(h1);
      o[9 + c] = S * ti(h0);
    } else if (MU == 1) {
      h0 = p0 - S * p3;
      h1 = p1 + S * p2;
      o[6 + c] = S * h1;
      o[9 + c] = -(S * h0);
    } else if (MU == 2) {
      h0 = p0 - S * ti(p2);
      h1 = p1 + S * ti(p3);
      o[6 + c] = S * ti(h0);
      o[9 + c] = -(S * ti(h1));
    } else {
      h0 = p0 + S * p2;
      h1 = p1 + S * p3;
      o[6 + c] = S * h0;
      o[9 + c] = S * h1;
    }
    o[c] = h0;
    o[3 + c] = h1;
  }
}

__device__ __forceinline__ void load12(const double2* p, zd (&o)[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 v = p[k];
    o[k] = zd{v.x, v.y};
  }
}

template <int MU>
__device__ void force_site(const Geom& g, const double2* __restrict__ links, double kappa,
                           const double2* __restrict__ lam, const double2* __restrict__ x, int nrhs,
                           int kind, void* F, int y, int yf) {
  zd G[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) G[i] = zd{0.0, 0.0};
  for (int r = 0; r < nrhs; ++r) {
    const long long base = (long long)r * g.V * 12;
    zd ly[12], xf[12], xy[12], lf[12], a[12], z[12];
    load12(lam + base + (long long)y * 12, ly);
    load12(x + base + (long long)yf * 12, xf);
    load12(x + base + (long long)y * 12, xy);
    load12(lam + base + (long long)yf * 12, lf);
    proj_full<MU>(-1.0, xf, a);  // (1 - gamma_mu) x(y+mu)
    proj_full<MU>(+1.0, lf, z);  // (1 + gamma_mu) lambda(y+mu)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          G[3 * i + j] = G[3 * i + j] + ly[3 * s + i] * conj(a[3 * s + j]) + xy[3 * s + i] * conj(z[3 * s + j]);
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) G[i] = kappa * G[i];
  const long long li = (long long)MU * g.V + y;
  if (kind == 1) {
    double2* out = (double2*)F + li * 9;
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = make_double2(G[i].re, G[i].im);
    return;
  }
  // M = U G^H, F_c = Re(i tr[T_c M]) with T_c = Gell-Mann / 2
  zd U[9];
  const double2* up = links + li * 9;
#pragma unroll
  for (int i = 0; i < 9; ++i) U[i] = zd{up[i].x, up[i].y};
  zd M[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      zd s{0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) s = s + U[3 * i + k] * conj(G[3 * j + k]);
      M[3 * i + j] = s;
    }
  auto m = [&](int i, int j) { return M[3 * i + j]; };
  const zd I{0.0, 1.0};
  zd tr[8];
  tr[0] = m(1, 0) + m(0, 1);
  tr[1] = I * (m(0, 1) - m(1, 0));
  tr[2] = m(0, 0) - m(1, 1);
  tr[3] = m(2, 0) + m(0, 2);
  tr[4] = I * (m(0, 2) - m(2, 0));
  tr[5] = m(2, 1) + m(1, 2);
  tr[6] = I * (m(1, 2) - m(2, 1));
  const double r3 = 0.57735026918962576451;  // 1/sqrt(3)
  tr[7] = r3 * (m(0, 0) + m(1, 1) - 2.0 * m(2, 2));
  double* out = (double*)F + li * 8;
#pragma unroll
  for (int c = 0; c < 8; ++c) out[c] = 0.5 * (-tr[c].im);  // Re(i z / 2) = -Im(z) / 2
}

__global__ __launch_bounds__(128) void k_force(Geom g, const double2* __restrict__ links,
                                               double kappa, const double2* __restrict__ lam,
                                               const double2* __restrict__ x, int nrhs, int kind,
                                               void* F) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  if (y >= g.V) return;
  int c[4];
  int rem = y;
  c[0] = rem % g.L[0];
  rem /= g.L[0];
  c[1] = rem % g.L[1];
  rem /= g.L[1];
  c[2] = rem % g.L[2];
  c[3] = rem / g.L[2];
  c[mu] = (c[mu] + 1 == g.L[mu]) ? 0 : c[mu] + 1;
  const int yf = lex_index(g, c);
  switch (mu) {
    case 0: force_site<0>(g, links, kappa, lam, x, nrhs, kind, F, y, yf); break;
    case 1: force_site<1>(g, links, kappa, lam, x, nrhs, kind, F, y, yf); break;
    case 2: force_site<2>(g, links, kappa, lam, x, nrhs, kind, F, y, yf); break;
    default: force_site<3>(g, links, kappa, lam, x, nrhs, kind, F, y, yf); break;
  }
}

}  // namespace

void launch_link_force(hipStream_t s, const Geom& g, const void* links, double kappa,
                       const void* lambda, const void* x, int nrhs, int kind, void* F) {
  hipLaunchKernelGGL(k_force, dim3((g.V + 127) / 128, 4), dim3(128), 0, s, g,
                     (const double2*)links, kappa, (const double2*)lambda, (const double2*)x, nrhs,
                     kind, F);
  DBQ_HIP(hipGetLastError());
}

}  // namespace dbq
