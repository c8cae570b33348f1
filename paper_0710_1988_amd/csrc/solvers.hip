// Host drivers of the solvers: D-BiCGStab(k) (Sec. 2), GMRES-DR(m,k) for the first right-hand side
// (Sec. 1 and Sec. 3), kappa_c (Sec. 3), the minimal-residual projection over previous shifts'
// solutions (Sec. 4), and the operator apply.  Every arithmetic step runs in the kernels; the
// host decides control flow from a few scalars read back at check points.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "ctx.h"
#include "kernels.h"
#include "solvers.h"

namespace dbq {

namespace {


struct Op {
  Geom g;
  double kappa = 0, mu = 0;
  bool schur = false;  // the even-odd reduced operator on the even sites
  double2* l64 = nullptr;
  float4* l32 = nullptr;
  // sites and complex elements of the vectors the solvers iterate on
  long long sites() const { return schur ? g.V / 2 : g.V; }
  long long n() const { return 12LL * sites(); }
  long long nfull() const { return 12LL * g.V; }
};

void check_op(const dbq_operator* o) {
  DBQ_CHECK(o != nullptr, "null operator");
  long long V = 1;
  for (int i = 0; i < 4; ++i) {
    DBQ_CHECK(o->L[i] >= 2 && o->L[i] % 2 == 0, "lattice extents must be even and >= 2");
    V *= o->L[i];
  }
  // byte offsets within one component array are 32-bit in the kernels
  DBQ_CHECK(V <= (1ll << 26), "lattice too large (V > 2^26)");
  DBQ_CHECK(o->links != nullptr, "null links");
  DBQ_CHECK(std::isfinite(o->kappa) && std::isfinite(o->mu), "non-finite kappa or mu");
  DBQ_CHECK(o->schur == 0 || o->schur == 1, "schur must be 0 or 1");
  DBQ_CHECK(o->pad == 0, "operator pad field must be 0");
}

Op make_op(dbq_ctx* c, WsScope& ws, const dbq_operator* o, bool f64, bool f32) {
  Op op;
  op.g = make_geom(o->L);
  op.kappa = o->kappa;
  op.mu = o->mu;
  op.schur = o->schur != 0;
  if (f64) {
    op.l64 = ws.get<double2>(36LL * op.g.V);
    pack_links_f64(c->stream, op.g, o->links, op.l64);
  }
  if (f32) {
    op.l32 = ws.get<float4>(12LL * op.g.V);
    pack_links_f32(c->stream, op.g, o->links, op.l32);
  }
  return op;
}

struct DsSpec {
  const Op* op;
  bool f32;
  const void* in;
  void* out;
  const void* aux;
  int nrhs;
  int rhs_base;
};

DsBatch make_batch(const std::vector<DsSpec>& v) {
  DBQ_CHECK(!v.empty() && v.size() <= size_t(MAXLAT), "batch: 1..8 lattices");
  DsBatch b;
  std::memset(&b, 0, sizeof(b));
  b.nlat = int(v.size());
  int nr = 0, ps = 1;
  for (size_t i = 0; i < v.size(); ++i) {
    DsLat& L = b.lat[i];
    L.g = v[i].op->g;
    L.links = v[i].f32 ? (const void*)v[i].op->l32 : (const void*)v[i].op->l64;
    L.in = v[i].in;
    L.out = v[i].out;
    L.aux = v[i].aux;
    L.cen = nullptr;
    L.nrhs = v[i].nrhs;
    L.rhs_base = v[i].rhs_base;
    // site blocks (set again by the launcher for the launch shape it uses)
    L.nsb = 2 * ((L.g.V / 2 + DS_BS - 1) / DS_BS);
    L.blk_begin = 0;  // laid out by the launcher
    L.kappa = v[i].op->kappa;
    L.mu = v[i].op->mu;
    nr = std::max(nr, L.rhs_base + L.nrhs);
    ps = std::max(ps, ds_partial_slots(L.g));
    DBQ_CHECK(v[i].op->schur == v[0].op->schur, "batch: mixed full and reduced operators");
  }
  b.schur = v[0].op->schur ? 1 : 0;
  b.nblocks = 0;
  b.nb = 1;
  b.nrhs_total = nr;
  b.pstride = ps;
  return b;
}

// Launch shape of the Dslash: nb = right-hand sides per thread of the site kernel (1, 2, 4), or in
// FP32 0 for the LDS-staged tile kernel; rg = for the site kernel how many of those thread groups
// sweep the site blocks together (1, 2, 4 or 0 = all), for the tile kernel the rhs per block
// (1, 2, 3, 4, 6 or 0 = all); order = the tile kernel's block-to-tile order (tile_of_block).
struct Shape {
  int nb = 1, rg = 0, order = 0;
};

// Forced shape from DBQ_DS_NB / DBQ_DS_RG / DBQ_TILE_ORDER, if any of them is set.
bool forced_shape(bool f32, bool half, Shape& sh) {
  const char* e_nb = std::getenv("DBQ_DS_NB");
  const char* e_rg = std::getenv("DBQ_DS_RG");
  const char* e_to = std::getenv("DBQ_TILE_ORDER");
  if (!e_nb && !e_rg && !e_to) return false;
  int nb = e_nb ? std::atoi(e_nb) : (f32 ? 0 : 1);
  if (half ? (nb != 0 && nb != 2) : (nb != 0 && nb != 1 && nb != 2 && nb != 4)) nb = 1;
  if (nb == 0 && !f32) nb = 1;
  sh.nb = nb;
  sh.rg = e_rg ? std::max(0, std::atoi(e_rg)) : 0;
  sh.order = e_to ? std::min(3, std::max(0, std::atoi(e_to))) : 0;
  return true;
}

// The timed candidates are every (nb, rg) above and, for the tile kernel, each tile order.  Timed
// once per (precision, volume, batch size) in this context on a scratch output (the operator
// input is only read).
Shape choose_shape(dbq_ctx* c, bool f32, const DsBatch& b) {
  int maxr = 1;
  for (int i = 0; i < b.nlat; ++i) maxr = std::max(maxr, b.lat[i].nrhs);
  Shape forced;
  if (forced_shape(f32, false, forced)) return forced;
  std::vector<Shape> cand;
  for (int nb : {1, 2, 4}) {
    if (nb > maxr || (!f32 && nb == 4)) continue;
    const int ng = (maxr + nb - 1) / nb;
    for (int rg : {1, 2, 4, 0})
      if (rg < ng) cand.push_back(Shape{nb, rg, 0});  // 0 (all) covers rg >= ng
  }
  if (f32) {
    for (int g : {1, 2, 3, 4, 6, 0})
      if (g < maxr)
        for (int o : {0, 1, 2, 3})
          if (o != 2 || (g != 0 && g < maxr)) cand.push_back(Shape{0, g, o});
  }
  if (cand.size() == 1) return cand[0];
  int big = 0;
  for (int i = 1; i < b.nlat; ++i)
    if ((long long)b.lat[i].g.V * b.lat[i].nrhs > (long long)b.lat[big].g.V * b.lat[big].nrhs) big = i;
  const auto key = std::make_tuple(f32 ? 1 : 0, b.lat[big].g.V, b.lat[big].nrhs);
  auto it = c->ds_tune.find(key);
  if (it != c->ds_tune.end())
    return Shape{std::get<0>(it->second), std::get<1>(it->second), std::get<2>(it->second)};
  WsScope ws(c);
  DsBatch t;
  std::memset(&t, 0, sizeof(t));
  t.nlat = 1;
  t.lat[0] = b.lat[big];
  t.lat[0].rhs_base = 0;
  t.lat[0].aux = nullptr;
  t.nrhs_total = t.lat[0].nrhs;
  t.pstride = ds_partial_slots(t.lat[0].g);
  const size_t bytes =
      size_t(t.lat[0].nrhs) * t.lat[0].g.V * (f32 ? 6 * sizeof(float4) : 12 * sizeof(double2));
  t.lat[0].out = ws.take(bytes);
  hipEvent_t e0, e1;
  DBQ_HIP(hipEventCreate(&e0));
  DBQ_HIP(hipEventCreate(&e1));
  Shape best = cand[0];
  float best_ms = 1e30f;
  for (const auto& sh : cand) {
    t.torder = sh.order;
    for (int rep = 0; rep < 2; ++rep) {  // warm-up, then timed
      DBQ_HIP(hipEventRecord(e0, c->stream));
      for (int k = 0; k < 3; ++k) {
        if (f32) launch_dslash_f32(c->stream, t, 0, EPI_NONE, nullptr, nullptr, sh.nb, sh.rg);
        else launch_dslash_f64(c->stream, t, 0, EPI_NONE, nullptr, nullptr, sh.nb, sh.rg);
      }
      DBQ_HIP(hipEventRecord(e1, c->stream));
    }
    DBQ_HIP(hipEventSynchronize(e1));
    float ms = 0;
    DBQ_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (std::getenv("DBQ_DEBUG"))
      std::fprintf(stderr, "[dbq] tune %s V=%d nrhs=%d nb=%d rg=%d order=%d: %.1f us\n",
                   f32 ? "fp32" : "fp64", t.lat[0].g.V, maxr, sh.nb, sh.rg, sh.order,
                   ms * 1e3f / 3);
    if (ms < best_ms) {
      best_ms = ms;
      best = sh;
    }
  }
  DBQ_HIP(hipEventDestroy(e0));
  DBQ_HIP(hipEventDestroy(e1));
  c->ds_tune[key] = std::make_tuple(best.nb, best.rg, best.order);
  return best;
}

// Launch shape of the half-lattice kernels for a batch of the reduced operator: nb = 1 or 2 rhs
// per thread with rg as for the site kernel, or in FP32 nb = 0 for the LDS-staged tile kernel
// with rg rhs per block and a tile order; timed once per (precision, volume, batch size) on step
// 1 into a scratch output.  DBQ_DS_NB / DBQ_DS_RG / DBQ_TILE_ORDER force the values.
Shape choose_shape_half(dbq_ctx* c, bool f32, const DsBatch& b) {
  int maxr = 1;
  for (int i = 0; i < b.nlat; ++i) maxr = std::max(maxr, b.lat[i].nrhs);
  Shape forced;
  if (forced_shape(f32, true, forced)) return forced;
  std::vector<Shape> cand;
  for (int nb : {1, 2}) {
    if (nb > maxr) continue;
    const int ng = (maxr + nb - 1) / nb;
    for (int rg : {1, 2, 4, 0})
      if (rg < ng) cand.push_back(Shape{nb, rg, 0});
  }
  if (f32) {
    for (int g : {1, 2, 3, 4, 6, 0})
      if (g < maxr)
        for (int o : {0, 1, 2, 3})
          if (o != 2 || (g != 0 && g < maxr)) cand.push_back(Shape{0, g, o});
  }
  if (cand.size() == 1) return cand[0];
  int big = 0;
  for (int i = 1; i < b.nlat; ++i)
    if ((long long)b.lat[i].g.V * b.lat[i].nrhs > (long long)b.lat[big].g.V * b.lat[big].nrhs) big = i;
  const auto key = std::make_tuple(f32 ? 3 : 2, b.lat[big].g.V, b.lat[big].nrhs);
  auto it = c->ds_tune.find(key);
  if (it != c->ds_tune.end())
    return Shape{std::get<0>(it->second), std::get<1>(it->second), std::get<2>(it->second)};
  WsScope ws(c);
  DsBatch t;
  std::memset(&t, 0, sizeof(t));
  t.nlat = 1;
  t.schur = 1;
  t.lat[0] = b.lat[big];
  t.lat[0].rhs_base = 0;
  t.lat[0].aux = nullptr;
  t.lat[0].cen = nullptr;
  t.lat[0].kappa = 1.0;
  t.nrhs_total = t.lat[0].nrhs;
  t.pstride = ds_partial_slots(t.lat[0].g);
  const size_t bytes = size_t(t.lat[0].nrhs) * (t.lat[0].g.V / 2) *
                       (f32 ? 6 * sizeof(float4) : 12 * sizeof(double2));
  t.lat[0].out = ws.take(bytes);
  hipEvent_t e0, e1;
  DBQ_HIP(hipEventCreate(&e0));
  DBQ_HIP(hipEventCreate(&e1));
  Shape best = cand[0];
  float best_ms = 1e30f;
  for (const auto& sh : cand) {
    t.torder = sh.order;
    for (int rep = 0; rep < 2; ++rep) {  // warm-up, then timed
      DBQ_HIP(hipEventRecord(e0, c->stream));
      for (int k = 0; k < 3; ++k) {
        if (f32) launch_dslash_half_f32(c->stream, t, 1, 0, EPI_NONE, nullptr, nullptr, sh.nb, sh.rg, 0);
        else launch_dslash_half_f64(c->stream, t, 1, 0, EPI_NONE, nullptr, nullptr, sh.nb, sh.rg, 0);
      }
      DBQ_HIP(hipEventRecord(e1, c->stream));
    }
    DBQ_HIP(hipEventSynchronize(e1));
    float ms = 0;
    DBQ_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (std::getenv("DBQ_DEBUG"))
      std::fprintf(stderr, "[dbq] tune half %s V=%d nrhs=%d nb=%d rg=%d order=%d: %.1f us\n",
                   f32 ? "fp32" : "fp64", t.lat[0].g.V, maxr, sh.nb, sh.rg, sh.order,
                   ms * 1e3f / 3);
    if (ms < best_ms) {
      best_ms = ms;
      best = sh;
    }
  }
  DBQ_HIP(hipEventDestroy(e0));
  DBQ_HIP(hipEventDestroy(e1));
  c->ds_tune[key] = std::make_tuple(best.nb, best.rg, best.order);
  return best;
}

// The reduced operator Ahat = D - kappa^2 H_eo D^{-1} H_oe on a batch of half vectors: step 1
// into a scratch odd-site vector, step 2 (with the batch's epilogue) into the output.  Gated
// launches skip the same rhs in both steps.
void run_schur(dbq_ctx* c, bool f32, const DsBatch& b0, int dagger, int epi, RhsScal* sc,
               double* partials) {
  WsScope ws(c);
  const int gate = sc ? (epi == EPI_RESID ? 2 : 1) : 0;
  DsBatch b1 = b0;
  b1.acct = DsAcct{};
  size_t need = 0;
  for (int i = 0; i < b1.nlat; ++i)
    need += size_t(b1.lat[i].nrhs) * (b1.lat[i].g.V / 2) *
            (f32 ? 6 * sizeof(float4) : 12 * sizeof(double2));
  char* tmp = (c->schur_tmp && c->schur_tmp_bytes >= need) ? (char*)c->schur_tmp
                                                            : (char*)ws.take(need);
  for (int i = 0; i < b1.nlat; ++i) {
    DsLat& L = b1.lat[i];
    L.out = tmp;
    tmp += size_t(L.nrhs) * (L.g.V / 2) * (f32 ? 6 * sizeof(float4) : 12 * sizeof(double2));
    L.cen = nullptr;
    L.aux = nullptr;
    L.kappa = 1.0;
  }
  const Shape shape = choose_shape_half(c, f32, b1);
  b1.torder = shape.order;
  DsBatch b2 = b0;
  b2.acct = DsAcct{};
  for (int i = 0; i < b2.nlat; ++i) {
    DsLat& L = b2.lat[i];
    L.in = b1.lat[i].out;
    L.cen = b0.lat[i].in;
    L.kappa = b0.lat[i].kappa * b0.lat[i].kappa;
  }
  b2.torder = shape.order;
  if (f32) {
    launch_dslash_half_f32(c->stream, b1, 1, dagger, EPI_NONE, sc, partials, shape.nb, shape.rg, gate);
    launch_dslash_half_f32(c->stream, b2, 2, dagger, epi, sc, partials, shape.nb, shape.rg, gate);
  } else {
    launch_dslash_half_f64(c->stream, b1, 1, dagger, EPI_NONE, sc, partials, shape.nb, shape.rg, gate);
    launch_dslash_half_f64(c->stream, b2, 2, dagger, epi, sc, partials, shape.nb, shape.rg, gate);
  }
  launch_ds_finalize(c->stream, b2, epi, sc, partials);
}

void run_dslash(dbq_ctx* c, bool f32, const DsBatch& b0, int dagger, int epi, RhsScal* sc,
                double* partials) {
  if (b0.schur) {
    run_schur(c, f32, b0, dagger, epi, sc, partials);
    return;
  }
  const Shape shape = choose_shape(c, f32, b0);
  const int kind = f32 ? 1 : 0;
  DsBatch b = b0;
  b.acct = DsAcct{};
  b.torder = shape.order;
  hipEvent_t e0;
  timer_begin(c, kind, &e0);  // null unless this launch is a timed sample
  // a gated launch (scalars given) skips inactive rhs: the bytes of a timed one are counted on
  // the device
  const bool dev_acct = e0 != nullptr && sc != nullptr && epi != EPI_NONE;
  if (dev_acct) {
    b.acct.bytes = c->acct + kind;
    b.acct.tags = c->acct + 8 + 8 * kind;
    b.acct.spinor_passes = ds_spinor_passes(epi);
    b.acct.spinor_bytes = f32 ? 24 * 4 : 12 * 16;
    b.acct.link_bytes = f32 ? 4 * 12 * 4 : 4 * 9 * 16;
  }
  // residual launches select few rhs: with all rhs groups of a site block adjacent, the selected
  // ones still cover every XCD (chunks of rhs groups would put one rhs on one or two XCDs)
  const int rg = (epi == EPI_RESID && shape.nb > 0) ? 0 : shape.rg;
  const double bytes =
      f32 ? launch_dslash_f32(c->stream, b, dagger, epi, sc, partials, shape.nb, rg)
          : launch_dslash_f64(c->stream, b, dagger, epi, sc, partials, shape.nb, rg);
  timer_end(c, kind, e0, dev_acct ? 0.0 : bytes);
  launch_ds_finalize(c->stream, b, epi, sc, partials);
}

// ---- even-odd reduced system: half vectors and the full system's right-hand side and solution.
// Internal vectors are [rhs][6][sites] of esize-byte elements (32 in FP64, 16 in FP32); the even
// sites are the first V/2 of each component array and the odd sites the rest, so a half vector
// is a strided copy.
void split_parity(hipStream_t s, const Geom& g, const void* full, void* even, void* odd, int nrhs,
                  size_t esize) {
  const size_t row = size_t(g.V / 2) * esize, pitch = size_t(g.V) * esize;
  const size_t rows = size_t(6) * nrhs;
  if (even)
    DBQ_HIP(hipMemcpy2DAsync(even, row, full, pitch, row, rows, hipMemcpyDeviceToDevice, s));
  if (odd)
    DBQ_HIP(hipMemcpy2DAsync(odd, row, (const char*)full + row, pitch, row, rows,
                             hipMemcpyDeviceToDevice, s));
}
// full vector from its halves; odd = null gives zero odd sites
void merge_parity(hipStream_t s, const Geom& g, const void* even, const void* odd, void* full,
                  int nrhs, size_t esize) {
  const size_t row = size_t(g.V / 2) * esize, pitch = size_t(g.V) * esize;
  const size_t rows = size_t(6) * nrhs;
  DBQ_HIP(hipMemcpy2DAsync(full, pitch, even, row, row, rows, hipMemcpyDeviceToDevice, s));
  if (odd)
    DBQ_HIP(hipMemcpy2DAsync((char*)full + row, pitch, odd, row, row, rows,
                             hipMemcpyDeviceToDevice, s));
  else
    DBQ_HIP(hipMemset2DAsync((char*)full + row, pitch, 0, row, rows, s));
}

// one FP64 half-lattice launch on nrhs vectors of one operator (coefficient c, twisted mass t)
void half_step(dbq_ctx* c, const Op& op, int step, const double2* in, const double2* cen,
               double2* out, double coef, double t, int nrhs, int dagger) {
  DsBatch b = make_batch({DsSpec{&op, false, in, out, nullptr, nrhs, 0}});
  b.lat[0].cen = cen;
  b.lat[0].kappa = coef;
  b.lat[0].mu = t;
  launch_dslash_half_f64(c->stream, b, step, dagger, EPI_NONE, nullptr, nullptr, 1, 0, 0);
}

// canonical vectors -> even half of the packed FP64 vectors (x0, deflation vectors)
void pack_even_f64(dbq_ctx* c, WsScope& ws, const Op& op, const void* canon, double2* half,
                   int nrhs) {
  double2* f = ws.get<double2>(size_t(op.nfull()) * nrhs);
  pack_spinor_f64(c->stream, op.g, canon, f, nrhs);
  split_parity(c->stream, op.g, f, half, nullptr, nrhs, 32);
}
// even-site half vectors -> canonical full vectors with zero odd sites
void unpack_even_f64(dbq_ctx* c, WsScope& ws, const Op& op, const double2* half, void* canon,
                     int nrhs) {
  double2* f = ws.get<double2>(size_t(op.nfull()) * nrhs);
  merge_parity(c->stream, op.g, half, nullptr, f, nrhs, 32);
  unpack_spinor_f64(c->stream, op.g, f, canon, nrhs);
}
// bhat = b_e + kappa H_eo D^{-1} b_o (dagger: H^dagger and D(-mu)) from a packed full b; b_o is
// left in bodd for the odd half of the solution
void schur_rhs(dbq_ctx* c, WsScope& ws, const Op& op, const double2* bfull, double2* bhat,
               double2* bodd, int nrhs, int dagger) {
  const size_t nh = size_t(op.n()) * nrhs;
  double2* be = ws.get<double2>(nh);
  double2* u = ws.get<double2>(nh);
  split_parity(c->stream, op.g, bfull, be, bodd, nrhs, 32);
  half_step(c, op, 1, be, bodd, u, 0.0, op.mu, nrhs, dagger);       // u = D^{-1} b_o
  half_step(c, op, 2, u, be, bhat, -op.kappa, 0.0, nrhs, dagger);   // b_e + kappa H_eo u
}
// canonical full solution from x_e: x_o = D^{-1} (b_o + kappa H_oe x_e)
void schur_solution(dbq_ctx* c, WsScope& ws, const Op& op, const double2* xe, const double2* bodd,
                    void* canon, int nrhs, int dagger) {
  double2* xo = ws.get<double2>(size_t(op.n()) * nrhs);
  double2* f = ws.get<double2>(size_t(op.nfull()) * nrhs);
  half_step(c, op, 1, xe, bodd, xo, op.kappa, op.mu, nrhs, dagger);
  merge_parity(c->stream, op.g, xe, xo, f, nrhs, 32);
  unpack_spinor_f64(c->stream, op.g, f, canon, nrhs);
}

template <typename T>
T* upload(dbq_ctx* c, WsScope& ws, const std::vector<T>& h) {
  T* d = ws.get<T>(std::max<size_t>(h.size(), 1));
  if (!h.empty()) {
    DBQ_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    DBQ_HIP(hipStreamSynchronize(c->stream));
  }
  return d;
}

VecSet make_vecset(dbq_ctx* c, WsScope& ws, const std::vector<int>& nelem) {
  std::vector<long long> off(nelem.size());
  std::vector<int> nch(nelem.size());
  long long o = 0;
  int ps = 1;
  for (size_t j = 0; j < nelem.size(); ++j) {
    off[j] = o;
    o += nelem[j];
    nch[j] = (nelem[j] + BL_CHUNK - 1) / BL_CHUNK;
    ps = std::max(ps, nch[j]);
  }
  // chunk-major block order: the right-hand sides alternate, so that a launch in which only a
  // few of them are selected still spreads their chunks over every XCD
  std::vector<int2> blk;
  for (int ch = 0; ch < ps; ++ch)
    for (size_t j = 0; j < nelem.size(); ++j)
      if (ch < nch[j]) blk.push_back(make_int2(int(j), ch));
  DBQ_CHECK(blk.size() < (size_t(1) << 31), "vector set too large");
  VecSet vs;
  vs.off = upload(c, ws, off);
  vs.nelem = upload(c, ws, nelem);
  vs.blk = upload(c, ws, blk);
  vs.nblocks = int(blk.size());
  vs.nrhs = int(nelem.size());
  vs.pstride = ps;
  return vs;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t norm_work(long long n, int count) { return size_t((n + 2047) / 2048) * size_t(count) + 64; }

}  // namespace

// ============================================================================ operator apply
void apply_operator(dbq_ctx* c, const dbq_operator* o, const void* in, void* out, int nrhs,
                    int dagger, int prec) {
  check_op(o);
  DBQ_CHECK(in && out, "null vector");
  DBQ_CHECK(in != out, "in and out must not alias");
  DBQ_CHECK(nrhs >= 1, "nrhs must be >= 1");
  DBQ_CHECK(prec == DBQ_FP64 || prec == DBQ_MIXED, "bad precision");
  WsScope ws(c);
  const bool f32 = prec == DBQ_MIXED;
  Op op = make_op(c, ws, o, !f32, f32);
  const long long V = op.g.V;
  if (op.schur) {
    // out_e = Ahat in_e, out_o = 0
    if (!f32) {
      double2* a = ws.get<double2>(size_t(op.n()) * nrhs);
      double2* b = ws.get<double2>(size_t(op.n()) * nrhs);
      pack_even_f64(c, ws, op, in, a, nrhs);
      DsBatch bt = make_batch({DsSpec{&op, false, a, b, nullptr, nrhs, 0}});
      run_dslash(c, false, bt, dagger, EPI_NONE, nullptr, nullptr);
      unpack_even_f64(c, ws, op, b, out, nrhs);
    } else {
      float4* f = ws.get<float4>(6LL * V * nrhs);
      float4* a = ws.get<float4>(3LL * V * nrhs);
      float4* b = ws.get<float4>(3LL * V * nrhs);
      pack_spinor_f32(c->stream, op.g, in, f, nrhs);
      split_parity(c->stream, op.g, f, a, nullptr, nrhs, 16);
      DsBatch bt = make_batch({DsSpec{&op, true, a, b, nullptr, nrhs, 0}});
      run_dslash(c, true, bt, dagger, EPI_NONE, nullptr, nullptr);
      merge_parity(c->stream, op.g, b, nullptr, f, nrhs, 16);
      unpack_spinor_f32(c->stream, op.g, f, out, nrhs);
    }
    return;
  }
  if (!f32) {
    double2* a = ws.get<double2>(12LL * V * nrhs);
    double2* b = ws.get<double2>(12LL * V * nrhs);
    pack_spinor_f64(c->stream, op.g, in, a, nrhs);
    DsBatch bt = make_batch({DsSpec{&op, false, a, b, nullptr, nrhs, 0}});
    run_dslash(c, false, bt, dagger, EPI_NONE, nullptr, nullptr);
    unpack_spinor_f64(c->stream, op.g, b, out, nrhs);
  } else {
    float4* a = ws.get<float4>(6LL * V * nrhs);
    float4* b = ws.get<float4>(6LL * V * nrhs);
    pack_spinor_f32(c->stream, op.g, in, a, nrhs);
    DsBatch bt = make_batch({DsSpec{&op, true, a, b, nullptr, nrhs, 0}});
    run_dslash(c, true, bt, dagger, EPI_NONE, nullptr, nullptr);
    unpack_spinor_f32(c->stream, op.g, b, out, nrhs);
  }
}

// ============================================================================ D-BiCGStab(k)
namespace {

// HIP graphs of the mixed-precision iteration blocks of one solve, keyed by block length.
// DBQ_GRAPH=0 runs every block eagerly, and so does a solve with kernel timing on.  A capture that fails (an operation the runtime cannot
// capture) ends the capture and the solve continues eagerly.
struct LoopGraphs {
  struct G {
    int key = 0;
    hipGraphExec_t exec = nullptr;
    std::vector<dbq_ctx::GraphTimer> timers;
  };
  dbq_ctx* c;
  std::vector<std::unique_ptr<G>> gs;
  bool enabled, warm = false;
  LoopGraphs(dbq_ctx* ctx, size_t schur_bytes, WsScope& ws) : c(ctx) {
    const char* e = std::getenv("DBQ_GRAPH");
    // timed launches run eagerly: an event recorded by a graph node cannot be read back as a
    // timestamp pair on this runtime
    enabled = !(e && std::atoi(e) == 0) && !c->timing;
    if (enabled && schur_bytes) {
      c->schur_tmp = ws.take(schur_bytes);
      c->schur_tmp_bytes = schur_bytes;
    }
  }
  LoopGraphs(const LoopGraphs&) = delete;
  LoopGraphs& operator=(const LoopGraphs&) = delete;
  ~LoopGraphs() {
    for (auto& g : gs) {
      if (g->exec) (void)hipGraphExecDestroy(g->exec);
      graph_timers_release(c, g->timers);
    }
    c->schur_tmp = nullptr;
    c->schur_tmp_bytes = 0;
  }
  // run a block of n iterations; returns the graph replayed, or null when it ran eagerly.  key
  // names the block's launch sequence (its length and whatever else the caller varies)
  template <typename F>
  const G* run(int key, int n, F&& block) {
    if (!enabled || !warm) {
      block(n);
      warm = true;
      return nullptr;
    }
    G* g = nullptr;
    for (auto& q : gs)
      if (q->key == key) g = q.get();
    if (!g) {
      g = capture(key, n, block);
      if (!g) {
        enabled = false;
        block(n);
        return nullptr;
      }
    }
    DBQ_HIP(hipGraphLaunch(g->exec, c->stream));
    return g;
  }
  template <typename F>
  G* capture(int key, int n, F&& block) {
    if (!c->cap_stream) DBQ_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    std::unique_ptr<G> g(new G());
    g->key = key;
    const hipStream_t orig = c->stream;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    c->stream = c->cap_stream;
    c->cap_timers = &g->timers;
    bool ok = true;
    try {
      block(n);
    } catch (const Error&) {
      ok = false;
    }
    c->stream = orig;
    c->cap_timers = nullptr;
    if (hipStreamEndCapture(c->cap_stream, &graph) != hipSuccess || !ok || !graph) {
      (void)hipGetLastError();
      if (graph) (void)hipGraphDestroy(graph);
      graph_timers_release(c, g->timers);
      return nullptr;
    }
    const hipError_t e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      graph_timers_release(c, g->timers);
      return nullptr;
    }
    gs.push_back(std::move(g));
    return gs.back().get();
  }
};

}  // namespace

int dbicgstab(dbq_ctx* c, const dbq_operator* ops, int nops, const void* const* Vin,
              const int32_t* kk, const void* const* B, void* const* X, const int32_t* nrhs,
              double tol, int64_t max_mv, int prec, int dagger, dbq_stats* st) {
  const double t0 = now_s();
  DBQ_CHECK(nops >= 1 && nops <= MAXLAT, "nops must be in 1..8");
  DBQ_CHECK(ops && kk && B && X && nrhs && st, "null argument");
  DBQ_CHECK(tol > 0 && std::isfinite(tol), "tol must be positive");
  DBQ_CHECK(max_mv >= 1, "max_mv must be >= 1");
  DBQ_CHECK(prec == DBQ_FP64 || prec == DBQ_MIXED, "bad precision");
  for (int i = 0; i < nops; ++i) {
    check_op(&ops[i]);
    DBQ_CHECK(nrhs[i] >= 1, "nrhs must be >= 1");
    DBQ_CHECK(kk[i] >= 0 && kk[i] <= 128, "k must be in 0..128");
    DBQ_CHECK(kk[i] == 0 || (Vin && Vin[i]), "null deflation vectors");
    DBQ_CHECK(B[i] && X[i], "null right-hand side or solution");
  }
  // s follows c->stream, which a graph capture points at the capture stream for its duration
  hipStream_t& s = c->stream;
  const bool mixed = prec == DBQ_MIXED;
  WsScope ws(c);
  std::vector<Op> op(nops);
  for (int i = 0; i < nops; ++i) op[i] = make_op(c, ws, &ops[i], true, mixed);
  for (int i = 1; i < nops; ++i)
    DBQ_CHECK(op[i].schur == op[0].schur, "operators of one call must all be full or all reduced");

  // ---- right-hand-side bookkeeping
  std::vector<int> base(nops), lat_of;
  std::vector<int> ne64, ne32;
  std::vector<long long> off64, off32;
  int NR = 0;
  long long tot64 = 0, tot32 = 0;
  for (int i = 0; i < nops; ++i) {
    base[i] = NR;
    for (int r = 0; r < nrhs[i]; ++r) {
      lat_of.push_back(i);
      ne64.push_back(int(op[i].n()));
      ne32.push_back(int(op[i].n() / 2));
      off64.push_back(tot64);
      off32.push_back(tot32);
      tot64 += op[i].n();
      tot32 += op[i].n() / 2;
      ++NR;
    }
  }
  double2* b64 = ws.get<double2>(tot64);
  double2* x64 = ws.get<double2>(tot64);
  double2* r64 = ws.get<double2>(tot64);
  // reduced operator: the iteration runs on bhat and x_e; the packed full b gives ||b|| and its
  // odd half the odd half of the solution
  std::vector<double2*> bfull(nops, nullptr), bodd(nops, nullptr);
  for (int i = 0; i < nops; ++i) {
    const long long o = off64[base[i]];
    if (op[i].schur) {
      bfull[i] = ws.get<double2>(size_t(op[i].nfull()) * nrhs[i]);
      bodd[i] = ws.get<double2>(size_t(op[i].n()) * nrhs[i]);
      pack_spinor_f64(s, op[i].g, B[i], bfull[i], nrhs[i]);
      schur_rhs(c, ws, op[i], bfull[i], b64 + o, bodd[i], nrhs[i], dagger);
      pack_even_f64(c, ws, op[i], X[i], x64 + o, nrhs[i]);
    } else {
      pack_spinor_f64(s, op[i].g, B[i], b64 + o, nrhs[i]);
      pack_spinor_f64(s, op[i].g, X[i], x64 + o, nrhs[i]);
    }
  }
  VecSet vs64 = make_vecset(c, ws, ne64);
  VecSet vs32{};
  if (mixed) vs32 = make_vecset(c, ws, ne32);

  // ---- scratch for reductions
  int pstride = std::max(vs64.pstride, mixed ? vs32.pstride : 1);
  for (int i = 0; i < nops; ++i) pstride = std::max(pstride, ds_partial_slots(op[i].g));
  // 3 doubles per slot, and 4 more for <rhat, t> and <rhat, s> of the <t, s> epilogue
  double* partials = ws.get<double>(size_t(NR) * pstride * DS_NSUM);
  RhsScal* sc = ws.get<RhsScal>(NR);
  // pinned host area: scalars | norms | cond
  const size_t pin_bytes = sizeof(RhsScal) * NR + sizeof(double) * (2 * NR + MAXLAT) + 256;
  char* pin = (char*)pinned_get(c, pin_bytes);
  RhsScal* hs = (RhsScal*)pin;
  double* hn = (double*)(pin + sizeof(RhsScal) * NR);
  double* hcond = hn + 2 * NR;
  auto pull = [&]() {
    DBQ_HIP(hipMemcpyAsync(hs, sc, sizeof(RhsScal) * NR, hipMemcpyDeviceToHost, s));
    DBQ_HIP(hipStreamSynchronize(s));
  };
  auto push = [&]() {
    DBQ_HIP(hipMemcpyAsync(sc, hs, sizeof(RhsScal) * NR, hipMemcpyHostToDevice, s));
  };

  // ---- norms of b and x0
  double* dn = ws.get<double>(2 * NR);
  long long maxn = 0;
  int maxr = 1;
  for (int i = 0; i < nops; ++i) {
    maxn = std::max(maxn, op[i].nfull());
    maxr = std::max(maxr, nrhs[i]);
  }
  size_t nw = norm_work(maxn, maxr);
  double* nwork = ws.get<double>(nw);
  for (int i = 0; i < nops; ++i) {
    // tol is relative to ||b|| of the full system also for the reduced operator
    const double2* bn = op[i].schur ? bfull[i] : b64 + off64[base[i]];
    const long long nn = op[i].schur ? op[i].nfull() : op[i].n();
    norm2_f64(s, bn, nn, nrhs[i], nn, dn + base[i], nwork, nw);
    norm2_f64(s, x64 + off64[base[i]], op[i].n(), nrhs[i], op[i].n(), dn + NR + base[i], nwork, nw);
  }
  DBQ_HIP(hipMemcpyAsync(hn, dn, sizeof(double) * 2 * NR, hipMemcpyDeviceToHost, s));
  DBQ_HIP(hipStreamSynchronize(s));

  std::vector<long long> mvb(NR, 0);
  std::vector<int> status(NR, DBQ_NOT_CONVERGED), restarts(NR, 0), relup(NR, 0);
  std::vector<char> done(NR, 0), have_true(NR, 0), stalled(NR, 0), rescued(NR, 0);
  // FP32 iterations that produced a non-finite value: their FP32 correction is dropped, and
  // zero_start marks those whose FP64 solution is not finite either
  std::vector<char> discard(NR, 0), zero_start(NR, 0);
  std::vector<double> rrt(NR, 0.0);
  std::memset(hs, 0, sizeof(RhsScal) * NR);
  bool any_x0 = false;
  for (int j = 0; j < NR; ++j) {
    RhsScal& q = hs[j];
    q.bb = hn[j];
    q.stop2 = tol * tol * hn[j];
    // reliable update (FP64 residual, then a restart of the FP32 recursion from it) when ||r||
    // drops by 1000x.  Against replacing r at 10x drops and keeping rhat and p, restarts stop
    // the FP32 recursion from stagnating on the twisted-mass shifts at kappa_c and save products
    // on 16^4.  Measured drop factors 30 / 100 / 300 / 1000, ms per source on 16^4 x 72 sources:
    // 13.1 / 12.6 / 12.8 / 12.1; 20^3 x 32 x 24: 47.9 / 42.6 / 39.2 / 39.6; seconds for the
    // mu = 0.0015 shift on 24^3 x 48 x 12: 11.6 / 12.7 / 11.6 / 14.5.  (With the forced check
    // after 500 iterations, 3000 and 10000: 12.5 and 12.6 ms on 16^4, 39.0 and 41.5 ms on
    // 20^3 x 32, 13.8 and 14.0 s on the shift, against 12.2 / 39.6 / 12.5 at 1000.)
    q.delta2 = mixed ? 1e-6 : 0.0;
    q.sel = hn[NR + j] > 0.0 ? 1 : 0;
    if (q.sel) {
      any_x0 = true;
      mvb[j] += 1;
    }
    q.active = 0;
    if (!std::isfinite(hn[j]) || !std::isfinite(hn[NR + j]))
      throw Error(DBQ_EINVAL, "non-finite right-hand side or initial guess");
  }
  push();

  // ---- r0 = b - A x0
  double2* rt = mixed ? r64 : ws.get<double2>(tot64);  // FP64 true-residual target
  std::vector<DsSpec> sres, sx0;
  for (int i = 0; i < nops; ++i) {
    const long long o = off64[base[i]];
    sx0.push_back(DsSpec{&op[i], false, x64 + o, r64 + o, b64 + o, nrhs[i], base[i]});
    sres.push_back(DsSpec{&op[i], false, x64 + o, rt + o, b64 + o, nrhs[i], base[i]});
  }
  const DsBatch bx0 = make_batch(sx0), bres = make_batch(sres);
  copy_f64(s, b64, r64, tot64);
  if (any_x0) run_dslash(c, false, bx0, dagger, EPI_RESID, sc, partials);

  // ---- deflation: (U^H A V) y = U^H r0, x0 += V y with U = gamma5 V (roles swapped for A^H)
  bool any_defl = false;
  double* dcond = ws.get<double>(MAXLAT);
  // Mixed precision keeps W = A V (and forms (U^H A V)^{-1} when first needed) to apply the same
  // projection again to the FP64 residual of an rhs whose FP32 recursion stalled, and from then
  // on at each of its reliable updates, before a second stall gives it to the FP64 continuation.
  // DBQ_REPROJECT=1 applies it to every rhs at every reliable update (measured: slower on the
  // benchmark problem, where no rhs stalls)
  struct Reproj {
    const double2 *left = nullptr, *right = nullptr, *W = nullptr, *M = nullptr;
    double2 *Minv = nullptr, *C = nullptr, *Y = nullptr, *lw = nullptr;
    double* gwork = nullptr;
    size_t gw = 0;
    bool inverted = false;
  };
  std::vector<Reproj> rp(nops);
  bool reproject = false;
  if (mixed)
    if (const char* e = std::getenv("DBQ_REPROJECT")) reproject = std::atoi(e) != 0;
  // DBQ_STALL_REPROJECT=0 sends a stalled rhs straight to the FP64 continuation
  bool rescue = mixed;
  if (const char* e = std::getenv("DBQ_STALL_REPROJECT")) rescue = mixed && std::atoi(e) != 0;
  for (int i = 0; i < nops; ++i) {
    const int k = kk[i];
    if (k == 0) continue;
    any_defl = true;
    const long long n = op[i].n(), V = op[i].sites();
    const long long o = off64[base[i]];
    double2* Vp = ws.get<double2>(k * n);
    if (op[i].schur) pack_even_f64(c, ws, op[i], Vin[i], Vp, k);
    else pack_spinor_f64(s, op[i].g, Vin[i], Vp, k);
    const double2* right = Vp;
    if (dagger) {
      double2* R5 = ws.get<double2>(k * n);
      gamma5_f64(s, Vp, R5, V, k);
      right = R5;
    }
    double2* W = ws.get<double2>(k * n);
    const DsBatch bw = make_batch({DsSpec{&op[i], false, right, W, nullptr, k, 0}});
    run_dslash(c, false, bw, dagger, EPI_NONE, nullptr, nullptr);
    const size_t gw = gram_work_elems(n, k, std::max(k, nrhs[i]));
    double* gwork = ws.get<double>(gw);
    double2* M = ws.get<double2>(k * k);
    double2* Cm = ws.get<double2>(k * nrhs[i]);
    gram_f64(s, Vp, n, k, W, n, k, n, V, dagger ? 0 : 1, M, gwork, gw);
    gram_f64(s, Vp, n, k, r64 + o, n, nrhs[i], n, V, dagger ? 0 : 1, Cm, gwork, gw);
    double2* lw = ws.get<double2>(2 * k * k + k);
    if (reproject || rescue) {
      Reproj& R = rp[i];
      R.left = Vp;
      R.right = Vp;
      R.W = W;
      R.M = M;
      R.lw = ws.get<double2>(2 * k * k + k);
      R.Minv = ws.get<double2>(size_t(k) * k);
      R.C = ws.get<double2>(size_t(k) * nrhs[i]);
      R.Y = ws.get<double2>(size_t(k) * nrhs[i]);
      R.gwork = gwork;
      R.gw = gw;
    }
    dense_lu_solve(s, M, k, Cm, nrhs[i], lw, dcond + i);
    combine_f64(s, Vp, n, k, Cm, k, x64 + o, n, nrhs[i], n, V, dagger ? 1 : 0, 1);
    DBQ_HIP(hipMemcpyAsync(hcond + i, dcond + i, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  if (any_defl) {
    DBQ_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nops; ++i)
      if (kk[i] > 0 && !(hcond[i] <= 1e12))
        throw Error(DBQ_ESINGULAR, "projected matrix U^H A V is numerically singular (cond " +
                                       std::to_string(hcond[i]) + ")");
    // r = b - A x after the projection (one MVP per rhs)
    pull();
    for (int j = 0; j < NR; ++j) {
      hs[j].sel = kk[lat_of[j]] > 0 ? 1 : 0;
      if (hs[j].sel) mvb[j] += 1;
    }
    push();
    run_dslash(c, false, bx0, dagger, EPI_RESID, sc, partials);
  }

  // ---- BiCGStab working vectors
  double2 *rhat = nullptr, *p = nullptr, *v = nullptr, *t = nullptr;
  float4 *x32 = nullptr, *r32 = nullptr, *rhat32 = nullptr, *p32 = nullptr, *v32 = nullptr,
         *t32 = nullptr;
  if (mixed) {
    x32 = ws.get<float4>(tot32);
    // zeroed here so that right-hand sides which never start iterating (b = 0) add nothing
    zero_f64(s, reinterpret_cast<double2*>(x32), tot32);
    r32 = ws.get<float4>(tot32);
    rhat32 = ws.get<float4>(tot32);
    p32 = ws.get<float4>(tot32);
    v32 = ws.get<float4>(tot32);
    t32 = ws.get<float4>(tot32);
  } else {
    rhat = ws.get<double2>(tot64);
    p = ws.get<double2>(tot64);
    v = ws.get<double2>(tot64);
    t = ws.get<double2>(tot64);
  }
  std::vector<DsSpec> sv, stt;
  for (int i = 0; i < nops; ++i) {
    if (mixed) {
      const long long o = off32[base[i]];
      sv.push_back(DsSpec{&op[i], true, p32 + o, v32 + o, rhat32 + o, nrhs[i], base[i]});
      stt.push_back(DsSpec{&op[i], true, r32 + o, t32 + o, rhat32 + o, nrhs[i], base[i]});
    } else {
      const long long o = off64[base[i]];
      sv.push_back(DsSpec{&op[i], false, p + o, v + o, rhat + o, nrhs[i], base[i]});
      stt.push_back(DsSpec{&op[i], false, r64 + o, t + o, rhat + o, nrhs[i], base[i]});
    }
  }
  const DsBatch bv = make_batch(sv), bt = make_batch(stt);
  // Mixed precision: the update step's partial sums of ||r||^2 go to the second partial region
  // (which only the <t, s> epilogue uses, later in the iteration), so that they outlast the next
  // iteration's v = A p and the <rhat, v> finalize (batch bv_xr) can end the iteration in place
  // of a separate finalize launch.  FP64 keeps the separate launch and the first region.
  double* xr_part = mixed ? partials + size_t(NR) * pstride * 3 : partials;
  DsBatch bv_xr = bv;
  if (mixed) {
    bv_xr.xr_part = xr_part;
    bv_xr.xr_nelem = vs32.nelem;
    bv_xr.xr_pstride = vs32.pstride;
  }

  pull();
  for (int j = 0; j < NR; ++j) {
    hs[j].sel = 0;
    if (hs[j].bb == 0.0) {
      done[j] = 1;
      status[j] = DBQ_OK;
      have_true[j] = 1;
      rrt[j] = 0.0;
      hs[j].active = 0;
      zero_f64(s, x64 + off64[j], ne64[j]);
    } else {
      hs[j].active = 1;
    }
  }
  push();
  if (mixed)
    bicg_aux_f32(s, AX_INIT, vs32, vs64, r64, r32, rhat32, p32, v32, x32, sc, partials);
  else
    bicg_aux_f64(s, AX_INIT, vs64, r64, r64, rhat, p, v, sc, partials);

  // pending: the previous iteration's end (fin_xr) is still to be done, by this iteration's
  // <rhat, v> finalize; defer: leave this iteration's end to the next one (mixed precision only,
  // and only where another iteration follows before anything reads the scalars)
  auto iterate = [&](bool pending, bool defer) {
    if (mixed) {
      run_dslash(c, true, pending ? bv_xr : bv, dagger, EPI_RHAT, sc, partials);
      bicg_step_f32(s, BI_S, vs32, x32, r32, rhat32, p32, v32, t32, sc, partials);
      run_dslash(c, true, bt, dagger, EPI_TS, sc, partials);
      // the update kernel alone is timed (kind 2), its bytes counted on the device
      hipEvent_t e0;
      timer_begin(c, 2, &e0);
      bicg_step_f32(s, BI_XR, vs32, x32, r32, rhat32, p32, v32, t32, sc, xr_part,
                    e0 ? c->acct + 2 : nullptr);
      timer_end(c, 2, e0, 0.0);
      if (!defer) bicg_fin_xr(s, vs32, sc, xr_part);
    } else {
      run_dslash(c, false, bv, dagger, EPI_RHAT, sc, partials);
      bicg_step_f64(s, BI_S, vs64, x64, r64, rhat, p, v, t, sc, partials);
      run_dslash(c, false, bt, dagger, EPI_TS, sc, partials);
      bicg_step_f64(s, BI_XR, vs64, x64, r64, rhat, p, v, t, sc, partials);
      bicg_fin_xr(s, vs64, sc, partials);
    }
  };

  const bool debug = std::getenv("DBQ_DEBUG") != nullptr;
  auto trace = [&]() {
    if (!debug) return;
    for (int j = 0; j < NR; ++j)
      if (!done[j])
        std::fprintf(stderr, "[dbq] rhs %d it %d flags %d act %d sel %d rr %.3e/%.3e rr_max %.3e nrel %d\n",
                     j, hs[j].iters, hs[j].flags, hs[j].active, hs[j].sel, hs[j].rr, hs[j].bb,
                     hs[j].rr_max, hs[j].nrel);
  };
  // breakdowns: restart with rhat <- r (the selection is pushed with the host scalars).  Polls
  // of the mixed loop follow a reliable-update block, after which no rhs waits with sel set;
  // a selection that is still pending is kept (the restart then restarts that rhs as well and
  // it carries on iterating) rather than cleared, which would leave it neither live nor done.
  auto restart = [&](const std::vector<int>& Bk) {
    if (!mixed)
      for (int j = 0; j < NR; ++j) hs[j].sel = 0;
    bool any = false;
    for (int j : Bk) {
      if (done[j]) continue;
      restarts[j] += 1;
      if (restarts[j] > 10) {
        done[j] = 1;
        status[j] = DBQ_EBREAKDOWN;
        hs[j].active = 0;
      } else {
        hs[j].sel = 1;
        any = true;
      }
    }
    push();
    if (any) {
      if (mixed)
        bicg_aux_f32(s, AX_RESTART, vs32, vs64, r64, r32, rhat32, p32, v32, x32, sc, partials);
      else
        bicg_aux_f64(s, AX_RESTART, vs64, r64, r64, rhat, p, v, sc, partials);
    }
  };
  if (mixed) {
    // Reliable updates on the device: every `every` iterations the rhs that claimed convergence
    // or dropped by the reliable-update factor (selected by the iteration's finalize) get
    // x64 += x32 and the FP64 residual; the residual's finalize stops the converged ones and the
    // others continue from the replaced residual.  The host only polls for rhs that finished,
    // broke down or ran out of MVPs, at intervals that double up to 32 iterations.
    // (every = 16: a flagged rhs idles until the next check, so the interval changes no
    // iteration or product count; on 16^4 with 6 x 12 sources 8 -> 16 is 0.7% faster per source,
    // 24 and 32 are 3% slower than 16: the last rhs of a batch waits longer for its check)
    int every = 16;
    if (const char* e = std::getenv("DBQ_RELUP_EVERY")) every = std::max(1, std::atoi(e));
    DsBatch bres_dec = bres;
    bres_dec.decide = 1;
    // (U^H A V)^{-1}, formed when first needed (outside any captured block)
    auto invert = [&]() {
      for (int i = 0; i < nops; ++i) {
        Reproj& R = rp[i];
        if (!R.W || R.inverted) continue;
        const int k = kk[i];
        std::vector<double2> id(size_t(k) * k, make_double2(0.0, 0.0));
        for (int q = 0; q < k; ++q) id[q + size_t(q) * k] = make_double2(1.0, 0.0);
        DBQ_HIP(hipMemcpyAsync(R.Minv, id.data(), sizeof(double2) * id.size(),
                               hipMemcpyHostToDevice, s));
        DBQ_HIP(hipStreamSynchronize(s));
        dense_lu_solve(s, R.M, k, R.Minv, k, R.lw, dcond + i);
        R.inverted = true;
      }
    };
    if (reproject) invert();
    // y = (U^H A V)^{-1} U^H r for the selected rhs (with flagged_only, those with reproj set),
    // x += V y, r -= W y (FP64; no products)
    bool any_reproj = false;
    auto project_sel = [&](bool flagged_only) {
      for (int i = 0; i < nops; ++i) {
        const Reproj& R = rp[i];
        if (!R.W) continue;
        const int k = kk[i];
        const long long n = op[i].n(), V = op[i].sites(), o = off64[base[i]];
        gram_f64(s, R.left, n, k, r64 + o, n, nrhs[i], n, V, dagger ? 0 : 1, R.C, R.gwork, R.gw);
        combine_f64(s, R.Minv, k, k, R.C, k, R.Y, k, nrhs[i], k, 1, 0, 0);
        mask_unselected_f64(s, R.Y, k, nrhs[i], sc + base[i], flagged_only);
        combine_f64(s, R.right, n, k, R.Y, k, x64 + o, n, nrhs[i], n, V, dagger ? 1 : 0, 1);
        combine_f64(s, R.W, n, k, R.Y, k, r64 + o, n, nrhs[i], n, V, 0, -1);
      }
    };
    auto relup_dev = [&]() {
      bicg_xacc(s, vs32, vs64, x64, x32, sc);
      run_dslash(c, false, bres_dec, dagger, EPI_RESID, sc, partials);
      if (reproject || any_reproj) project_sel(!reproject);
      bicg_aux_f32(s, AX_REPLACE, vs32, vs64, r64, r32, rhat32, p32, v32, x32, sc, partials);
    };
    // an iteration followed by another one leaves its end to that one's <rhat, v> finalize;
    // the last one before a reliable-update step ends itself
    auto block = [&](int n) {
      for (int it = 1; it <= n; ++it) {
        iterate(it > 1 && (it - 1) % every != 0, it % every != 0);
        if (it % every == 0) relup_dev();
      }
    };
    // Blocks of iterations between two polls run as HIP graphs: the launches of a block (6-7 per
    // iteration, 5 for the reliable-update step) are captured once per solve and block length
    // and replayed, so the host issues one launch per block.  The first block runs eagerly
    // (it tunes the launch shapes and settles the workspace the graphs capture).
    LoopGraphs graphs(c, op[0].schur ? tot64 * sizeof(double2) : 0, ws);
    const LoopGraphs::G* replayed = nullptr;
    relup_dev();  // rhs whose starting residual already meets the tolerance
    int nchk = every;
    while (true) {
      pull();
      if (replayed && c->timing) graph_timers_add(c, replayed->timers);
      replayed = nullptr;
      trace();
      std::vector<int> Bk, Cc, Rs;
      bool live = false;
      for (int j = 0; j < NR; ++j) {
        if (done[j]) continue;
        const RhsScal& q = hs[j];
        const long long mv = mvb[j] + q.nrel + 2LL * q.iters;
        if (q.flags & F_DONE) {
          done[j] = 1;
          status[j] = DBQ_OK;
          rrt[j] = q.rr_true;
          have_true[j] = 1;
        } else if (q.flags & F_STALL) {
          if (rescue && !rescued[j] && rp[lat_of[j]].W) {
            // first stall: the deflation projection again, then FP32 from there with the
            // projection repeated at each FP64 residual of this rhs (a second stall hands it to
            // the FP64 continuation)
            Rs.push_back(j);
          } else {
            done[j] = 1;
            stalled[j] = 1;
            rrt[j] = q.rr_true;
            have_true[j] = 1;
          }
        } else if (q.flags & F_NAN) {
          // continued in FP64 like a stall, from the last accumulated solution
          done[j] = 1;
          stalled[j] = 1;
          discard[j] = 1;
          zero_start[j] = std::isfinite(q.rr_true) ? 0 : 1;
          rrt[j] = q.rr_true;
          have_true[j] = 1;
          Cc.push_back(j);
        } else if (q.flags & F_BREAK) {
          Bk.push_back(j);
        } else if (mv >= max_mv) {
          Cc.push_back(j);
        } else if (q.active || q.sel) {
          live = true;
        }
      }
      if (!Cc.empty()) {
        for (int j : Cc) {
          done[j] = 1;
          if (status[j] != DBQ_EBREAKDOWN) status[j] = DBQ_NOT_CONVERGED;
          hs[j].active = 0;
          hs[j].sel = 0;
        }
        if (Bk.empty()) push();
      }
      if (!Rs.empty()) {
        // r64 holds the stalled rhs' FP64 residual of that check and x64 its solution
        for (int j = 0; j < NR; ++j)
          if (!done[j]) hs[j].sel = 0;
        for (int j : Rs) {
          hs[j].sel = 1;
          hs[j].flags = 0;
          hs[j].stalls = 0;
          hs[j].reproj = 1;
          rescued[j] = 1;
        }
        any_reproj = true;
        push();
        invert();
        project_sel(false);
        bicg_aux_f32(s, AX_REPLACE, vs32, vs64, r64, r32, rhat32, p32, v32, x32, sc, partials);
        pull();
        for (int j : Rs) hs[j].rr_prev = hs[j].rr;  // the next check compares with this residual
        push();
        live = true;
      }
      if (!Bk.empty()) {
        restart(Bk);
        live = true;
      }
      if (!live) break;
      nchk = (Bk.empty() && Cc.empty()) ? std::min(nchk * 2, std::max(32, every)) : every;
      // every poll comes right after a reliable-update block
      nchk = ((nchk + every - 1) / every) * every;
      replayed = graphs.run(2 * nchk + (any_reproj ? 1 : 0), nchk, block);
    }
    for (int j = 0; j < NR; ++j)
      if (!done[j])
        throw Error(DBQ_EHIP, "internal error: right-hand side " + std::to_string(j) +
                                  " left the mixed-precision loop undecided (flags " +
                                  std::to_string(hs[j].flags) + ")");
  } else {
    int nchk = 1;
    bool first = true;
    while (true) {
      if (!first)
        for (int it = 0; it < nchk; ++it) iterate(false, false);
      first = false;
      pull();
      if (debug) {
        for (int j = 0; j < NR; ++j)
          if (!done[j])
            std::fprintf(stderr, "[dbq] rhs %d it %d flags %d act %d rr %.3e/%.3e rr_max %.3e mvb %lld\n",
                         j, hs[j].iters, hs[j].flags, hs[j].active, hs[j].rr, hs[j].bb, hs[j].rr_max,
                         (long long)mvb[j]);
      }
      std::vector<int> A, Bk, Cc;
      bool any_active = false;
      for (int j = 0; j < NR; ++j) {
        if (done[j]) continue;
        const RhsScal& q = hs[j];
        const long long mv = mvb[j] + 2LL * q.iters;
        if (q.flags & F_NAN) {
          done[j] = 1;
          status[j] = DBQ_EBREAKDOWN;
          Cc.push_back(j);
        } else if (q.flags & (F_CONV | F_RELIABLE)) {
          A.push_back(j);
        } else if (q.flags & F_BREAK) {
          Bk.push_back(j);
        } else if (mv >= max_mv) {
          Cc.push_back(j);
        }
        if (q.active) any_active = true;
      }
      if (A.empty() && Bk.empty() && Cc.empty()) {
        if (!any_active) break;
        nchk = std::min(nchk * 2, 16);
        continue;
      }
      nchk = 1;
      // (1) convergence claims and reliable updates: FP64 residual of the accumulated solution
      if (!A.empty()) {
        for (int j = 0; j < NR; ++j) hs[j].sel = 0;
        for (int j : A) hs[j].sel = 1;
        push();
        if (mixed) bicg_xacc(s, vs32, vs64, x64, x32, sc);
        run_dslash(c, false, bres, dagger, EPI_RESID, sc, partials);
        pull();
        bool any_rep = false;
        for (int j : A) {
          mvb[j] += 1;
          if (mixed) relup[j] += 1;
          rrt[j] = hs[j].rr_true;
          have_true[j] = 1;
          const long long mv = mvb[j] + 2LL * hs[j].iters;
          if (hs[j].rr_true <= hs[j].stop2) {
            done[j] = 1;
            status[j] = DBQ_OK;
            hs[j].sel = 0;
            hs[j].active = 0;
          } else if (mv >= max_mv || !std::isfinite(hs[j].rr_true)) {
            done[j] = 1;
            status[j] = std::isfinite(hs[j].rr_true) ? DBQ_NOT_CONVERGED : DBQ_EBREAKDOWN;
            hs[j].sel = 0;
            hs[j].active = 0;
          } else {
            any_rep = true;
            have_true[j] = 0;
          }
        }
        push();
        if (any_rep) {
          if (mixed)
            bicg_aux_f32(s, AX_REPLACE, vs32, vs64, r64, r32, rhat32, p32, v32, x32, sc, partials);
          else
            bicg_aux_f64(s, AX_REPLACE, vs64, rt, r64, rhat, p, v, sc, partials);
        }
      }
      // (2) breakdowns: restart with rhat <- r
      if (!Bk.empty()) {
        pull();
        for (int j = 0; j < NR; ++j) hs[j].sel = 0;
        bool any = false;
        for (int j : Bk) {
          if (done[j]) continue;
          restarts[j] += 1;
          if (restarts[j] > 10) {
            done[j] = 1;
            status[j] = DBQ_EBREAKDOWN;
            hs[j].active = 0;
          } else {
            hs[j].sel = 1;
            any = true;
          }
        }
        push();
        if (any) {
          if (mixed)
            bicg_aux_f32(s, AX_RESTART, vs32, vs64, r64, r32, rhat32, p32, v32, x32, sc, partials);
          else
            bicg_aux_f64(s, AX_RESTART, vs64, r64, r64, rhat, p, v, sc, partials);
        }
      }
      // (3) out of matrix-vector products
      if (!Cc.empty()) {
        pull();
        for (int j = 0; j < NR; ++j) hs[j].sel = 0;
        for (int j : Cc) {
          done[j] = 1;
          if (status[j] != DBQ_EBREAKDOWN) status[j] = DBQ_NOT_CONVERGED;
          hs[j].active = 0;
        }
        push();
      }
    }
  }

  // ---- final solution and residuals of the rhs that ended without one
  pull();
  bool need = false;
  for (int j = 0; j < NR; ++j) {
    hs[j].sel = discard[j] ? 0 : 1;  // accumulate any FP32 correction that is left
    hs[j].active = 0;
  }
  push();
  if (mixed) bicg_xacc(s, vs32, vs64, x64, x32, sc);
  pull();
  for (int j = 0; j < NR; ++j) {
    hs[j].sel = have_true[j] ? 0 : 1;
    need = need || !have_true[j];
  }
  push();
  if (need) {
    run_dslash(c, false, bres, dagger, EPI_RESID, sc, partials);
    pull();
    for (int j = 0; j < NR; ++j)
      if (!have_true[j]) rrt[j] = hs[j].rr_true;
  }
  for (int i = 0; i < nops; ++i) {
    if (op[i].schur) schur_solution(c, ws, op[i], x64 + off64[base[i]], bodd[i], X[i], nrhs[i], dagger);
    else unpack_spinor_f64(s, op[i].g, x64 + off64[base[i]], X[i], nrhs[i]);
  }
  DBQ_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < NR; ++j) {
    dbq_stats& o = st[j];
    o.matvecs = mvb[j] + hs[j].nrel + 2LL * hs[j].iters;
    o.iterations = hs[j].iters;
    o.restarts = restarts[j];
    o.reliable_updates = relup[j] + hs[j].nrel;
    o.rel_true_resid = hs[j].bb > 0 ? std::sqrt(rrt[j] / hs[j].bb) : 0.0;
    o.status = status[j];
    o.fp64_continued = 0;
  }

  // ---- rhs whose FP32 iteration stalled, diverged or broke down with a non-finite value:
  // continue them in FP64 from their current solution (from zero if that is not finite; same
  // deflation space, remaining MVP budget), gathered per lattice into contiguous buffers
  if (std::any_of(stalled.begin(), stalled.end(), [](char v) { return v != 0; })) {
    std::vector<dbq_operator> ops2;
    std::vector<const void*> V2, B2;
    std::vector<void*> X2;
    std::vector<int32_t> k2, n2;
    std::vector<std::vector<int>> rows;  // global rhs index of each rescued rhs, per lattice
    std::vector<int> lat;                // lattice of each entry of rows
    int64_t used = 0;
    for (int i = 0; i < nops; ++i) {
      std::vector<int> js;
      for (int jl = 0; jl < nrhs[i]; ++jl)
        if (stalled[base[i] + jl]) js.push_back(base[i] + jl);
      if (js.empty()) continue;
      const size_t vb = size_t(op[i].nfull()) * sizeof(double2);  // canonical full vectors
      char* bs = (char*)ws.take(vb * js.size());
      char* xs = (char*)ws.take(vb * js.size());
      for (size_t q = 0; q < js.size(); ++q) {
        const size_t jl = size_t(js[q] - base[i]);
        DBQ_HIP(hipMemcpyAsync(bs + q * vb, (const char*)B[i] + jl * vb, vb,
                               hipMemcpyDeviceToDevice, s));
        if (zero_start[js[q]])
          DBQ_HIP(hipMemsetAsync(xs + q * vb, 0, vb, s));
        else
          DBQ_HIP(hipMemcpyAsync(xs + q * vb, (const char*)X[i] + jl * vb, vb,
                                 hipMemcpyDeviceToDevice, s));
        used = std::max<int64_t>(used, st[js[q]].matvecs);
      }
      ops2.push_back(ops[i]);
      V2.push_back(Vin ? Vin[i] : nullptr);
      k2.push_back(kk[i]);
      B2.push_back(bs);
      X2.push_back(xs);
      n2.push_back(int32_t(js.size()));
      rows.push_back(js);
      lat.push_back(i);
    }
    std::vector<dbq_stats> st2(stalled.size());
    dbicgstab(c, ops2.data(), int(ops2.size()), V2.data(), k2.data(), B2.data(), X2.data(),
              n2.data(), tol, std::max<int64_t>(1, max_mv - used), DBQ_FP64, dagger, st2.data());
    size_t q2 = 0;
    for (size_t l = 0; l < rows.size(); ++l) {
      const int li = lat[l];
      const size_t vb = size_t(op[li].nfull()) * sizeof(double2);
      for (size_t q = 0; q < rows[l].size(); ++q, ++q2) {
        const int j = rows[l][q];
        DBQ_HIP(hipMemcpyAsync((char*)X[li] + size_t(j - base[li]) * vb,
                               (const char*)X2[l] + q * vb, vb, hipMemcpyDeviceToDevice, s));
        dbq_stats& o = st[j];
        const dbq_stats& r = st2[q2];
        o.matvecs += r.matvecs;
        o.iterations += r.iterations;
        o.restarts += r.restarts;
        o.rel_true_resid = r.rel_true_resid;
        o.status = r.status;
        o.fp64_continued = 1;
      }
    }
    DBQ_HIP(hipStreamSynchronize(s));
  }
  timer_collect(c);
  const double secs = now_s() - t0;
  int worst = DBQ_OK;
  for (int j = 0; j < NR; ++j) {
    st[j].seconds = secs;
    const int sj = st[j].status;
    if (sj < 0) worst = std::min(worst, sj);
    else if (worst >= 0) worst = std::max(worst, sj);
  }
  return worst;
}

// ============================================================================ Arnoldi machinery
namespace {

struct Arnoldi {
  dbq_ctx* c;
  const Op* op;
  int m;
  long long n, V;
  double2 *Vb, *Vb2;  // (m+1) x n bases
  double2 *Hbar, *Hnew, *cv, *cnew;
  double2 *d, *P, *theta, *h1, *h2, *dwork;
  double2 *G2, *cf0, *cf1;  // Gram of the step, coefficients of its combination sweep
  double *info, *nrm, *gwork, *nwork, *c1;
  size_t gw, nw;
  int dagger = 0;
  int64_t mv = 0;
  // DBQ_ARNOLDI_CGS2=1: classical Gram-Schmidt twice in four sweeps per step (for comparison)
  bool cgs2 = false;

  Arnoldi(dbq_ctx* ctx, WsScope& ws, const Op* o, int mm, int k) : c(ctx), op(o), m(mm) {
    n = o->n();
    V = o->sites();
    const int m1 = m + 1;
    Vb = ws.get<double2>(size_t(m1) * n);
    Vb2 = ws.get<double2>(size_t(m1) * n);
    Hbar = ws.get<double2>(size_t(m1) * m);
    Hnew = ws.get<double2>(size_t(m1) * m);
    cv = ws.get<double2>(m1);
    cnew = ws.get<double2>(m1);
    d = ws.get<double2>(m);
    P = ws.get<double2>(size_t(m1) * (k + 1));
    theta = ws.get<double2>(m);
    h1 = ws.get<double2>(m1);
    h2 = ws.get<double2>(m1);
    dwork = ws.get<double2>(dense_cycle_work(m));
    info = ws.get<double>(8);
    nrm = ws.get<double>(4);
    G2 = ws.get<double2>(2 * size_t(m1));
    cf0 = ws.get<double2>(m1);
    cf1 = ws.get<double2>(m1);
    c1 = ws.get<double>(1);
    const char* e = std::getenv("DBQ_ARNOLDI_CGS2");
    cgs2 = e && std::atoi(e) != 0;
    gw = gram_work_elems(n, m1, 2);
    gwork = ws.get<double>(gw);
    nw = norm_work(n, 1);
    nwork = ws.get<double>(nw);
    zero_f64(c->stream, Hbar, size_t(m1) * m);
  }

  double2* col(int j) { return Vb + size_t(j) * n; }

  // extend the Arnoldi relation from column j0 to m; columns 0..j0 are orthonormal on entry and
  // 0..m on exit
  void extend(int j0) {
    if (cgs2) {
      extend_cgs2(j0);
      return;
    }
    hipStream_t s = c->stream;
    for (int j = j0; j < m; ++j) {
      // w = A z_j, then one Gram sweep and one combination sweep over columns 0..j
      const DsBatch b = make_batch({DsSpec{op, false, col(j), col(j + 1), nullptr, 1, 0}});
      run_dslash(c, false, b, dagger, EPI_NONE, nullptr, nullptr);
      ++mv;
      gram2_f64(s, Vb, n, j + 1, col(j), n, n, G2, gwork, gw);
      arn_coef_f64(s, G2, j, j == j0 ? 1 : 0, 0, Hbar, m + 1, cf0, cf1, c1);
      arn_combine_f64(s, Vb, n, j, n, cf0, cf1, c1);
    }
    // the second pass of the last vector
    gram_f64(s, Vb, n, m + 1, col(m), n, 1, n, V, 0, G2, gwork, gw);
    arn_coef_f64(s, G2, m, 0, 1, Hbar, m + 1, cf0, nullptr, c1);
    arn_combine_f64(s, Vb, n, m, n, cf0, nullptr, c1);
  }

  void extend_cgs2(int j0) {
    hipStream_t s = c->stream;
    for (int j = j0; j < m; ++j) {
      const DsBatch b = make_batch({DsSpec{op, false, col(j), col(j + 1), nullptr, 1, 0}});
      run_dslash(c, false, b, dagger, EPI_NONE, nullptr, nullptr);
      ++mv;
      double2* w = col(j + 1);
      gram_f64(s, Vb, n, j + 1, w, n, 1, n, V, 0, h1, gwork, gw);
      combine_f64(s, Vb, n, j + 1, h1, j + 1, w, n, 1, n, V, 0, -1);
      gram_f64(s, Vb, n, j + 1, w, n, 1, n, V, 0, h2, gwork, gw);
      combine_f64(s, Vb, n, j + 1, h2, j + 1, w, n, 1, n, V, 0, -1);
      norm2_f64(s, w, n, 1, n, nrm, nwork, nw);
      write_col_f64(s, Hbar, m + 1, j, j + 1, h1, h2, nrm, j + 1);
      scale_f64(s, w, w, n, nrm);
    }
  }

  void cycle_end(int k, int mode, double tol_abs) {
    CycleArgs a;
    a.Hbar = Hbar;
    a.c = cv;
    a.m = m;
    a.k = k;
    a.mode = mode;
    a.tol_abs = tol_abs;
    a.d = d;
    a.P = P;
    a.Hnew = Hnew;
    a.cnew = cnew;
    a.theta = theta;
    a.info = info;
    a.work = dwork;
    zero_f64(c->stream, Hnew, size_t(m + 1) * m);
    dense_cycle(c->stream, a);
  }

  // V_{k+1} = V_{m+1} P_{k+1}; Hbar <- Hnew; c <- cnew
  void restart(int k) {
    combine_f64(c->stream, Vb, n, m + 1, P, m + 1, Vb2, n, k + 1, n, V, 0, 0);
    std::swap(Vb, Vb2);
    std::swap(Hbar, Hnew);
    std::swap(cv, cnew);
  }
};

}  // namespace

// ============================================================================ GMRES-DR(m,k)
int gmresdr(dbq_ctx* c, const dbq_operator* o, const void* b, void* x, int m, int k, double tol,
            int64_t max_mv, void* Vout, double* theta, int32_t* k_out, dbq_stats* st) {
  const double t0 = now_s();
  check_op(o);
  DBQ_CHECK(b && x && Vout && theta && k_out && st, "null argument");
  DBQ_CHECK(k >= 2 && k < m && m <= 128, "need 2 <= k < m <= 128");
  DBQ_CHECK(tol > 0 && std::isfinite(tol), "tol must be positive");
  DBQ_CHECK(max_mv >= 1, "max_mv must be >= 1");
  hipStream_t s = c->stream;
  WsScope ws(c);
  Op op = make_op(c, ws, o, true, false);
  const long long n = op.n();
  double2* b64 = ws.get<double2>(n);
  double2* x64 = ws.get<double2>(n);
  double2* tmp = ws.get<double2>(n);
  double2 *bfull = nullptr, *bodd = nullptr;
  if (op.schur) {
    // the Krylov space of Ahat from bhat and x_e; ||b|| of the full system sets the tolerance
    bfull = ws.get<double2>(op.nfull());
    bodd = ws.get<double2>(n);
    pack_spinor_f64(s, op.g, b, bfull, 1);
    schur_rhs(c, ws, op, bfull, b64, bodd, 1, 0);
    pack_even_f64(c, ws, op, x, x64, 1);
  } else {
    pack_spinor_f64(s, op.g, b, b64, 1);
    pack_spinor_f64(s, op.g, x, x64, 1);
  }
  Arnoldi ar(c, ws, &op, m, k);
  double* dn = ws.get<double>(4);
  double* hp = (double*)pinned_get(c, 64 * sizeof(double) + 2 * 128 * sizeof(double2));
  if (op.schur) {
    const size_t nwf = norm_work(op.nfull(), 1);
    double* wf = ws.get<double>(nwf);
    norm2_f64(s, bfull, op.nfull(), 1, op.nfull(), dn, wf, nwf);
  } else {
    norm2_f64(s, b64, n, 1, n, dn, ar.nwork, ar.nw);
  }
  norm2_f64(s, x64, n, 1, n, dn + 1, ar.nwork, ar.nw);
  DBQ_HIP(hipMemcpyAsync(hp, dn, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  DBQ_HIP(hipStreamSynchronize(s));
  const double bn = std::sqrt(hp[0]);
  DBQ_CHECK(std::isfinite(hp[0]) && std::isfinite(hp[1]), "non-finite b or x0");
  DBQ_CHECK(bn > 0, "b must be nonzero");
  // r0 -> v_1, c = ||r0|| e_1
  if (hp[1] > 0) {
    const DsBatch bb = make_batch({DsSpec{&op, false, x64, tmp, nullptr, 1, 0}});
    run_dslash(c, false, bb, 0, EPI_NONE, nullptr, nullptr);
    sub_f64(s, b64, tmp, ar.col(0), n);
    ar.mv += 1;
  } else {
    copy_f64(s, b64, ar.col(0), n);
  }
  norm2_f64(s, ar.col(0), n, 1, n, ar.nrm, ar.nwork, ar.nw);
  set_e1_f64(s, ar.cv, m + 1, ar.nrm);
  scale_f64(s, ar.col(0), ar.col(0), n, ar.nrm);
  int j0 = 0, cycles = 0;
  bool conv = false;
  while (true) {
    ar.extend(j0);
    ++cycles;
    ar.cycle_end(k, 0, tol * bn);
    combine_f64(s, ar.Vb, n, m, ar.d, m, x64, n, 1, n, op.sites(), 0, 1);
    DBQ_HIP(hipMemcpyAsync(hp, ar.info, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    DBQ_HIP(hipStreamSynchronize(s));
    conv = hp[2] != 0.0;
    if (!std::isfinite(hp[0])) throw Error(DBQ_EBREAKDOWN, "GMRES-DR residual is not finite");
    if (conv || ar.mv >= max_mv) break;
    if (hp[4] != 0.0) throw Error(DBQ_EBREAKDOWN, "harmonic Ritz eigensolver did not converge");
    ar.restart(k);
    j0 = k;
  }
  // eigenvector output of the last cycle (harmonic Ritz, conjugate-closed k)
  ar.cycle_end(k, 1, tol * bn);
  DBQ_HIP(hipMemcpyAsync(hp, ar.info, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
  double2* th_h = (double2*)(hp + 64);
  DBQ_HIP(hipMemcpyAsync(th_h, ar.theta, sizeof(double2) * m, hipMemcpyDeviceToHost, s));
  DBQ_HIP(hipStreamSynchronize(s));
  const int kout = int(hp[1]);
  double2* Vint = ws.get<double2>(size_t(kout) * n);
  combine_f64(s, ar.Vb, n, m, ar.P, m + 1, Vint, n, kout, n, op.sites(), 0, 0);
  if (op.schur) {
    unpack_even_f64(c, ws, op, Vint, Vout, kout);
    schur_solution(c, ws, op, x64, bodd, x, 1, 0);
  } else {
    unpack_spinor_f64(s, op.g, Vint, Vout, kout);
    unpack_spinor_f64(s, op.g, x64, x, 1);
  }
  for (int i = 0; i < kout; ++i) {
    theta[2 * i] = th_h[i].x;
    theta[2 * i + 1] = th_h[i].y;
  }
  for (int i = kout; i < k; ++i) theta[2 * i] = theta[2 * i + 1] = 0.0;
  *k_out = kout;
  // true residual for the statistics (not charged as a matrix-vector product)
  const DsBatch bb = make_batch({DsSpec{&op, false, x64, tmp, nullptr, 1, 0}});
  run_dslash(c, false, bb, 0, EPI_NONE, nullptr, nullptr);
  sub_f64(s, b64, tmp, tmp, n);
  norm2_f64(s, tmp, n, 1, n, dn + 2, ar.nwork, ar.nw);
  DBQ_HIP(hipMemcpyAsync(hp, dn + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  DBQ_HIP(hipStreamSynchronize(s));
  timer_collect(c);
  st->matvecs = ar.mv;
  st->iterations = cycles;
  st->restarts = cycles - 1;
  st->reliable_updates = 0;
  st->rel_true_resid = std::sqrt(hp[0]) / bn;
  st->seconds = now_s() - t0;
  st->status = conv ? DBQ_OK : DBQ_NOT_CONVERGED;
  st->fp64_continued = 0;
  return st->status;
}

// ============================================================================ kappa_c
int kappa_crit(dbq_ctx* c, const int32_t L[4], const void* links, int m, int k, double tol,
               int64_t max_mv, double* kappa_c, double* lambda, double* resid, int nritz,
               double* ritz) {
  DBQ_CHECK(L && links && kappa_c && lambda && resid, "null argument");
  DBQ_CHECK(k >= 2 && k < m && m <= 128, "need 2 <= k < m <= 128");
  DBQ_CHECK(nritz >= 0 && nritz <= k && (nritz == 0 || ritz), "nritz must be in 0..k");
  dbq_operator o;
  for (int i = 0; i < 4; ++i) o.L[i] = L[i];
  o.links = links;
  o.kappa = -1.0;  // apply I + H: same eigenvectors, eigenvalues shifted by one
  o.mu = 0.0;
  o.schur = 0;
  o.pad = 0;
  check_op(&o);
  hipStream_t s = c->stream;
  WsScope ws(c);
  Op op = make_op(c, ws, &o, true, false);
  const long long n = op.n();
  Arnoldi ar(c, ws, &op, m, k);
  double* hp = (double*)pinned_get(c, 64 * sizeof(double) + 2 * 128 * sizeof(double2));
  fill_hash_f64(s, ar.col(0), n, 0x5DEECE66Dull);
  norm2_f64(s, ar.col(0), n, 1, n, ar.nrm, ar.nwork, ar.nw);
  scale_f64(s, ar.col(0), ar.col(0), n, ar.nrm);
  int j0 = 0;
  double lam_re = 0, lam_im = 0, res = INFINITY;
  const bool debug = std::getenv("DBQ_DEBUG") != nullptr;
  while (true) {
    ar.extend(j0);
    ar.cycle_end(k, 2, 0.0);
    DBQ_HIP(hipMemcpyAsync(hp, ar.info, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    double2* th_h = (double2*)(hp + 64);
    DBQ_HIP(hipMemcpyAsync(th_h, ar.theta, sizeof(double2), hipMemcpyDeviceToHost, s));
    DBQ_HIP(hipStreamSynchronize(s));
    if (hp[4] != 0.0) throw Error(DBQ_EBREAKDOWN, "Ritz eigensolver did not converge");
    lam_re = th_h[0].x - 1.0;
    lam_im = th_h[0].y;
    res = hp[3];
    if (debug)
      std::fprintf(stderr, "[dbq] kappa_c cycle: mv %lld lambda %.10f%+.10fi resid %.3e\n",
                   (long long)ar.mv, lam_re, lam_im, res);
    if (res <= tol * std::hypot(th_h[0].x, th_h[0].y) || ar.mv >= max_mv) break;
    ar.restart(k);
    j0 = k;
  }
  timer_collect(c);
  if (nritz > 0) {
    // the final cycle's Ritz values of largest real part (of I + H, sorted by real part)
    double2* th_h = (double2*)(hp + 64);
    DBQ_HIP(hipMemcpyAsync(th_h, ar.theta, sizeof(double2) * nritz, hipMemcpyDeviceToHost, s));
    DBQ_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nritz; ++i) {
      ritz[2 * i] = th_h[i].x - 1.0;
      ritz[2 * i + 1] = th_h[i].y;
    }
  }
  lambda[0] = lam_re;
  lambda[1] = lam_im;
  *resid = res;
  *kappa_c = 1.0 / lam_re;
  return (res <= tol * std::hypot(lam_re + 1.0, lam_im)) ? DBQ_OK : DBQ_NOT_CONVERGED;
}

// ============================================================================ MR projection
int mr_project(dbq_ctx* c, const dbq_operator* o, const void* Q, int nq, const void* B, void* X0,
               int nrhs, double* rn) {
  check_op(o);
  DBQ_CHECK(Q && B && X0 && rn, "null argument");
  DBQ_CHECK(nq >= 1 && nq <= 32, "nq must be in 1..32");
  DBQ_CHECK(nrhs >= 1, "nrhs must be >= 1");
  hipStream_t s = c->stream;
  WsScope ws(c);
  Op op = make_op(c, ws, o, true, false);
  const long long n = op.n(), V = op.sites();
  double2* b64 = ws.get<double2>(size_t(nrhs) * n);
  double2* x64 = ws.get<double2>(size_t(nrhs) * n);
  double2* r64 = ws.get<double2>(size_t(nrhs) * n);
  double2* Qp = ws.get<double2>(size_t(nrhs) * nq * n);
  double2* W = ws.get<double2>(size_t(nrhs) * nq * n);
  double2* bodd = nullptr;
  if (op.schur) {
    // projection on the reduced system of the new operator: bhat, x0_e and the even parts of Q
    double2* bfull = ws.get<double2>(size_t(nrhs) * op.nfull());
    bodd = ws.get<double2>(size_t(nrhs) * n);
    pack_spinor_f64(s, op.g, B, bfull, nrhs);
    schur_rhs(c, ws, op, bfull, b64, bodd, nrhs, 0);
    pack_even_f64(c, ws, op, X0, x64, nrhs);
    pack_even_f64(c, ws, op, Q, Qp, nrhs * nq);
  } else {
    pack_spinor_f64(s, op.g, B, b64, nrhs);
    pack_spinor_f64(s, op.g, X0, x64, nrhs);
    pack_spinor_f64(s, op.g, Q, Qp, nrhs * nq);
  }
  // r0 = b - A x0, W = A Q
  const DsBatch bx = make_batch({DsSpec{&op, false, x64, r64, nullptr, nrhs, 0}});
  run_dslash(c, false, bx, 0, EPI_NONE, nullptr, nullptr);
  sub_f64(s, b64, r64, r64, size_t(nrhs) * n);
  const DsBatch bq = make_batch({DsSpec{&op, false, Qp, W, nullptr, nrhs * nq, 0}});
  run_dslash(c, false, bq, 0, EPI_NONE, nullptr, nullptr);
  const size_t gw = gram_work_elems(n, nq, 1);
  double* gwork = ws.get<double>(gw);
  const size_t nw = norm_work(n, nrhs);
  double* nwork = ws.get<double>(nw);
  double2* h1 = ws.get<double2>(nq);
  double2* h2 = ws.get<double2>(nq);
  double2* R = ws.get<double2>(size_t(nq) * nq);
  double2* z = ws.get<double2>(nq);
  double* nrm = ws.get<double>(2 * nrhs + 2);
  norm2_f64(s, r64, n, nrhs, n, nrm, nwork, nw);
  for (int j = 0; j < nrhs; ++j) {
    double2* Wj = W + size_t(j) * nq * n;
    const double2* Qj = Qp + size_t(j) * nq * n;
    double2* rj = r64 + size_t(j) * n;
    zero_f64(s, R, size_t(nq) * nq);
    // W = Qw R (classical Gram-Schmidt twice)
    for (int q = 0; q < nq; ++q) {
      double2* w = Wj + size_t(q) * n;
      if (q > 0) {
        gram_f64(s, Wj, n, q, w, n, 1, n, V, 0, h1, gwork, gw);
        combine_f64(s, Wj, n, q, h1, q, w, n, 1, n, V, 0, -1);
        gram_f64(s, Wj, n, q, w, n, 1, n, V, 0, h2, gwork, gw);
        combine_f64(s, Wj, n, q, h2, q, w, n, 1, n, V, 0, -1);
      }
      norm2_f64(s, w, n, 1, n, nrm + 2 * nrhs, nwork, nw);
      write_col_f64(s, R, nq, q, q, h1, h2, nrm + 2 * nrhs, q);
      scale_f64(s, w, w, n, nrm + 2 * nrhs);
    }
    // z = Qw^H r0, d = R^{-1} z, x += Q d, r = r0 - Qw z
    gram_f64(s, Wj, n, nq, rj, n, 1, n, V, 0, z, gwork, gw);
    combine_f64(s, Wj, n, nq, z, nq, rj, n, 1, n, V, 0, -1);
    dense_trsolve_upper(s, R, nq, nq, z, 1, nq);
    combine_f64(s, Qj, n, nq, z, nq, x64 + size_t(j) * n, n, 1, n, V, 0, 1);
  }
  norm2_f64(s, r64, n, nrhs, n, nrm + nrhs, nwork, nw);
  if (op.schur) schur_solution(c, ws, op, x64, bodd, X0, nrhs, 0);
  else unpack_spinor_f64(s, op.g, x64, X0, nrhs);
  double* hp = (double*)pinned_get(c, sizeof(double) * 2 * nrhs);
  DBQ_HIP(hipMemcpyAsync(hp, nrm, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
  DBQ_HIP(hipStreamSynchronize(s));
  timer_collect(c);
  for (int j = 0; j < nrhs; ++j) {
    rn[2 * j] = std::sqrt(hp[j]);
    rn[2 * j + 1] = std::sqrt(hp[nrhs + j]);
  }
  return DBQ_OK;
}

// ============================================================================ GMRES(m)-Proj(k)
// The comparison method of Sec. 1 and Sec. 3 for later right-hand sides: a minimal-residual
// projection over the right eigenvectors V from GMRES-DR (d = argmin ||r - A V d||, x += V d; W = A V
// factorised once as Qw R by classical Gram-Schmidt twice, so a projection is r -= Qw Qw^H r and
// x += V R^{-1} Qw^H r, no products) alternating with cycles of GMRES(m) from the current r.
// FP64, right-hand sides one after another.
int gmres_proj(dbq_ctx* c, const dbq_operator* o, const void* Vin, int k, const void* B, void* X,
               int nrhs, int m, double tol, int64_t max_mv, dbq_stats* st) {
  const double t0 = now_s();
  check_op(o);
  DBQ_CHECK(B && X && st, "null argument");
  DBQ_CHECK(k >= 0 && k <= 128, "k must be in 0..128");
  DBQ_CHECK(k == 0 || Vin, "null eigenvectors");
  DBQ_CHECK(m >= 2 && m <= 128, "m must be in 2..128");
  DBQ_CHECK(nrhs >= 1, "nrhs must be >= 1");
  DBQ_CHECK(tol > 0 && std::isfinite(tol), "tol must be positive");
  DBQ_CHECK(max_mv >= 1, "max_mv must be >= 1");
  hipStream_t s = c->stream;
  WsScope ws(c);
  Op op = make_op(c, ws, o, true, false);
  const long long n = op.n(), Vs = op.sites();
  double2* b64 = ws.get<double2>(size_t(nrhs) * n);
  double2* x64 = ws.get<double2>(size_t(nrhs) * n);
  double2* bodd = nullptr;
  const size_t nwf = norm_work(op.nfull(), nrhs);
  double* wf = ws.get<double>(nwf);
  double* dn = ws.get<double>(2 * nrhs + 8);
  if (op.schur) {
    double2* bfull = ws.get<double2>(size_t(nrhs) * op.nfull());
    bodd = ws.get<double2>(size_t(nrhs) * n);
    pack_spinor_f64(s, op.g, B, bfull, nrhs);
    norm2_f64(s, bfull, op.nfull(), nrhs, op.nfull(), dn, wf, nwf);
    schur_rhs(c, ws, op, bfull, b64, bodd, nrhs, 0);
    pack_even_f64(c, ws, op, X, x64, nrhs);
  } else {
    pack_spinor_f64(s, op.g, B, b64, nrhs);
    pack_spinor_f64(s, op.g, X, x64, nrhs);
    norm2_f64(s, b64, n, nrhs, n, dn, wf, nwf);
  }
  norm2_f64(s, x64, n, nrhs, n, dn + nrhs, wf, nwf);
  double* hp = (double*)pinned_get(c, sizeof(double) * (2 * nrhs + 16));
  DBQ_HIP(hipMemcpyAsync(hp, dn, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
  DBQ_HIP(hipStreamSynchronize(s));
  std::vector<double> bn(nrhs), xn(nrhs);
  for (int j = 0; j < nrhs; ++j) {
    bn[j] = std::sqrt(hp[j]);
    xn[j] = hp[nrhs + j];
    DBQ_CHECK(std::isfinite(hp[j]) && std::isfinite(hp[nrhs + j]), "non-finite b or x0");
  }
  Arnoldi ar(c, ws, &op, m, 1);
  const size_t gw = gram_work_elems(n, std::max(k, 1), 1);
  double* gwork = ws.get<double>(gw);
  // ---- setup: W = A V (k products), W = Qw R
  double2 *Vp = nullptr, *Qw = nullptr, *R = nullptr, *z = nullptr, *h1 = nullptr, *h2 = nullptr;
  if (k > 0) {
    Vp = ws.get<double2>(size_t(k) * n);
    Qw = ws.get<double2>(size_t(k) * n);
    R = ws.get<double2>(size_t(k) * k);
    z = ws.get<double2>(k);
    h1 = ws.get<double2>(k);
    h2 = ws.get<double2>(k);
    if (op.schur) pack_even_f64(c, ws, op, Vin, Vp, k);
    else pack_spinor_f64(s, op.g, Vin, Vp, k);
    const DsBatch bw = make_batch({DsSpec{&op, false, Vp, Qw, nullptr, k, 0}});
    run_dslash(c, false, bw, 0, EPI_NONE, nullptr, nullptr);
    zero_f64(s, R, size_t(k) * k);
    double* nq = dn + 2 * nrhs;
    for (int q = 0; q < k; ++q) {
      double2* w = Qw + size_t(q) * n;
      if (q > 0) {
        gram_f64(s, Qw, n, q, w, n, 1, n, Vs, 0, h1, gwork, gw);
        combine_f64(s, Qw, n, q, h1, q, w, n, 1, n, Vs, 0, -1);
        gram_f64(s, Qw, n, q, w, n, 1, n, Vs, 0, h2, gwork, gw);
        combine_f64(s, Qw, n, q, h2, q, w, n, 1, n, Vs, 0, -1);
      }
      norm2_f64(s, w, n, 1, n, nq, ar.nwork, ar.nw);
      write_col_f64(s, R, k, q, q, h1, h2, nq, q);
      scale_f64(s, w, w, n, nq);
    }
  }
  double2* r = ws.get<double2>(n);
  double* rn2 = dn + 2 * nrhs + 1;
  for (int j = 0; j < nrhs; ++j) {
    double2* bj = b64 + size_t(j) * n;
    double2* xj = x64 + size_t(j) * n;
    int64_t mv = 0;
    int cycles = 0;
    if (xn[j] > 0) {
      const DsBatch bx = make_batch({DsSpec{&op, false, xj, r, nullptr, 1, 0}});
      run_dslash(c, false, bx, 0, EPI_NONE, nullptr, nullptr);
      sub_f64(s, bj, r, r, n);
      mv += 1;
    } else {
      copy_f64(s, bj, r, n);
    }
    bool conv = false;
    double rel = 0.0;
    if (bn[j] == 0.0) {
      zero_f64(s, xj, n);
      conv = true;
    }
    while (!conv) {
      if (k > 0) {
        gram_f64(s, Qw, n, k, r, n, 1, n, Vs, 0, z, gwork, gw);
        combine_f64(s, Qw, n, k, z, k, r, n, 1, n, Vs, 0, -1);
        dense_trsolve_upper(s, R, k, k, z, 1, k);
        combine_f64(s, Vp, n, k, z, k, xj, n, 1, n, Vs, 0, 1);
      }
      norm2_f64(s, r, n, 1, n, rn2, ar.nwork, ar.nw);
      DBQ_HIP(hipMemcpyAsync(hp, rn2, sizeof(double), hipMemcpyDeviceToHost, s));
      DBQ_HIP(hipStreamSynchronize(s));
      rel = std::sqrt(hp[0]) / bn[j];
      if (!std::isfinite(rel)) throw Error(DBQ_EBREAKDOWN, "GMRES-Proj residual is not finite");
      if (rel <= tol) {
        conv = true;
        break;
      }
      if (mv >= max_mv) break;
      // one GMRES(m) cycle from r
      scale_f64(s, r, ar.col(0), n, rn2);
      set_e1_f64(s, ar.cv, m + 1, rn2);
      ar.extend(0);
      mv += m;
      ar.cycle_end(1, 3, tol * bn[j]);
      combine_f64(s, ar.Vb, n, m, ar.d, m, xj, n, 1, n, Vs, 0, 1);
      combine_f64(s, ar.Vb, n, m + 1, ar.cnew, m + 1, r, n, 1, n, Vs, 0, 0);
      ++cycles;
      DBQ_HIP(hipMemcpyAsync(hp, ar.info, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
      DBQ_HIP(hipStreamSynchronize(s));
      rel = hp[0] / bn[j];
      if (!std::isfinite(rel)) throw Error(DBQ_EBREAKDOWN, "GMRES-Proj residual is not finite");
      if (rel <= tol) {
        conv = true;
        break;
      }
      if (mv >= max_mv) break;
    }
    // true residual for the statistics (not charged)
    const DsBatch bx = make_batch({DsSpec{&op, false, xj, r, nullptr, 1, 0}});
    run_dslash(c, false, bx, 0, EPI_NONE, nullptr, nullptr);
    sub_f64(s, bj, r, r, n);
    norm2_f64(s, r, n, 1, n, rn2, ar.nwork, ar.nw);
    DBQ_HIP(hipMemcpyAsync(hp, rn2, sizeof(double), hipMemcpyDeviceToHost, s));
    DBQ_HIP(hipStreamSynchronize(s));
    dbq_stats& o2 = st[j];
    o2.matvecs = mv;
    o2.iterations = cycles;
    o2.restarts = 0;
    o2.reliable_updates = 0;
    o2.rel_true_resid = bn[j] > 0 ? std::sqrt(hp[0]) / bn[j] : 0.0;
    o2.status = conv ? DBQ_OK : DBQ_NOT_CONVERGED;
    o2.fp64_continued = 0;
  }
  if (op.schur) schur_solution(c, ws, op, x64, bodd, X, nrhs, 0);
  else unpack_spinor_f64(s, op.g, x64, X, nrhs);
  DBQ_HIP(hipStreamSynchronize(s));
  timer_collect(c);
  const double secs = now_s() - t0;
  int worst = DBQ_OK;
  for (int j = 0; j < nrhs; ++j) {
    st[j].seconds = secs;
    worst = std::max(worst, int(st[j].status));
  }
  return worst;
}

// ============================================================================ link force
void force(dbq_ctx* c, const dbq_operator* o, const void* lambda, const void* x, int nrhs,
           int kind, void* F) {
  check_op(o);
  DBQ_CHECK(lambda && x && F, "null argument");
  DBQ_CHECK(nrhs >= 1, "nrhs must be >= 1");
  DBQ_CHECK(kind == 0 || kind == 1, "kind must be 0 or 1");
  DBQ_CHECK(o->schur == 0, "link_force needs the full operator (schur = 0)");
  const Geom g = make_geom(o->L);
  launch_link_force(c->stream, g, o->links, o->kappa, lambda, x, nrhs, kind, F);
}

}  // namespace dbq
