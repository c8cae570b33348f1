// extern "C" entry points: argument checks, error capture, no exceptions across the boundary.
#include <cstring>
#include <string>

#include "ctx.h"
#include "kernels.h"
#include "solvers.h"

using dbq::Error;

namespace {

template <typename F>
int guarded(dbq_ctx* c, F&& f) {
  if (!c) return DBQ_EINVAL;
  try {
    c->err.clear();
    return f();
  } catch (const Error& e) {
    c->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return DBQ_ENOMEM;
  } catch (const std::exception& e) {
    c->err = e.what();
    return DBQ_EHIP;
  }
}

}  // namespace

extern "C" {

int dbq_create(dbq_ctx** out, void* stream) {
  if (!out) return DBQ_EINVAL;
  *out = nullptr;
  dbq_ctx* c = new (std::nothrow) dbq_ctx();
  if (!c) return DBQ_ENOMEM;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess ||
      hipMalloc(&c->acct, sizeof(unsigned long long) * 32) != hipSuccess ||
      hipMemset(c->acct, 0, sizeof(unsigned long long) * 32) != hipSuccess) {
    (void)hipGetLastError();
    if (c->acct) (void)hipFree(c->acct);
    delete c;
    return DBQ_EHIP;
  }
  // set-up of the allocation-free apply: this device's address of its static scratch array
  // (a failure here leaves it null; that entry point then retries and reports the error)
  try {
    c->scratch = dbq::noalloc_scratch(c->device);
  } catch (const Error&) {
    (void)hipGetLastError();
    c->scratch = nullptr;
  }
  *out = c;
  return DBQ_OK;
}

int dbq_destroy(dbq_ctx* c) {
  if (!c) return DBQ_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  for (auto& b : c->pool) (void)hipFree(b.p);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->acct) (void)hipFree(c->acct);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto& t : c->timers) {
    for (auto& pr : t.ev) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    for (auto e : t.spare) (void)hipEventDestroy(e);
  }
  delete c;
  return DBQ_OK;
}

const char* dbq_last_error(const dbq_ctx* c) { return c ? c->err.c_str() : "null context"; }

int dbq_set_stream(dbq_ctx* c, void* stream) {
  return guarded(c, [&]() {
    c->stream = (hipStream_t)stream;
    return DBQ_OK;
  });
}

int dbq_geometry(dbq_ctx* c, const int32_t L[4], int32_t* lex_of_eo, int32_t* nbr) {
  return guarded(c, [&]() {
    DBQ_CHECK(L && lex_of_eo && nbr, "null argument");
    for (int i = 0; i < 4; ++i) DBQ_CHECK(L[i] >= 2 && L[i] % 2 == 0, "extents must be even, >= 2");
    const dbq::Geom g = dbq::make_geom(L);
    dbq::launch_geometry(c->stream, g, lex_of_eo, nbr);
    return DBQ_OK;
  });
}

int dbq_site_tile(const int32_t L[4], int32_t* T) {
  if (!L || !T) return DBQ_EINVAL;
  for (int i = 0; i < 4; ++i)
    if (L[i] < 2 || L[i] % 2) return DBQ_EINVAL;
  const dbq::Geom g = dbq::make_geom(L);
  for (int i = 0; i < 4; ++i) T[i] = g.T[i];
  return DBQ_OK;
}

int dbq_geometry_host(const int32_t L[4], int32_t* lex_of_eo, int32_t* nbr) {
  if (!L || !lex_of_eo || !nbr) return DBQ_EINVAL;
  for (int i = 0; i < 4; ++i)
    if (L[i] < 2 || L[i] % 2) return DBQ_EINVAL;
  const dbq::Geom g = dbq::make_geom(L);
  for (int s = 0; s < g.V; ++s) {
    int c[4], p;
    dbq::eo_coords(g, s, c, p);
    lex_of_eo[s] = dbq::lex_index(g, c);
    nbr[0 * g.V + s] = dbq::eo_neighbour<0, +1>(g, c);
    nbr[1 * g.V + s] = dbq::eo_neighbour<0, -1>(g, c);
    nbr[2 * g.V + s] = dbq::eo_neighbour<1, +1>(g, c);
    nbr[3 * g.V + s] = dbq::eo_neighbour<1, -1>(g, c);
    nbr[4 * g.V + s] = dbq::eo_neighbour<2, +1>(g, c);
    nbr[5 * g.V + s] = dbq::eo_neighbour<2, -1>(g, c);
    nbr[6 * g.V + s] = dbq::eo_neighbour<3, +1>(g, c);
    nbr[7 * g.V + s] = dbq::eo_neighbour<3, -1>(g, c);
  }
  return DBQ_OK;
}

int dbq_tile_schedule_host(const int32_t L[4], int32_t nchunks, int32_t order, int32_t* tile,
                           int32_t* chunk) {
  if (!L || !tile || !chunk || nchunks < 1 || order < 0 || order > 3) return DBQ_EINVAL;
  for (int i = 0; i < 4; ++i)
    if (L[i] < 2 || L[i] % 2) return DBQ_EINVAL;
  const dbq::Geom g = dbq::make_geom(L);
  const int ntiles = g.NT[0] * g.NT[1] * g.NT[2] * g.NT[3];
  for (int loc = 0; loc < ntiles * nchunks; ++loc) {
    int tc[4];
    dbq::tile_of_block(g, loc, nchunks, order, tc, tile[loc], chunk[loc]);
  }
  return DBQ_OK;
}

int dbq_stream_probe(dbq_ctx* c, const void* src, void* dst, int64_t bytes, int32_t kind,
                     int32_t reps, double* ms) {
  return guarded(c, [&]() {
    DBQ_CHECK(ms, "null argument");
    *ms = dbq::stream_probe(c, src, dst, bytes, kind, reps);
    return DBQ_OK;
  });
}

int wilson_apply(dbq_ctx* c, const dbq_operator* op, const void* in, void* out, int32_t nrhs,
                 int32_t dagger, int32_t prec) {
  return guarded(c, [&]() {
    dbq::apply_operator(c, op, in, out, nrhs, dagger ? 1 : 0, prec);
    return DBQ_OK;
  });
}

int wilson_apply_noalloc(dbq_ctx* c, const dbq_operator* op, const void* in, void* out,
                         int32_t nrhs, int32_t dagger, int32_t prec) {
  return guarded(c, [&]() {
    dbq::apply_operator_noalloc(c, op, in, out, nrhs, dagger ? 1 : 0, prec);
    return DBQ_OK;
  });
}

int gmresdr_first_rhs(dbq_ctx* c, const dbq_operator* op, const void* b, void* x, int32_t m,
                      int32_t k, double tol, int64_t max_mv, void* V_out, double* theta,
                      int32_t* k_out, dbq_stats* stats) {
  return guarded(c, [&]() { return dbq::gmresdr(c, op, b, x, m, k, tol, max_mv, V_out, theta, k_out, stats); });
}

int dbicgstab_solve(dbq_ctx* c, const dbq_operator* ops, int32_t nops, const void* const* V,
                    const int32_t* k, const void* const* B, void* const* X, const int32_t* nrhs,
                    double tol, int64_t max_mv, int32_t prec, int32_t dagger, dbq_stats* per_rhs) {
  return guarded(c, [&]() {
    return dbq::dbicgstab(c, ops, nops, V, k, B, X, nrhs, tol, max_mv, prec, dagger ? 1 : 0, per_rhs);
  });
}

int project_shifts(dbq_ctx* c, const dbq_operator* op_new, const void* Q, int32_t nq,
                   const void* B, void* X0, int32_t nrhs, double* rnorm_before_after) {
  return guarded(c, [&]() { return dbq::mr_project(c, op_new, Q, nq, B, X0, nrhs, rnorm_before_after); });
}

int gmres_proj_solve(dbq_ctx* c, const dbq_operator* op, const void* V, int32_t k, const void* B,
                     void* X, int32_t nrhs, int32_t m, double tol, int64_t max_mv,
                     dbq_stats* per_rhs) {
  return guarded(c, [&]() {
    return dbq::gmres_proj(c, op, V, k, B, X, nrhs, m, tol, max_mv, per_rhs);
  });
}

int link_force(dbq_ctx* c, const dbq_operator* op, const void* lambda, const void* x,
               int32_t nrhs, int32_t kind, void* F) {
  return guarded(c, [&]() {
    dbq::force(c, op, lambda, x, nrhs, kind, F);
    return DBQ_OK;
  });
}

int kappa_critical(dbq_ctx* c, const int32_t L[4], const void* links, int32_t m, int32_t k,
                   double tol, int64_t max_mv, double* kappa_c, double* lambda, double* resid) {
  return guarded(c, [&]() {
    return dbq::kappa_crit(c, L, links, m, k, tol, max_mv, kappa_c, lambda, resid, 0, nullptr);
  });
}

int kappa_critical_ritz(dbq_ctx* c, const int32_t L[4], const void* links, int32_t m, int32_t k,
                        double tol, int64_t max_mv, double* kappa_c, double* lambda, double* resid,
                        int32_t nritz, double* ritz) {
  return guarded(c, [&]() {
    return dbq::kappa_crit(c, L, links, m, k, tol, max_mv, kappa_c, lambda, resid, nritz, ritz);
  });
}

int dbq_set_timing(dbq_ctx* c, int32_t on) {
  return guarded(c, [&]() {
    DBQ_CHECK(on >= 0, "timing: on must be >= 0");
    c->timing = on != 0;
    c->timing_sample = on > 1 ? on : 1;
    return DBQ_OK;
  });
}

int dbq_kernel_time(dbq_ctx* c, int32_t kind, double* total_ms, int64_t* launches,
                    double* algorithmic_bytes) {
  return guarded(c, [&]() {
    DBQ_CHECK(kind >= 0 && kind <= 2, "kind must be 0, 1 or 2");
    DBQ_CHECK(total_ms && launches && algorithmic_bytes, "null argument");
    dbq::timer_collect(c);
    *total_ms = c->timers[kind].ms;
    *launches = c->timers[kind].n;
    *algorithmic_bytes = c->timers[kind].bytes;
    return DBQ_OK;
  });
}

int dbq_reset_timing(dbq_ctx* c) {
  return guarded(c, [&]() {
    dbq::timer_collect(c);
    for (auto& t : c->timers) {
      t.ms = 0;
      t.n = 0;
      t.bytes = 0;
      t.calls = 0;
    }
    return DBQ_OK;
  });
}

const char* dbq_version(void) { return "dbq 0.1 (gfx950)"; }

}  // extern "C"
