// Solver drivers behind the C ABI (see dbq.h for the contract of each call).
#pragma once

#include "ctx.h"

namespace dbq {

void apply_operator(dbq_ctx* c, const dbq_operator* o, const void* in, void* out, int nrhs,
                    int dagger, int prec);
int dbicgstab(dbq_ctx* c, const dbq_operator* ops, int nops, const void* const* V,
              const int32_t* k, const void* const* B, void* const* X, const int32_t* nrhs,
              double tol, int64_t max_mv, int prec, int dagger, dbq_stats* st);
int gmresdr(dbq_ctx* c, const dbq_operator* o, const void* b, void* x, int m, int k, double tol,
            int64_t max_mv, void* Vout, double* theta, int32_t* k_out, dbq_stats* st);
int kappa_crit(dbq_ctx* c, const int32_t L[4], const void* links, int m, int k, double tol,
               int64_t max_mv, double* kappa_c, double* lambda, double* resid, int nritz,
               double* ritz);
int mr_project(dbq_ctx* c, const dbq_operator* o, const void* Q, int nq, const void* B, void* X0,
               int nrhs, double* rn);
int gmres_proj(dbq_ctx* c, const dbq_operator* o, const void* V, int k, const void* B, void* X,
               int nrhs, int m, double tol, int64_t max_mv, dbq_stats* st);
void force(dbq_ctx* c, const dbq_operator* o, const void* lambda, const void* x, int nrhs,
           int kind, void* F);
// average milliseconds of one streaming probe launch (probe.hip)
double stream_probe(dbq_ctx* c, const void* src, void* dst, long long bytes, int kind, int reps);
// the operator apply on the static scratch array of noalloc.hip (no device allocation)
void apply_operator_noalloc(dbq_ctx* c, const dbq_operator* o, const void* in, void* out,
                            int nrhs, int dagger, int prec);
// device address of the current device's scratch array (looked up once per device)
void* noalloc_scratch(int device);
size_t noalloc_scratch_bytes();

}  // namespace dbq
