// Launch interface of the slot kernels (batch.hip) used by the serving
// sessions (api.hip).  All launches are asynchronous on `st`.
#pragma once

#include "kernels.h"

namespace ebicg {

// One column (slot) of a batch, for serving sessions: r[:, col] = src and
// e[:, col] = 0; rhat, p = r on column col with rho_0 (history index col) and
// the column's state (target tol_abs, maxiter); x += e[:, col]; and the
// rebase at the end of a chunk of jl iterations (the next chunk counts from 1).
template <typename S>
void launch_slot_load(S *r, S *e, const double2 *src, size_t N, int kc, int col, hipStream_t st);
template <typename S>
void launch_slot_init(S *rhat, S *p, const S *r, size_t N, int kc, int col, double tol_abs, int maxiter,
                      KrylovState *K, KrylovHistory h, const RedScratch &rs, hipStream_t st);
template <typename S>
void launch_slot_add(double2 *x, const S *e, size_t N, int kc, int col, hipStream_t st);
void launch_batch_rebase(KrylovState *K, KrylovHistory h, int kc, int jl, hipStream_t st);

}  // namespace ebicg
