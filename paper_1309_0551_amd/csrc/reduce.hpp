// reduce.hpp -- deterministic FP64 reductions and the solver's scalar steps.
//
// Each workgroup reduces its values (wavefront butterfly over 64 lanes, then
// the 4 wave sums in LDS) into one partial per workgroup, written with a plain
// store; a later kernel (the one-workgroup finalize, or every workgroup of the
// CG update for alpha) sums the partials in index order. The order is fixed,
// so repeated runs give bit-identical scalars.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace lgt {

// sum over the workgroup; the value is valid in thread 0
__device__ __forceinline__ double block_sum(double v, double *lds)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (int)(blockDim.x >> 6); // waves of this workgroup (<= kBS / 64)
        for (int i = 0; i < nw; i++) s += lds[i];
    }
    __syncthreads();
    return s;
}

// sum over the workgroup in block_sum's order, returned to every thread
__device__ __forceinline__ double block_sum_all(double v, double *lds)
{
    const double s = block_sum(v, lds);
    if (threadIdx.x == 0) lds[0] = s;
    __syncthreads();
    const double r = lds[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ bool gate_open(int gate, const CgState *st)
{
    if (gate == GATE_NONE) return true;
    const int s = st->state;
    if (gate == GATE_ITER) return s == ST_RUN;
    return s == ST_INIT || s == ST_INNER || (s == ST_RUN && st->ru_fixed);
}

// The scalar step that follows a reduction (one thread, after all partial sums
// of the reducing kernel or phase have been added in a fixed order).
__device__ inline void finalize(int fin, CgState *st, double sum)
{
    switch (fin) {
    case FIN_ALPHA: // alpha = rho / <p, A p>
        st->pAp = sum;
        st->pend = 0; // the previous alpha p went into x in k_xpay
        if (!(sum > 0.0) || !isfinite(sum)) st->state = ST_FAIL;
        else st->alpha = st->rho / sum;
        break;
    case FIN_UPDATE: { // rho' = |r|^2, beta = rho'/rho
        st->iter += 1;
        st->pend = 1; // x += alpha p still to do
        st->pcur ^= 1; // double-buffered p: the p of this iteration is current
        if (!isfinite(sum)) {
            st->state = ST_FAIL;
            break;
        }
        st->beta = sum / st->rho;
        st->rho_prev = st->rho;
        st->rho = sum;
        if (sum <= st->stop_inner) st->state = ST_INNER;
        else if (st->iter >= st->max_iter) st->state = ST_MAXIT;
        break;
    }
    case FIN_RU: { // sum = |b - A x|^2 in FP64
        st->pend = 0; // applied by k_x_pending before the residual
        const bool init = st->state == ST_INIT;
        if (!init) st->updates += 1;
        st->last_true = sum;
        if (!isfinite(sum)) {
            st->state = ST_FAIL;
        } else if (sum <= st->stop_outer) {
            st->state = ST_DONE;
        } else {
            if (init || st->scheme == SCH_REFINE) {
                st->beta = 0.0; // restart: p = r
                if (st->scheme == SCH_REFINE) st->stop_inner = st->inner2 * sum;
            } else {
                st->beta = sum / st->rho_prev; // reliable update keeps p
            }
            st->rho = sum;
            st->state = st->iter >= st->max_iter ? ST_MAXIT : ST_RUN;
        }
        break;
    }
    case FIN_INIT: // sum = |b|^2; the tolerance was stored in stop_outer
        st->bnorm2 = sum;
        st->stop_outer = st->stop_outer * sum;
        if (st->scheme != SCH_REFINE) st->stop_inner = st->inner2 * sum;
        break;
    case FIN_FINAL:
        st->pend = 0;
        st->last_true = sum;
        break;
    default:
        break;
    }
}

// Write this workgroup's partial sum (logical workgroup index `blk`). The sum
// over workgroups and the scalar step run in k_finalize, launched next on the
// same stream: the kernel boundary makes the partials visible to it, which is
// far cheaper than a device-scope fence in every workgroup (on a multi-XCD
// part such a fence writes back the workgroup's whole L2).
__device__ __forceinline__ void write_partial(double v, double *partials, int blk)
{
    __shared__ double lds[kBS / 64];
    const double s = block_sum(v, lds);
    if (threadIdx.x == 0) partials[blk] = s;
}

} // namespace lgt
