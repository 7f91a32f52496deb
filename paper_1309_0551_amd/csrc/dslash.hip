// dslash.hip -- the staggered Dslash and the packing / geometry kernels.
//
// One thread per output site x of parity `par` (V/2 threads):
//   out(x) = sum_mu eta_mu(x) [ s+ U_mu(x) in(x+mu) - s- U_mu(x-mu)^dag in(x-mu) ]
// i.e. the forward half (Table 1: mult_su3_mat_vec_sum_4dir), four adjoint
// products (mult_adj_su3_mat_vec, Eqs (1.1)-(2.3)) and their subtraction
// (sub_four_su3_vecs): 570 flop/site. The forward link lives at x in the
// plane set of parity `par`; the backward link U_mu(x-mu) at the neighbour, in
// the plane set of the other parity. Every link is read exactly once per call
// and the kernel is bound by HBM bandwidth: link loads are marked
// non-temporal so they do not evict the reused input vector from L2 (or cached,
// for fields that the Infinity Cache holds between calls), and so are the
// output stores, which no thread of the kernel reads back: write-allocating
// them in L2 would evict input lines that neighbouring sites still gather.
#include <hip/hip_ext.h>

#include "fields.hpp"
#include "kernels.hpp"
#include "reduce.hpp"

namespace lgt {

// HPI = hops whose loads are issued together. The whole unrolled body is one
// basic block in which the backend hoists all 96 loads of the FP64 kernel
// (256 VGPRs, one wave per SIMD); a runtime loop over directions (HPI = 2) or
// over single hops (HPI = 1) bounds the loads in flight per thread and lets
// more waves share each SIMD. HPI = 0 is the improved operator: a runtime loop
// over the 8 hop pairs (one-link and Naik three-link per direction), 16 links
// per site from two link fields of the same format.
//
// HPI = 4 is the direction loop of HPI = 2 with the input vector staged in LDS:
// a workgroup's bs output sites (64, 128 or 256) are consecutive cb indices,
// x rows (Lx/2 sites each) of a few y values, so their x and y neighbours of
// the other parity lie in the cb range [first - Lx/2, last + Lx/2]. The
// workgroup copies that range (bs + Lx sites) into LDS once with coalesced
// loads; every hop whose neighbour falls in it reads LDS, the others (z and t,
// and wrapped x/y hops) read global memory.
extern __shared__ __align__(16) unsigned char lds_dyn[];

// sites of the staged cb range of a workgroup of bs sites
__host__ __device__ __forceinline__ int staged_sites(const Geom &g, int bs) { return bs + 2 * g.hx; }

template <class LF, int EPI, int HPI, bool NTL>
__global__ __launch_bounds__(kBS) void k_dslash(DslashArgs a)
{
    using T = typename LF::real;
    using VF = VecFmt<T>;
    using S2 = typename VF::store_t;
    if (!gate_open(a.gate, a.st)) return;
    const int bs = (int)blockDim.x; // 64, 128 or 256 sites per workgroup
    const int blk = xcd_block(blockIdx.x, a.l.nblk_pad);
    const int cb = blk * bs + threadIdx.x;
    const size_t Vh = (size_t)a.g.Vh;
    [[maybe_unused]] const int s0 = blk * bs - a.g.hx, ns = staged_sites(a.g, bs);
    [[maybe_unused]] S2 *lds = (S2 *)lds_dyn; // [3][ns]
    // EPI_PAPX: the gathered input is p' = r + beta p_old, formed here with the
    // same arithmetic as k_xpay (so the results do not depend on which runs)
    [[maybe_unused]] const void *pin = a.in;
    [[maybe_unused]] T beta = T(0);
    if constexpr (EPI == EPI_PAPX) {
        pin = a.st->pcur ? a.pb : a.in;
        beta = (T)a.st->beta;
    }
    auto load_in = [&](int n, cx<T> v[3]) __attribute__((always_inline)) {
        VF::template load<false>(pin, Vh, n, v);
        if constexpr (EPI == EPI_PAPX) {
            cx<T> rr[3];
            VF::template load<false>(a.rin, Vh, n, rr);
#pragma unroll
            for (int i = 0; i < 3; i++) {
                v[i].re = fma(beta, v[i].re, rr[i].re);
                v[i].im = fma(beta, v[i].im, rr[i].im);
            }
        }
    };
    if constexpr (HPI == 4) {
        for (int i = threadIdx.x; i < ns; i += bs) {
            const int n = s0 + i;
            if (n >= 0 && n < a.g.Vh) {
                if constexpr (EPI == EPI_PAPX) {
                    cx<T> v[3];
                    load_in(n, v);
#pragma unroll
                    for (int k = 0; k < 3; k++) lds[k * ns + i] = S2{v[k].re, v[k].im};
                } else {
#pragma unroll
                    for (int k = 0; k < 3; k++) lds[k * ns + i] = ((const S2 *)a.in)[k * Vh + n];
                }
            }
        }
        __syncthreads();
    }
    double part = 0.0;
    cx<T> acc[3];
    [[maybe_unused]] cx<T> pu[3], ru[3]; // EPI_UPD: p and r at this site, loaded before alpha
    if (cb < a.g.Vh) {
        int c[4];
        decode(a.g, a.par, cb, c);
#pragma unroll
        for (int i = 0; i < 3; i++) acc[i].re = acc[i].im = T(0);
        if constexpr (HPI == 0) {
#pragma unroll 1
            for (int k = 0; k < 8; k++) {
                const int mu = k >> 1;
                const bool naik = k & 1;
                const Hop h = naik ? hop3_rt(a.g, c, cb, mu) : hop_rt(a.g, c, cb, mu);
                const void *W = naik ? a.U3 : a.U;
                cx<T> u[9], v[3], w[9], z[3];
                LF::template load<NTL>(W, Vh, a.par * 4 + mu, cb, u);
                load_in(h.f, v);
                LF::template load<NTL>(W, Vh, (1 - a.par) * 4 + mu, h.b, w);
                load_in(h.b, z);
                negate_if(h.fneg, v);
                mv_add(u, v, acc);
                negate_if(h.bneg, z);
                amv_sub(w, z, acc);
            }
        } else if constexpr (HPI == 8) {
#pragma unroll
            for (int mu = 0; mu < 4; mu++) {
                cx<T> u[9], v[3];
                // forward hop: U_mu(x) in(x+mu)
                LF::template load<NTL>(a.U, Vh, a.par * 4 + mu, cb, u);
                load_in(nbr_fwd(a.g, c, cb, mu), v);
                negate_if(fwd_neg(a.g, c, mu), v);
                mv_add(u, v, acc);
                // backward hop: U_mu(x-mu)^dag in(x-mu)
                const int b = nbr_bwd(a.g, c, cb, mu);
                LF::template load<NTL>(a.U, Vh, (1 - a.par) * 4 + mu, b, u);
                load_in(b, v);
                negate_if(bwd_neg(a.g, c, mu), v);
                amv_sub(u, v, acc);
            }
        } else if constexpr (HPI == 4) {
            // a neighbour in the staged range (every x hop, y hops except across
            // the y wrap) is read from LDS, any other from global memory, through
            // one generic pointer so the two cases share the instruction stream
            const S2 *gin = (const S2 *)a.in;
            auto vsrc = [&](int n, size_t &stride) -> const S2 * {
                const unsigned j = (unsigned)(n - s0);
                const bool staged = j < (unsigned)ns;
                stride = staged ? (size_t)ns : Vh;
                return staged ? lds + j : gin + n;
            };
            // EPI_PAPX: a hop outside the staged range forms r + beta p itself
            auto fetch = [&](int n, cx<T> v[3]) __attribute__((always_inline)) {
                if constexpr (EPI == EPI_PAPX) {
                    const unsigned j = (unsigned)(n - s0);
                    if (j < (unsigned)ns) {
#pragma unroll
                        for (int k = 0; k < 3; k++) {
                            const S2 x = lds[k * ns + j];
                            v[k].re = x.x;
                            v[k].im = x.y;
                        }
                    } else {
                        load_in(n, v);
                    }
                } else {
                    size_t st;
                    const S2 *q = vsrc(n, st);
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        const S2 x = q[k * st];
                        v[k].re = x.x;
                        v[k].im = x.y;
                    }
                }
            };
#pragma unroll 1
            for (int mu = 0; mu < 4; mu++) {
                const Hop h = hop_rt(a.g, c, cb, mu);
                cx<T> u[9], v[3], w[9], z[3];
                LF::template load<NTL>(a.U, Vh, a.par * 4 + mu, cb, u);
                fetch(h.f, v);
                LF::template load<NTL>(a.U, Vh, (1 - a.par) * 4 + mu, h.b, w);
                fetch(h.b, z);
                negate_if(h.fneg, v);
                mv_add(u, v, acc);
                negate_if(h.bneg, z);
                amv_sub(w, z, acc);
            }
        } else if constexpr (HPI == 2) {
#pragma unroll 1
            for (int mu = 0; mu < 4; mu++) {
                const Hop h = hop_rt(a.g, c, cb, mu);
                cx<T> u[9], v[3], w[9], z[3];
                LF::template load<NTL>(a.U, Vh, a.par * 4 + mu, cb, u);
                load_in(h.f, v);
                LF::template load<NTL>(a.U, Vh, (1 - a.par) * 4 + mu, h.b, w);
                load_in(h.b, z);
                negate_if(h.fneg, v);
                mv_add(u, v, acc);
                negate_if(h.bneg, z);
                amv_sub(w, z, acc);
            }
        } else {
#pragma unroll 1
            for (int hop = 0; hop < 8; hop++) {
                const int mu = hop >> 1;
                const bool fwd = !(hop & 1);
                const Hop h = hop_rt(a.g, c, cb, mu);
                cx<T> u[9], v[3];
                LF::template load<NTL>(a.U, Vh, fwd ? a.par * 4 + mu : (1 - a.par) * 4 + mu, fwd ? cb : h.b, u);
                load_in(fwd ? h.f : h.b, v);
                negate_if(fwd ? h.fneg : h.bneg, v);
                if (fwd) mv_add(u, v, acc);
                else amv_sub(u, v, acc);
            }
        }
        if constexpr (EPI == EPI_UPD) {
            // double-buffered p: the new p is buffer 1 - pcur (pcur flips at the beta step)
            const void *pn = a.pb ? (a.st->pcur ? a.aux0 : a.pb) : a.aux0;
            VF::template load<false>(pn, Vh, cb, pu);
            VF::template load<false>(a.rw, Vh, cb, ru);
        }
    }
    [[maybe_unused]] double alpha64 = 0.0;
    if constexpr (EPI == EPI_UPD) {
        // alpha after the hops, so that this sum waits while the hops of other
        // workgroups run (every thread of the workgroup takes part; four
        // strided accumulators, so four loads are in flight: with one the
        // 32^4 solves took 1-3 % longer)
        if (a.nparts_in > 0) {
            __shared__ double red[kBS / 64];
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int i = threadIdx.x;
            for (; i + 3 * bs < a.nparts_in; i += 4 * bs) {
                s0 += a.parts_in[i];
                s1 += a.parts_in[i + bs];
                s2 += a.parts_in[i + 2 * bs];
                s3 += a.parts_in[i + 3 * bs];
            }
            for (; i < a.nparts_in; i += bs) s0 += a.parts_in[i];
            const double pAp = block_sum_all((s0 + s1) + (s2 + s3), red);
            const bool bad = !(pAp > 0.0) || !isfinite(pAp);
            alpha64 = a.st->rho / pAp;
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                // fields no other workgroup reads in this kernel
                a.st->pAp = pAp;
                a.st->pend = 0; // the previous alpha p went into x in k_xpay
                if (bad) a.st->state = ST_FAIL;
                else a.st->alpha = alpha64;
            }
            if (bad) return; // the whole workgroup; the beta step is gated off
        } else {
            alpha64 = a.st->alpha;
        }
    }
    if (cb < a.g.Vh) {
        if constexpr (EPI == EPI_PLAIN) {
            VF::template store<true>(a.out, Vh, cb, acc);
        } else if constexpr (EPI == EPI_PAP) {
            // out = D in ; partial m4 |p|^2 + |out|^2 (p at the same cb of the other parity)
            cx<T> p[3];
            VF::template load<false>(a.aux0, Vh, cb, p);
#pragma unroll
            for (int i = 0; i < 3; i++)
                part += a.m4 * ((double)p[i].re * (double)p[i].re + (double)p[i].im * (double)p[i].im) +
                        ((double)acc[i].re * (double)acc[i].re + (double)acc[i].im * (double)acc[i].im);
            VF::template store<true>(a.out, Vh, cb, acc);
        } else if constexpr (EPI == EPI_PAPX) {
            // p' = r + beta p_old into the other buffer, x += alpha p_old if
            // pending, out = D p' ; partial m4 |p'|^2 + |out|^2
            cx<T> po[3], pn[3];
            VF::template load<false>(pin, Vh, cb, po);
            VF::template load<false>(a.rin, Vh, cb, pn);
#pragma unroll
            for (int i = 0; i < 3; i++) {
                pn[i].re = fma(beta, po[i].re, pn[i].re);
                pn[i].im = fma(beta, po[i].im, pn[i].im);
                part += a.m4 * ((double)pn[i].re * (double)pn[i].re + (double)pn[i].im * (double)pn[i].im) +
                        ((double)acc[i].re * (double)acc[i].re + (double)acc[i].im * (double)acc[i].im);
            }
            VF::template store<false>(pin == a.in ? a.pb : (void *)a.in, Vh, cb, pn);
            if (a.st->pend) {
                const T alpha = (T)a.st->alpha;
                cx<T> x[3];
                VF::template load<false>(a.xw, Vh, cb, x);
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    x[i].re = fma(alpha, po[i].re, x[i].re);
                    x[i].im = fma(alpha, po[i].im, x[i].im);
                }
                VF::template store<false>(a.xw, Vh, cb, x);
            }
            VF::template store<true>(a.out, Vh, cb, acc);
        } else if constexpr (EPI == EPI_UPD) {
            // Ap = m4 p - D in ; r -= alpha Ap ; partial |r|^2
            const T m4 = (T)a.m4, alpha = (T)alpha64;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const T apr = m4 * pu[i].re - acc[i].re;
                const T api = m4 * pu[i].im - acc[i].im;
                ru[i].re = fma(-alpha, apr, ru[i].re);
                ru[i].im = fma(-alpha, api, ru[i].im);
                part += (double)ru[i].re * (double)ru[i].re + (double)ru[i].im * (double)ru[i].im;
            }
            VF::template store<false>(a.rw, Vh, cb, ru);
        } else if constexpr (EPI == EPI_A) {
            // out = m4 p - D in ; partial Re <p, out>
            cx<T> p[3];
            VF::template load<false>(a.aux0, Vh, cb, p);
            const T m4 = (T)a.m4;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                acc[i].re = m4 * p[i].re - acc[i].re;
                acc[i].im = m4 * p[i].im - acc[i].im;
                part += (double)p[i].re * (double)acc[i].re + (double)p[i].im * (double)acc[i].im;
            }
            VF::template store<true>(a.out, Vh, cb, acc);
        } else {
            // r = b - (m4 x - D in), FP64 only; partial |r|^2
            cx<double> x[3], bb[3];
            VecFmt<double>::load<false>(a.aux0, Vh, cb, x);
            VecFmt<double>::load<false>(a.aux1, Vh, cb, bb);
#pragma unroll
            for (int i = 0; i < 3; i++) {
                acc[i].re = bb[i].re - (a.m4 * x[i].re - acc[i].re);
                acc[i].im = bb[i].im - (a.m4 * x[i].im - acc[i].im);
                part += acc[i].re * acc[i].re + acc[i].im * acc[i].im;
            }
            if constexpr (EPI == EPI_RES) {
                VF::template store<true>(a.out, Vh, cb, acc);
            } else {
                cx<float> lo[3];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    lo[i].re = (float)acc[i].re;
                    lo[i].im = (float)acc[i].im;
                }
                VecFmt<float>::store<true>(a.out_lo, Vh, cb, lo);
            }
        }
    }
    if constexpr (EPI != EPI_PLAIN) write_partial(part, a.partials, blk);
}

// One Dslash launch. With events, they are carried by the kernel's own
// dispatch packet (hipExtLaunchKernel) and time the kernel alone -- what a
// kernel trace reports -- without the marker packets (and their stream time)
// that separate event records add around it.
template <class K>
static void launch_k(K kernel, dim3 grid, dim3 block, size_t shm, hipStream_t s, const DslashArgs &a, hipEvent_t e0,
                     hipEvent_t e1)
{
    if (e0 || e1) hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shm, s, e0, e1, 0u, a);
    else hipLaunchKernelGGL(kernel, grid, block, shm, s, a);
}

template <class LF, int HPI, bool NTL>
static hipError_t launch_fmt(int epi, const DslashArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid(a.l.nblk_pad), block(a.l.bs);
    const size_t shm =
        HPI == 4 ? (size_t)3 * staged_sites(a.g, a.l.bs) * sizeof(typename VecFmt<typename LF::real>::store_t) : 0;
    switch (epi) {
    case EPI_PLAIN: launch_k(k_dslash<LF, EPI_PLAIN, HPI, NTL>, grid, block, shm, s, a, e0, e1); break;
    case EPI_A: launch_k(k_dslash<LF, EPI_A, HPI, NTL>, grid, block, shm, s, a, e0, e1); break;
    case EPI_PAP: launch_k(k_dslash<LF, EPI_PAP, HPI, NTL>, grid, block, shm, s, a, e0, e1); break;
    case EPI_UPD: launch_k(k_dslash<LF, EPI_UPD, HPI, NTL>, grid, block, shm, s, a, e0, e1); break;
    case EPI_PAPX: launch_k(k_dslash<LF, EPI_PAPX, HPI, NTL>, grid, block, shm, s, a, e0, e1); break;
    case EPI_RES:
    case EPI_RES_LO:
        if constexpr (std::is_same<typename LF::real, double>::value) {
            if (epi == EPI_RES) launch_k(k_dslash<LF, EPI_RES, HPI, NTL>, grid, block, shm, s, a, e0, e1);
            else launch_k(k_dslash<LF, EPI_RES_LO, HPI, NTL>, grid, block, shm, s, a, e0, e1);
        } else {
            return hipErrorInvalidValue;
        }
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LF, bool NTL>
static hipError_t launch_hpi_ntl(int epi, const DslashArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (a.U3) {
        // improved operator: fat and Naik fields are general complex 3x3 (18 reals)
        if constexpr (std::is_same<LF, LinkF64R18>::value || std::is_same<LF, LinkF32R18>::value)
            return launch_fmt<LF, 0, NTL>(epi, a, s, e0, e1);
        else return hipErrorInvalidValue;
    }
    switch (a.hpi) {
    case 1: return launch_fmt<LF, 1, NTL>(epi, a, s, e0, e1);
    case 2: return launch_fmt<LF, 2, NTL>(epi, a, s, e0, e1);
    case 4:
        // the staged range must fit the LDS budget of a workgroup
        if (staged_sites(a.g, a.l.bs) > kMaxStagedSites) return launch_fmt<LF, 2, NTL>(epi, a, s, e0, e1);
        return launch_fmt<LF, 4, NTL>(epi, a, s, e0, e1);
    case 8: return launch_fmt<LF, 8, NTL>(epi, a, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

// Variant = (hops whose loads issue together, streaming or cached link loads).
// Streaming (non-temporal) link loads keep a link field that is far larger
// than the caches from evicting the input vector; a field that fits in the
// 256 MB Infinity Cache (FP32/BF16 12-real at 32^4) may instead stay there
// from one Dslash to the next with cached loads.
template <class LF>
static hipError_t launch_hpi(int epi, const DslashArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    return a.ntl ? launch_hpi_ntl<LF, true>(epi, a, s, e0, e1) : launch_hpi_ntl<LF, false>(epi, a, s, e0, e1);
}

hipError_t launch_dslash(Fmt f, int epi, const DslashArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (!dslash_bs_ok(a.l.bs) || a.l.nblk_pad % 8 || a.l.nblk_pad * a.l.bs < a.g.Vh) return hipErrorInvalidValue;
    switch (f) {
    case F64R18: return launch_hpi<LinkF64R18>(epi, a, s, e0, e1);
    case F64R12: return launch_hpi<LinkF64R12>(epi, a, s, e0, e1);
    case F32R18: return launch_hpi<LinkF32R18>(epi, a, s, e0, e1);
    case F32R12: return launch_hpi<LinkF32R12>(epi, a, s, e0, e1);
    case BF16R12: return launch_hpi<LinkBF16R12>(epi, a, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------- packing ---

// canonical [4][V][3][3][2] float64 (eo order) -> planes of format LF
template <class LF>
__global__ __launch_bounds__(kBS) void k_pack_links(const double *__restrict__ Uc, void *__restrict__ Up, Geom g)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t idx = (int64_t)blockIdx.x * kBS + threadIdx.x; // mu*V + eo
    if (idx >= 4 * V) return;
    const int mu = (int)(idx / V);
    const int64_t eo = idx - mu * V;
    const int par = eo >= g.Vh;
    const int cb = (int)(eo - par * (int64_t)g.Vh);
    double s[18];
    const dv2 *src = (const dv2 *)(Uc + idx * 18);
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const dv2 v = src[k];
        s[2 * k] = v.x;
        s[2 * k + 1] = v.y;
    }
    LF::store(Up, (size_t)g.Vh, par * 4 + mu, cb, s);
}

hipError_t launch_pack_links(Fmt f, const double *Uc, void *Up, const Geom &g, hipStream_t s)
{
    const int64_t n = 4 * 2 * (int64_t)g.Vh;
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    switch (f) {
    case F64R18: hipLaunchKernelGGL(k_pack_links<LinkF64R18>, grid, block, 0, s, Uc, Up, g); break;
    case F64R12: hipLaunchKernelGGL(k_pack_links<LinkF64R12>, grid, block, 0, s, Uc, Up, g); break;
    case F32R18: hipLaunchKernelGGL(k_pack_links<LinkF32R18>, grid, block, 0, s, Uc, Up, g); break;
    case F32R12: hipLaunchKernelGGL(k_pack_links<LinkF32R12>, grid, block, 0, s, Uc, Up, g); break;
    case BF16R12: hipLaunchKernelGGL(k_pack_links<LinkBF16R12>, grid, block, 0, s, Uc, Up, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// planes of format LF -> canonical [4][V][3][3][2] float64: stored reals are
// widened exactly; 12-real formats rebuild row 2 as the Dslash does
template <class LF>
__global__ __launch_bounds__(kBS) void k_unpack_links(const void *__restrict__ Up, double *__restrict__ Uc, Geom g)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t idx = (int64_t)blockIdx.x * kBS + threadIdx.x; // mu*V + eo
    if (idx >= 4 * V) return;
    const int mu = (int)(idx / V);
    const int64_t eo = idx - mu * V;
    const int par = eo >= g.Vh;
    const unsigned cb = (unsigned)(eo - par * (int64_t)g.Vh);
    cx<typename LF::real> u[9];
    LF::template load<false>(Up, (size_t)g.Vh, par * 4 + mu, cb, u);
    dv2 *dst = (dv2 *)(Uc + idx * 18);
#pragma unroll
    for (int k = 0; k < 9; k++) dst[k] = dv2{(double)u[k].re, (double)u[k].im};
}

hipError_t launch_unpack_links(Fmt f, const void *Up, double *Uc, const Geom &g, hipStream_t s)
{
    const int64_t n = 4 * 2 * (int64_t)g.Vh;
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    switch (f) {
    case F64R18: hipLaunchKernelGGL(k_unpack_links<LinkF64R18>, grid, block, 0, s, Up, Uc, g); break;
    case F64R12: hipLaunchKernelGGL(k_unpack_links<LinkF64R12>, grid, block, 0, s, Up, Uc, g); break;
    case F32R18: hipLaunchKernelGGL(k_unpack_links<LinkF32R18>, grid, block, 0, s, Up, Uc, g); break;
    case F32R12: hipLaunchKernelGGL(k_unpack_links<LinkF32R12>, grid, block, 0, s, Up, Uc, g); break;
    case BF16R12: hipLaunchKernelGGL(k_unpack_links<LinkBF16R12>, grid, block, 0, s, Up, Uc, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBS) void k_pack_vec(const double *__restrict__ src, void *__restrict__ dst, int Vh)
{
    const int cb = blockIdx.x * kBS + threadIdx.x;
    if (cb >= Vh) return;
    const dv2 *p = (const dv2 *)src + (size_t)cb * 3;
    cx<T> v[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const dv2 w = p[i];
        v[i].re = (T)w.x;
        v[i].im = (T)w.y;
    }
    VecFmt<T>::template store<false>(dst, (size_t)Vh, cb, v);
}

template <typename T>
__global__ __launch_bounds__(kBS) void k_unpack_vec(const void *__restrict__ src, double *__restrict__ dst, int Vh)
{
    const int cb = blockIdx.x * kBS + threadIdx.x;
    if (cb >= Vh) return;
    cx<T> v[3];
    VecFmt<T>::template load<false>(src, (size_t)Vh, cb, v);
    dv2 *p = (dv2 *)dst + (size_t)cb * 3;
#pragma unroll
    for (int i = 0; i < 3; i++) p[i] = dv2{(double)v[i].re, (double)v[i].im};
}

hipError_t launch_pack_vec(bool f64, const double *src, void *dst, const Geom &g, hipStream_t s)
{
    const dim3 grid((g.Vh + kBS - 1) / kBS), block(kBS);
    if (f64) hipLaunchKernelGGL(k_pack_vec<double>, grid, block, 0, s, src, dst, g.Vh);
    else hipLaunchKernelGGL(k_pack_vec<float>, grid, block, 0, s, src, dst, g.Vh);
    return hipGetLastError();
}

hipError_t launch_unpack_vec(bool f64, const void *src, double *dst, const Geom &g, hipStream_t s)
{
    const dim3 grid((g.Vh + kBS - 1) / kBS), block(kBS);
    if (f64) hipLaunchKernelGGL(k_unpack_vec<double>, grid, block, 0, s, src, dst, g.Vh);
    else hipLaunchKernelGGL(k_unpack_vec<float>, grid, block, 0, s, src, dst, g.Vh);
    return hipGetLastError();
}

// ------------------------------------------------------------ geometry ---

__global__ __launch_bounds__(kBS) void k_index_maps(int32_t *__restrict__ lex_of_eo, int32_t *__restrict__ nbr, Geom g)
{
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; // par*Vh + cb
    if (i >= 2 * (int64_t)g.Vh) return;
    const int par = i >= g.Vh;
    const int cb = (int)(i - par * (int64_t)g.Vh);
    int c[4];
    decode(g, par, cb, c);
    lex_of_eo[i] = c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        nbr[((size_t)par * 8 + mu) * g.Vh + cb] = nbr_fwd(g, c, cb, mu);
        nbr[((size_t)par * 8 + 4 + mu) * g.Vh + cb] = nbr_bwd(g, c, cb, mu);
    }
}

hipError_t launch_index_maps(int32_t *lex_of_eo, int32_t *nbr, const Geom &g, hipStream_t s)
{
    const int64_t n = 2 * (int64_t)g.Vh;
    hipLaunchKernelGGL(k_index_maps, dim3((unsigned)((n + kBS - 1) / kBS)), dim3(kBS), 0, s, lex_of_eo, nbr, g);
    return hipGetLastError();
}

} // namespace lgt
