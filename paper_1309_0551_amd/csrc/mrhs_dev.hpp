// mrhs_dev.hpp -- device building blocks of the multi-RHS Dslash.
//
// Multi-RHS vectors hold N right-hand sides of one parity as [3][V/2][N]
// complex (right-hand side fastest).
//
// One lane per (site, rhs): dslash_mrhs. The N lanes of a site read one
// contiguous run of each input and issue the same link address, which the
// load unit serves once.
//
// Four lanes per site: dslash_site4. A wavefront covers 16 sites; each of a site's 4 lanes owns R = N/4
// consecutive right-hand sides (rhs = lane*R + r). The 4 lanes share
// every link load and each lane's inputs are R contiguous complex numbers per
// colour. Two engines compute the 3x3 complex products:
//
//  * VALU: per lane, R matrix-vector products with FMAs.
//  * MFMA: the 16 sites of a wavefront are the 16 blocks of
//    v_mfma_f32_4x4x1f32, whose lane 4b+t supplies row t of block b's A
//    column, column t of its B row, and receives column t of the 4x4 result
//    (row i in VGPR i). In the real embedding out(6) = W(6x6) in(6) of each
//    hop, row i of a block is output real 4*ct + i (A operand: entry
//    W[4ct+i][k], built by lane i from the link), column j is right-hand side
//    lane_j*R + r (B operand: input real k of that right-hand side, from lane
//    j) -- each lane ends with the output reals of its own right-hand sides.
//    Per hop: 6 input reals x R column tiles x 2 row tiles (6 of 8 rows
//    used) = 12 R MFMAs.
//    Output reals o = (Re c0, Re c1, Re c2, Im c0, Im c1, Im c2); for a hop
//    matrix W: Re out_a = sum_b Re W_ab Re in_b - Im W_ab Im in_b,
//    Im out_a = sum_b Im W_ab Re in_b + Re W_ab Im in_b.
#pragma once
#include <hip/hip_runtime.h>

#include "fields.hpp"
#include "geom.hpp"

namespace lgt {

constexpr int kEven = 0, kOdd = 1; // output parity of a half-Dslash

// logical block (a tile of consecutive sites) of this workgroup, or -1
__device__ __forceinline__ int mrhs_block(const TileOrder &o, int nblk_pad)
{
    if (o.n_ts) return zorder_tile(o, blockIdx.x & 7, blockIdx.x >> 3);
    return xcd_block(blockIdx.x, nblk_pad);
}

// blocks to launch for nblk tiles under order o
inline int mrhs_grid(const TileOrder &o, int nblk) { return o.n_ts ? 8 * o.per : (nblk + 7) / 8 * 8; }

template <typename T> struct V2of;
template <> struct V2of<double> { using type = dv2; };
template <> struct V2of<float> { using type = fv2; };

// element (colour c, site, rhs) of a multi-RHS vector; the plane base is
// uniform. NT: non-temporal (streaming) loads
template <typename T, bool NT = false>
__device__ __forceinline__ void ldm(const void *v, size_t Vh, int logN, unsigned site, unsigned rhs, cx<T> o[3])
{
    using V2 = typename V2of<T>::type;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const V2 w = ld<NT>((const V2 *)v + ((size_t)c * Vh << logN), (site << logN) + rhs);
        o[c].re = w.x;
        o[c].im = w.y;
    }
}

// NT: non-temporal store, for an output the same kernel never reads back (the
// standalone multi-RHS Dslash): write-allocating it would evict the input
// that the neighbouring sites' gathers are about to reuse.
template <typename T, bool NT = false>
__device__ __forceinline__ void stm(void *v, size_t Vh, int logN, unsigned site, unsigned rhs, const cx<T> o[3])
{
    using V2 = typename V2of<T>::type;
#pragma unroll
    for (int c = 0; c < 3; c++) st<NT>((V2 *)v + ((size_t)c * Vh << logN), (site << logN) + rhs, V2{o[c].re, o[c].im});
}

// D on one (site, rhs): the input at a neighbour comes from `in(site, v)`.
template <class LF, class In>
__device__ __forceinline__ void dslash_mrhs(const Geom &g, int par, const void *U, int cb, In in,
                                            cx<typename LF::real> acc[3])
{
    using T = typename LF::real;
    const size_t Vh = (size_t)g.Vh;
    int c[4];
    decode(g, par, cb, c);
#pragma unroll
    for (int i = 0; i < 3; i++) acc[i].re = acc[i].im = T(0);
#pragma unroll 1
    for (int mu = 0; mu < 4; mu++) {
        const Hop h = hop_rt(g, c, cb, mu);
        cx<T> u[9], v[3];
        LF::template load<false>(U, Vh, par * 4 + mu, cb, u);
        in(h.f, v);
        negate_if(h.fneg, v);
        mv_add(u, v, acc);
        LF::template load<false>(U, Vh, (1 - par) * 4 + mu, h.b, u);
        in(h.b, v);
        negate_if(h.bneg, v);
        amv_sub(u, v, acc);
    }
}

typedef float f4v __attribute__((ext_vector_type(4)));

// R consecutive complex numbers per colour: element (c, site, rhs0 .. rhs0+R-1)
// NT: non-temporal (streaming) loads
template <typename T, int R, bool NT = false>
__device__ __forceinline__ void ldm_r(const void *v, size_t Vh, int logN, unsigned site, unsigned rhs0, cx<T> o[R][3])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const size_t plane = (size_t)c * Vh << logN;
        const unsigned i = (site << logN) + rhs0;
        if constexpr (std::is_same<T, float>::value && R % 2 == 0) {
#pragma unroll
            for (int q = 0; q < R / 2; q++) {
                const fv4 w = ld<NT>((const fv4 *)((const fv2 *)v + plane + i) + q, 0u);
                o[2 * q][c].re = w.x;
                o[2 * q][c].im = w.y;
                o[2 * q + 1][c].re = w.z;
                o[2 * q + 1][c].im = w.w;
            }
        } else {
            using V2 = typename std::conditional<std::is_same<T, double>::value, dv2, fv2>::type;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const V2 w = ld<NT>((const V2 *)v + plane, i + r);
                o[r][c].re = w.x;
                o[r][c].im = w.y;
            }
        }
    }
}

template <typename T, int R, bool NT = false>
__device__ __forceinline__ void stm_r(void *v, size_t Vh, int logN, unsigned site, unsigned rhs0, const cx<T> o[R][3])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const size_t plane = (size_t)c * Vh << logN;
        const unsigned i = (site << logN) + rhs0;
        if constexpr (std::is_same<T, float>::value && R % 2 == 0) {
#pragma unroll
            for (int q = 0; q < R / 2; q++)
                st<NT>((fv4 *)((fv2 *)v + plane + i) + q, 0u,
                          fv4{o[2 * q][c].re, o[2 * q][c].im, o[2 * q + 1][c].re, o[2 * q + 1][c].im});
        } else {
            using V2 = typename std::conditional<std::is_same<T, double>::value, dv2, fv2>::type;
#pragma unroll
            for (int r = 0; r < R; r++) st<NT>((V2 *)v + plane, i + r, V2{o[r][c].re, o[r][c].im});
        }
    }
}

// Row o of the real 6x6 embedding of the hop matrix
// W = (neg ? -1 : 1) * (fwd ? U : U^dag): the six entries W[o][k]
// (k = Re in_0..2, Im in_0..2); zero for the unused rows o = 6, 7.
__device__ __forceinline__ void w_row(const cx<float> u[9], bool fwd, bool neg, int o, float row[6])
{
    if (o >= 6) {
#pragma unroll
        for (int k = 0; k < 6; k++) row[k] = 0.f;
        return;
    }
    const int a = o >= 3 ? o - 3 : o;
    // select between values, never between element addresses (that would
    // keep u in private memory)
    auto sel = [a](float x0, float x1, float x2) __attribute__((always_inline)) {
        return a == 0 ? x0 : (a == 1 ? x1 : x2);
    };
    cx<float> w[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        // W_ak = U_ak (forward) or conj(U_ka) (adjoint)
        const float ar = sel(u[k].re, u[3 + k].re, u[6 + k].re);             // U_ak
        const float ai = sel(u[k].im, u[3 + k].im, u[6 + k].im);
        const float cr = sel(u[3 * k].re, u[3 * k + 1].re, u[3 * k + 2].re); // U_ka
        const float ci = sel(u[3 * k].im, u[3 * k + 1].im, u[3 * k + 2].im);
        w[k].re = fwd ? ar : cr;
        w[k].im = fwd ? ai : -ci;
        if (neg) {
            w[k].re = -w[k].re;
            w[k].im = -w[k].im;
        }
    }
    if (o < 3) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            row[k] = w[k].re;
            row[3 + k] = -w[k].im;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            row[k] = w[k].im;
            row[3 + k] = w[k].re;
        }
    }
}

// One hop for the lane's R right-hand sides: acc[r] += W v[r]
template <int R, bool MFMA>
__device__ __forceinline__ void hop_apply(const cx<float> u[9], bool fwd, bool neg, const cx<float> v[R][3], int lane4,
                                          cx<float> acc[R][3], f4v C[R][2])
{
    if constexpr (MFMA) {
        float w0[6], w1[6]; // this lane's rows of W: output reals lane4 and 4 + lane4
        w_row(u, fwd, neg, lane4, w0);
        w_row(u, fwd, neg, 4 + lane4, w1);
#pragma unroll
        for (int k = 0; k < 6; k++) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                const float x = k < 3 ? v[r][k].re : v[r][k - 3].im;
                C[r][0] = __builtin_amdgcn_mfma_f32_4x4x1f32(w0[k], x, C[r][0], 0, 0, 0);
                C[r][1] = __builtin_amdgcn_mfma_f32_4x4x1f32(w1[k], x, C[r][1], 0, 0, 0);
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; r++) {
            cx<float> w[3] = {v[r][0], v[r][1], v[r][2]};
            if (fwd) { // acc += (+-U) v
                negate_if(neg, w);
                mv_add(u, w, acc[r]);
            } else { // acc += (+-U^dag) v  ==  acc -= U^dag (-+v)
                negate_if(!neg, w);
                amv_sub(u, w, acc[r]);
            }
        }
    }
}

// D on one site for the lane's R right-hand sides. in(site, v[R][3]) loads the
// lane's inputs at a neighbour. FP32 vectors (F32 or BF16 links).
// UNR directions per trip of the direction loop (1, 2 or 4): the loads of
// 2 UNR hops in flight at once, for more registers. NTL: streaming
// (non-temporal) link loads.
template <class LF, int R, bool MFMA, int UNR = 1, bool NTL = false, class In>
__device__ __forceinline__ void dslash_site4(const Geom &g, int par, const void *U, int cb, int lane4, In in,
                                             cx<float> acc[R][3])
{
    const size_t Vh = (size_t)g.Vh;
    int c[4];
    decode(g, par, cb, c);
    f4v C[R][2];
#pragma unroll
    for (int r = 0; r < R; r++) {
        C[r][0] = f4v{0.f, 0.f, 0.f, 0.f};
        C[r][1] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 3; i++) acc[r][i].re = acc[r][i].im = 0.f;
    }
#pragma unroll 1
    for (int m0 = 0; m0 < 4; m0 += UNR) {
#pragma unroll
        for (int j = 0; j < UNR; j++) {
            const int mu = m0 + j;
            const Hop h = hop_rt(g, c, cb, mu);
            cx<float> u[9], v[R][3];
            LF::template load_quad<NTL>(U, Vh, par * 4 + mu, cb, u, lane4);
            in(h.f, v);
            hop_apply<R, MFMA>(u, true, h.fneg, v, lane4, acc, C);
            LF::template load_quad<NTL>(U, Vh, (1 - par) * 4 + mu, h.b, u, lane4);
            in(h.b, v);
            // the adjoint hop enters with a minus sign: fold it into neg
            hop_apply<R, MFMA>(u, false, !h.bneg, v, lane4, acc, C);
        }
    }
    if constexpr (MFMA) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            acc[r][0].re = C[r][0][0];
            acc[r][1].re = C[r][0][1];
            acc[r][2].re = C[r][0][2];
            acc[r][0].im = C[r][0][3];
            acc[r][1].im = C[r][1][0];
            acc[r][2].im = C[r][1][1];
        }
    }
}

} // namespace lgt
