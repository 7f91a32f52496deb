// geom.hpp -- checkerboarded 4-D lattice geometry for the device kernels.
//
// A site has a unique 4-tuple and eight neighbours, two per dimension (Sec. 1).
// Ordering: lex = x + Lx*(y + Ly*(z + Lz*t)), parity = (x+y+z+t)&1,
// cb = lex>>1, eo = parity*V/2 + cb. Neighbour cb indices, staggered phases and
// boundary signs are computed on the fly from cb: no index table is read from
// memory, so the Dslash streams only links and vectors.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lgt {

struct Geom {
    int L[4];      // extents x, y, z, t (even)
    int bc[4];     // +1 / -1 per direction
    int hx;        // Lx / 2
    int Vh;        // V / 2
    int str[4];    // cb stride of a unit step: str[1] = hx, str[2] = hx*Ly, str[3] = hx*Ly*Lz
};

// Coordinates of the site (par, cb).
__host__ __device__ __forceinline__ void decode(const Geom &g, int par, int cb, int c[4])
{
    const int q = cb / g.hx;
    const int xh = cb - q * g.hx;
    const int q2 = q / g.L[1];
    c[1] = q - q2 * g.L[1];
    const int q3 = q2 / g.L[2];
    c[2] = q2 - q3 * g.L[2];
    c[3] = q3;
    c[0] = 2 * xh + ((par + c[1] + c[2] + c[3]) & 1);
}

// cb index of x + mu (periodic wrap).
__host__ __device__ __forceinline__ int nbr_fwd(const Geom &g, const int c[4], int cb, int mu)
{
    if (mu == 0) {
        if (!(c[0] & 1)) return cb;                     // x even: x+1 shares x>>1
        return (c[0] == g.L[0] - 1) ? cb - (g.hx - 1) : cb + 1;
    }
    return (c[mu] == g.L[mu] - 1) ? cb - (g.L[mu] - 1) * g.str[mu] : cb + g.str[mu];
}

// cb index of x - mu (periodic wrap).
__host__ __device__ __forceinline__ int nbr_bwd(const Geom &g, const int c[4], int cb, int mu)
{
    if (mu == 0) {
        if (c[0] & 1) return cb;                        // x odd: x-1 shares x>>1
        return (c[0] == 0) ? cb + (g.hx - 1) : cb - 1;
    }
    return (c[mu] == 0) ? cb + (g.L[mu] - 1) * g.str[mu] : cb - g.str[mu];
}

// eta_mu(x): eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z)
__host__ __device__ __forceinline__ bool eta_neg(const int c[4], int mu)
{
    int s = 0;
    if (mu > 0) s += c[0];
    if (mu > 1) s += c[1];
    if (mu > 2) s += c[2];
    return s & 1;
}

// sign of the forward hop eta_mu s+_mu and of the backward hop eta_mu s-_mu
__host__ __device__ __forceinline__ bool fwd_neg(const Geom &g, const int c[4], int mu)
{
    return eta_neg(c, mu) ^ (c[mu] == g.L[mu] - 1 && g.bc[mu] < 0);
}
__host__ __device__ __forceinline__ bool bwd_neg(const Geom &g, const int c[4], int mu)
{
    return eta_neg(c, mu) ^ (c[mu] == 0 && g.bc[mu] < 0);
}

// Neighbours and hop signs for a direction mu known only at run time (all
// selects, no indexed access to c[] or g.L[], so a runtime loop over mu keeps
// everything in registers).
struct Hop {
    int f, b;        // cb of x + mu and x - mu
    bool fneg, bneg; // eta s+ < 0, eta s- < 0
};
__host__ __device__ __forceinline__ Hop hop_rt(const Geom &g, const int c[4], int cb, int mu)
{
    // read every field into a value first: selecting between field addresses
    // would turn into an indexed access to a private copy of g
    const int c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3];
    const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
    const int b0 = g.bc[0], b1 = g.bc[1], b2 = g.bc[2], b3 = g.bc[3];
    const int s1 = g.str[1], s2 = g.str[2], s3 = g.str[3];
    const int cm = mu == 0 ? c0 : mu == 1 ? c1 : mu == 2 ? c2 : c3;
    const int Lm = mu == 0 ? L0 : mu == 1 ? L1 : mu == 2 ? L2 : L3;
    const int bcm = mu == 0 ? b0 : mu == 1 ? b1 : mu == 2 ? b2 : b3;
    const int sm = mu == 1 ? s1 : mu == 2 ? s2 : s3;
    const int ep = (mu > 0 ? c0 : 0) + (mu > 1 ? c1 : 0) + (mu > 2 ? c2 : 0);
    Hop h;
    if (mu == 0) {
        h.f = (cm & 1) ? ((cm == Lm - 1) ? cb - (g.hx - 1) : cb + 1) : cb;
        h.b = (cm & 1) ? cb : ((cm == 0) ? cb + (g.hx - 1) : cb - 1);
    } else {
        h.f = (cm == Lm - 1) ? cb - (Lm - 1) * sm : cb + sm;
        h.b = (cm == 0) ? cb + (Lm - 1) * sm : cb - sm;
    }
    h.fneg = (ep & 1) ^ (cm == Lm - 1 && bcm < 0);
    h.bneg = (ep & 1) ^ (cm == 0 && bcm < 0);
    return h;
}

// Three-step neighbours x + 3 mu and x - 3 mu (improved operator's Naik hops)
// for a runtime mu, and their signs: eta_mu times bc_mu to the number of
// boundary crossings of the hop (twice for an extent of 2). On the x axis
// cb = (lex >> 1) moves by the change of x >> 1; on the others by the change
// of the coordinate times the cb stride.
__host__ __device__ __forceinline__ Hop hop3_rt(const Geom &g, const int c[4], int cb, int mu)
{
    const int c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3];
    const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
    const int b0 = g.bc[0], b1 = g.bc[1], b2 = g.bc[2], b3 = g.bc[3];
    const int s1 = g.str[1], s2 = g.str[2], s3 = g.str[3];
    const int cm = mu == 0 ? c0 : mu == 1 ? c1 : mu == 2 ? c2 : c3;
    const int Lm = mu == 0 ? L0 : mu == 1 ? L1 : mu == 2 ? L2 : L3;
    const int bcm = mu == 0 ? b0 : mu == 1 ? b1 : mu == 2 ? b2 : b3;
    const int sm = mu == 1 ? s1 : mu == 2 ? s2 : s3;
    const int ep = (mu > 0 ? c0 : 0) + (mu > 1 ? c1 : 0) + (mu > 2 ? c2 : 0);
    const int cf = (cm + 3) / Lm, xf = cm + 3 - cf * Lm;          // crossings, new coordinate
    const int cbk = (Lm + 2 - cm) / Lm, xb = cm - 3 + cbk * Lm;   // going down
    Hop h;
    if (mu == 0) {
        h.f = cb - (cm >> 1) + (xf >> 1);
        h.b = cb - (cm >> 1) + (xb >> 1);
    } else {
        h.f = cb + (xf - cm) * sm;
        h.b = cb + (xb - cm) * sm;
    }
    h.fneg = (ep & 1) ^ ((cf & 1) && bcm < 0);
    h.bneg = (ep & 1) ^ ((cbk & 1) && bcm < 0);
    return h;
}

// Workgroups are dispatched round-robin over the 8 XCDs. Remap so that each
// XCD walks a contiguous range of sites: neighbours in y, z and t then fall in
// the same XCD's L2. nblk_pad is a multiple of 8; blocks beyond nblk idle.
__host__ __device__ __forceinline__ int xcd_block(int bid, int nblk_pad)
{
    const int per = nblk_pad >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// z-blocked XCD order of site tiles, for kernels whose input vector is too
// large for an XCD's L2 to hold the three t-slices a slab walk reuses (many
// right-hand sides per site). Tiles are runs of `T` consecutive cb sites; when
// a t-slice (V/2 / Lt sites) holds a whole number n_ts >= 8 of them, the 8
// XCDs form a kz x (8 / kz) grid over (z, t): XCD x takes the tiles at
// positions [zx n_ts / kz, (zx+1) n_ts / kz) of each slice -- a range of z
// planes -- for the t-slices of range tx of the 8 / kz equal t ranges
// (zx = x mod kz, tx = x / kz), and walks them t-major. The input a tile reads
// from t +- 1 was then loaded a few tiles earlier by the same XCD; only the
// two z planes bounding the range (and the two slices bounding the t range)
// come from another XCD's share. Fewer z ranges halve the z-boundary
// fetches at the price of t-boundary ones and of a longer t-reuse distance.
struct TileOrder {
    int n_ts; // tiles per t-slice; 0: plain slab order (xcd_block)
    int Lt;
    int per;  // blocks launched per XCD: ceil(Lt / (8 / kz)) * ceil(n_ts / kz)
    int kz;   // z ranges: 8, 4, 2 or 1
};

__host__ __device__ __forceinline__ TileOrder tile_order(const Geom &g, int T, int kz = 8)
{
    TileOrder o{0, g.L[3], 0, kz};
    const int slice = g.Vh / g.L[3];
    if (T <= 0 || slice % T != 0 || slice / T < 8) return o;
    const int kt = 8 / kz;
    o.n_ts = slice / T;
    o.per = (g.L[3] + kt - 1) / kt * ((o.n_ts + kz - 1) / kz);
    return o;
}

// tile of the k-th block of XCD x under order o, or -1 past its share
__host__ __device__ __forceinline__ int zorder_tile(const TileOrder &o, int x, int k)
{
    const int kt = 8 / o.kz, zx = x % o.kz, tx = x / o.kz;
    const int lo = zx * o.n_ts / o.kz, hi = (zx + 1) * o.n_ts / o.kz, ns = hi - lo;
    const int t0 = tx * o.Lt / kt, nt = (tx + 1) * o.Lt / kt - t0;
    if (k >= nt * ns) return -1;
    const int t = k / ns;
    return (t0 + t) * o.n_ts + lo + (k - t * ns);
}

} // namespace lgt
