// march.h -- kernels that walk a band of lattice rows through consecutive time slices, holding
// the reuse along tau on chip: the normal operator M^dagger M of Eq. (22) in one pass over HBM,
// step A of the conjugate-gradient iteration, and the FP64 stencils of its reliable update.
//
// With chi = M psi (Eq. 17):  (M^dagger M psi)(tau) = A_tau chi(tau) + s_{tau-1} chi(tau - 1),
// where A_tau is the time-local part of M (diagonal, hopping, Yukawa coupling to phi(tau)) and
// s_{tau-1} the sign of the time link (-1 across the antiperiodic wrap at tau = 0).  Applying
// A_tau needs chi(tau) at the spatial neighbours, so chi(tau) = A_tau psi(tau) + s_tau psi(tau+1)
// is formed one row beyond the rows a workgroup writes, and chi(tau - 1) is the previous slice
// of the same workgroup.  HBM then sees psi and phi read once and the result written once:
// 76 B per site in FP32 (complex64 spinors, FP32 phi), 152 B in FP64, half the two-pass bytes.
//
// Workgroups own a band of whole rows (every y) of one vector and a segment of slices; they are
// ordered segment-major, so with the XCD remap each XCD sweeps every band of a run of
// consecutive segments and the rows beside a band are read through the same L2.  A second form
// of the normal operator takes one slice per workgroup and forms chi(tau - 1) itself.
//
// The one-pass normal operator and the reliable-update marches take the nearest-neighbour
// operator only; step A also takes the production model's two-site hops, with two rows beside
// the band on either side.  The arithmetic per site is that of the two-pass kernels, in the same
// order.
#pragma once

#include "kernels.h"

namespace hmc {

// Most threads of a marching workgroup (8 waves: up to 256 VGPRs per thread).
constexpr int kMarchMaxThreads = 512;

// The workgroup's vector, band and segment.
struct MarchPos {
    int k, x0, nr, t0, t1;
};
// Workgroup `rem` of vector k: segment-major, bands within a segment.
__device__ __forceinline__ MarchPos march_pos_in(const Lat& lat, const MarchPlan& mp, int k, int rem) {
    MarchPos p;
    p.k = k;
    const int seg = rem / mp.nband, band = rem - seg * mp.nband;
    p.x0 = band * mp.R;
    p.nr = lat.L - p.x0 < mp.R ? lat.L - p.x0 : mp.R;
    p.t0 = seg * mp.seglen;
    p.t1 = lat.Lt - p.t0 < mp.seglen ? lat.Lt : p.t0 + mp.seglen;
    return p;
}
// Workgroup wg of a launch over vectors cut alike, vector-major.
__device__ __forceinline__ MarchPos march_pos(const Lat& lat, const MarchPlan& mp, int wg) {
    const int per_vec = mp.nseg * mp.nband;
    const int k = wg / per_vec;
    return march_pos_in(lat, mp, k, wg - k * per_vec);
}

__device__ __forceinline__ int wrap_row(int x, int L) { return x < 0 ? x + L : (x >= L ? x - L : x); }

// Dynamic LDS of a marching workgroup: chi on R + 2 rows, 4 components, L sites.
template <typename R>
__host__ __device__ inline size_t march_lds(int Rrows, int L) {
    return size_t(Rrows + 2) * 4 * size_t(L) * sizeof(C2<R>);
}

// A_tau v + ts tt at the pair (x, y), y even: the time-local part of M (diagonal, hopping,
// Yukawa coupling) from v(tau) in LDS (row r of a band buffer, [row][component][y]), plus the
// time link ts tt, with phi(tau) at the pair given as (P1, P2, P3), each holding a component at
// the two sites.  The arithmetic of the two-pass pair stencil (dslash_pair) in its order, so
// both M (tt = v(tau + 1), ts = s_tau) and M^dagger (tt = v(tau - 1), ts = s_{tau-1}) come out
// as the separate passes compute them.  cen receives v(tau) at the pair.
// NN2: also the hops by two sites of the production model (rows r +- 2 of the buffer, the pairs
// (y - 2, y - 1) and (y + 2, y + 3)), added as the two-pass pair stencil adds them.
template <bool NN2 = false>
__device__ __forceinline__ void stencil_pair_lds(const float2* __restrict__ chi, int r, int x, int y, int L,
                                                 float2 P1, float2 P2, float2 P3, const Coef<float>& cf, float ts,
                                                 const float4 (&tt)[4], float4 (&o)[4], float4 (&cen)[4]) {
    const int rowc = 4 * L;
    auto lds4 = [&](int rr, int c, int yy) { return *reinterpret_cast<const float4*>(chi + rr * rowc + c * L + yy); };
    const int yl = y == 0 ? L - 1 : y - 1, yr = y + 2 == L ? 0 : y + 2;
    const int ym2 = y == 0 ? L - 2 : y - 2;
#pragma unroll
    for (int c = 0; c < 4; ++c) cen[c] = lds4(r, c, y);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int a = c >> 1;
        const float4 xp = lds4(r + 1, c, y), xm = lds4(r - 1, c, y), t4 = tt[c];
        float2 lo, hi;
        float4 m2, p2;
        if constexpr (NN2) {
            m2 = lds4(r, c, ym2);
            p2 = lds4(r, c, yr);
            lo = make_float2(m2.z, m2.w);
            hi = make_float2(p2.x, p2.y);
        } else {
            lo = chi[r * rowc + c * L + yl];
            hi = chi[r * rowc + c * L + yr];
        }
        const float4 ce = cen[c];
        const float dg = cf.diag[a], h0 = cf.hop[a][0], h1 = cf.hop[a][1];
        float4 v;
        v.x = dg * ce.x + h0 * (xp.x + xm.x) + h1 * (lo.x + ce.z) + ts * t4.x;
        v.y = dg * ce.y + h0 * (xp.y + xm.y) + h1 * (lo.y + ce.w) + ts * t4.y;
        v.z = dg * ce.z + h0 * (xp.z + xm.z) + h1 * (ce.x + hi.x) + ts * t4.z;
        v.w = dg * ce.w + h0 * (xp.w + xm.w) + h1 * (ce.y + hi.y) + ts * t4.w;
        if constexpr (NN2) {
            const float4 xx = f4add(lds4(r + 2, c, y), lds4(r - 2, c, y)), yy = f4add(m2, p2);
            const float u0 = cf.hop2[a][0], u1 = cf.hop2[a][1];
            v.x += u0 * xx.x + u1 * yy.x;
            v.y += u0 * xx.y + u1 * yy.y;
            v.z += u0 * xx.z + u1 * yy.z;
            v.w += u0 * xx.w + u1 * yy.w;
        }
        o[c] = v;
    }
    const float g0 = cf.cpl * float((x & 1) ? -1 : 1), g1 = -g0;   // (-1)^(x+y), y even
    const float q1a = g0 * P1.x, q2a = g0 * P2.x, q3a = g0 * P3.x;
    const float q1b = g1 * P1.y, q2b = g1 * P2.y, q3b = g1 * P3.y;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const float4 u = cen[2 * (1 - a)], w = cen[2 * (1 - a) + 1];
        o[2 * a].x += q3a * u.x + q1a * w.x + q2a * w.y;
        o[2 * a].y += q3a * u.y + q1a * w.y - q2a * w.x;
        o[2 * a].z += q3b * u.z + q1b * w.z + q2b * w.w;
        o[2 * a].w += q3b * u.w + q1b * w.w - q2b * w.z;
        o[2 * a + 1].x += q1a * u.x - q2a * u.y - q3a * w.x;
        o[2 * a + 1].y += q1a * u.y + q2a * u.x - q3a * w.y;
        o[2 * a + 1].z += q1b * u.z - q2b * u.w - q3b * w.z;
        o[2 * a + 1].w += q1b * u.w + q2b * u.z - q3b * w.w;
    }
}

// M^dagger at the pair (x, y) of slice tau (flat index s) from chi(tau) in LDS and chi(tau - 1)
// in registers (tt), with the time link's sign ts.
__device__ __forceinline__ void mdag_pair_lds(const float2* __restrict__ chi, int r, int x, int y, int s,
                                              const Lat& lat, const float* __restrict__ phi,
                                              const Coef<float>& cf, float ts, const float4 (&tt)[4],
                                              float4 (&o)[4], float4 (&cen)[4]) {
    const int vol = lat.vol;
    const float2 P1 = *reinterpret_cast<const float2*>(phi + s);
    const float2 P2 = *reinterpret_cast<const float2*>(phi + vol + s);
    const float2 P3 = *reinterpret_cast<const float2*>(phi + 2 * vol + s);
    stencil_pair_lds(chi, r, x, y, lat.L, P1, P2, P3, cf, ts, tt, o, cen);
}

// FP64 form of stencil_pair_lds at the site (x, y), phi(tau) there given as (q1, q2, q3) before
// the coupling and the staggered sign are applied.
template <bool NN2 = false>
__device__ __forceinline__ void stencil_site_lds(const double2* __restrict__ chi, int r, int x, int y, int L,
                                                 double f1, double f2, double f3, const Coef<double>& cf,
                                                 double ts, const double2 (&tt)[4], double2 (&o)[4],
                                                 double2 (&cen)[4]) {
    const int rowc = 4 * L;
    const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
    const int ypp = y + 2 >= L ? y + 2 - L : y + 2, ymm = y < 2 ? y - 2 + L : y - 2;
#pragma unroll
    for (int c = 0; c < 4; ++c) cen[c] = chi[r * rowc + c * L + y];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int a = c >> 1;
        const double2 hx = add<double>(chi[(r + 1) * rowc + c * L + y], chi[(r - 1) * rowc + c * L + y]);
        const double2 hy = add<double>(chi[r * rowc + c * L + yp], chi[r * rowc + c * L + ym]);
        double2 v = scl<double>(cf.diag[a], cen[c]);
        v = axpy<double>(cf.hop[a][0], hx, v);
        v = axpy<double>(cf.hop[a][1], hy, v);
        v = axpy<double>(ts, tt[c], v);
        if constexpr (NN2) {
            v = axpy<double>(cf.hop2[a][0], add<double>(chi[(r + 2) * rowc + c * L + y], chi[(r - 2) * rowc + c * L + y]), v);
            v = axpy<double>(cf.hop2[a][1], add<double>(chi[r * rowc + c * L + ypp], chi[r * rowc + c * L + ymm]), v);
        }
        o[c] = v;
    }
    const double g = cf.cpl * double(((x + y) & 1) ? -1 : 1);
    const double q1 = g * f1, q2 = g * f2, q3 = g * f3;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const double2 u = cen[2 * (1 - a)], w = cen[2 * (1 - a) + 1];
        o[2 * a].x += q3 * u.x + q1 * w.x + q2 * w.y;
        o[2 * a].y += q3 * u.y + q1 * w.y - q2 * w.x;
        o[2 * a + 1].x += q1 * u.x - q2 * u.y - q3 * w.x;
        o[2 * a + 1].y += q1 * u.y + q2 * u.x - q3 * w.y;
    }
}

__device__ __forceinline__ void mdag_site_lds(const double2* __restrict__ chi, int r, int x, int y, int s,
                                              const Lat& lat, const double* __restrict__ phi,
                                              const Coef<double>& cf, double ts, const double2 (&tt)[4],
                                              double2 (&o)[4], double2 (&cen)[4]) {
    const int vol = lat.vol;
    stencil_site_lds(chi, r, x, y, lat.L, phi[s], phi[vol + s], phi[2 * vol + s], cf, ts, tt, o, cen);
}

// The same operator with one workgroup per (vector, time slice, band) and no march: chi(tau) on
// the band's rows and the rows beside it into LDS, chi(tau - 1) at the thread's own element in
// registers.  A thread has one element of the band (the launch has R * L / 2 threads or more)
// and, for the first 2 L / 2 threads, one element of the rows beside it; the two stencils of
// its own element sit in one basic block, so their loads are in flight together.  Every slice of every band can then be
// resident at once, against the march's sequence of dependent steps; the slices before and after
// are formed again by their own workgroups (2 + 2 / R stencils per site instead of 1 + 2 / R),
// which the caches absorb.
__device__ __forceinline__ void tile_pos(const Lat& lat, const MarchPlan& mp, int wg, int& k, int& tau, int& x0,
                                         int& nr) {
    const int per_vec = lat.Lt * mp.nband;
    k = wg / per_vec;
    const int rem = wg - k * per_vec;
    tau = rem / mp.nband;
    const int band = rem - tau * mp.nband;
    x0 = band * mp.R;
    nr = lat.L - x0 < mp.R ? lat.L - x0 : mp.R;
}

__global__ __launch_bounds__(kMarchMaxThreads) void k_mdm2_tile(Lat lat, MarchPlan mp, const float2* __restrict__ in,
                                                               float2* __restrict__ out,
                                                               const float* __restrict__ phi, Coef<float> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    float2* chi = reinterpret_cast<float2*>(march_smem);      // [row][component][y]
    const int L = lat.L, vol = lat.vol, P = L / 2, rowc = 4 * L;
    int k, tau, x0, nr;
    tile_pos(lat, mp, xcd_remap(blockIdx.x, gridDim.x), k, tau, x0, nr);
    const size_t voff = size_t(k) * 4 * vol;
    const SrcPlain2 src{in + voff, vol};
    const int t = threadIdx.x, nint = nr * P;
    const bool own = t < nint, halo = t < 2 * P;
    const int e = own ? t : nint - 1;                 // a thread past the band repeats the last element
    const int lr = e / P, py = e - lr * P, x = x0 + lr, y = 2 * py;
    const int tm = tau == 0 ? lat.Lt - 1 : tau - 1;
    const int s = (tau * L + x) * L + y, sm = (tm * L + x) * L + y;
    const int hr = t < P ? 0 : nr + 1, hpy = t < P ? t : (halo ? t - P : 0);
    const int sh = (tau * L + wrap_row(x0 - 1 + hr, L)) * L + 2 * hpy;
    float4 a[4], ca[4], b[4], cb[4];
    dslash_pair<false, false>(src, phi, lat, cf, neighbours(lat, s), s, a, ca);     // chi(tau)
    dslash_pair<false, false>(src, phi, lat, cf, neighbours(lat, sm), sm, b, cb);   // chi(tau - 1)
    if (own) {
#pragma unroll
        for (int c = 0; c < 4; ++c) *reinterpret_cast<float4*>(chi + (lr + 1) * rowc + c * L + y) = a[c];
    }
    if (halo) {                                                                     // beside the band
        float4 h[4], ch[4];
        dslash_pair<false, false>(src, phi, lat, cf, neighbours(lat, sh), sh, h, ch);
#pragma unroll
        for (int c = 0; c < 4; ++c) *reinterpret_cast<float4*>(chi + hr * rowc + c * L + 2 * hpy) = h[c];
    }
    __syncthreads();
    if (own) {
        float4 o[4], cen[4];
        mdag_pair_lds(chi, lr + 1, x, y, s, lat, phi, cf, tau == 0 ? -1.f : 1.f, b, o, cen);
#pragma unroll
        for (int c = 0; c < 4; ++c) st4(out + voff, size_t(c) * vol + s, o[c]);
    }
}

__global__ __launch_bounds__(kMarchMaxThreads) void k_mdm_tile(Lat lat, MarchPlan mp, const double2* __restrict__ in,
                                                              double2* __restrict__ out,
                                                              const double* __restrict__ phi, Coef<double> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    double2* chi = reinterpret_cast<double2*>(march_smem);    // [row][component][y]
    const int L = lat.L, vol = lat.vol, rowc = 4 * L;
    int k, tau, x0, nr;
    tile_pos(lat, mp, xcd_remap(blockIdx.x, gridDim.x), k, tau, x0, nr);
    const size_t voff = size_t(k) * 4 * vol;
    const SrcPlain<double> src{in + voff, vol};
    const int t = threadIdx.x, nint = nr * L;
    const bool own = t < nint, halo = t < 2 * L;
    const int e = own ? t : nint - 1;
    const int lr = e / L, y = e - lr * L, x = x0 + lr;
    const int tm = tau == 0 ? lat.Lt - 1 : tau - 1;
    const int s = (tau * L + x) * L + y, sm = (tm * L + x) * L + y;
    const int hr = t < L ? 0 : nr + 1, hy = t < L ? t : (halo ? t - L : 0);
    const int sh = (tau * L + wrap_row(x0 - 1 + hr, L)) * L + hy;
    double2 a[4], ca[4], b[4], cb[4];
    dslash_site<double, false, false>(src, phi, lat, cf, neighbours(lat, s), s, a, ca);
    dslash_site<double, false, false>(src, phi, lat, cf, neighbours(lat, sm), sm, b, cb);
    if (own) {
#pragma unroll
        for (int c = 0; c < 4; ++c) chi[(lr + 1) * rowc + c * L + y] = a[c];
    }
    if (halo) {
        double2 h[4], ch[4];
        dslash_site<double, false, false>(src, phi, lat, cf, neighbours(lat, sh), sh, h, ch);
#pragma unroll
        for (int c = 0; c < 4; ++c) chi[hr * rowc + c * L + hy] = h[c];
    }
    __syncthreads();
    if (own) {
        double2 o[4], cen[4];
        mdag_site_lds(chi, lr + 1, x, y, s, lat, phi, cf, tau == 0 ? -1.0 : 1.0, b, o, cen);
#pragma unroll
        for (int c = 0; c < 4; ++c) out[voff + size_t(c) * vol + s] = o[c];
    }
}

// ------------------------------------------------------------------------------------
// CG step A as a march (one lattice, nearest-neighbour operator): the algebra of k_cg_a /
// k_cg_a2 (x += alpha p_old; p_new = z + beta p_old; t = M p_new; partial |t|^2), with the
// reuse along tau held on chip.  A workgroup owns a band of rows of one right-hand side and a
// segment of slices; one thread per element of the band and of the row on either side.  At
// each slice tau it forms p_new(tau + 1) on those rows from the z and p_old it loaded during
// the previous slice (so every value of z, p_old and x leaves HBM once, and the loads of the
// next slice are in flight while the current one is computed), writes p_new and x for its own
// rows, and forms t(tau) = A_tau p_new(tau) + s_tau p_new(tau + 1) from p_new(tau) in LDS
// (the spatial neighbours) and p_new(tau + 1) in registers (the time link).  The slice after a
// segment is formed again, not stored, by the segment before it.  Partials: one per workgroup
// (the consumer is told the count through CgCtl::nparts).
template <typename R>
__host__ __device__ inline size_t march_cg_lds(int Rrows, int L) {
    return 2 * size_t(Rrows + 2) * 4 * size_t(L) * sizeof(C2<R>);
}

// Most threads of a CG march workgroup (the band's elements and the two rows beside it).
constexpr int kMarchCgThreads = 512;

// The unit record of a march workgroup.
__device__ __forceinline__ UPos march_unit(const Lat& lat, int k, int blk, int nparts_in, int pstride) {
    UPos p;
    p.lat = lat;
    p.voff = size_t(k) * 4 * lat.vol;
    p.phioff = 0;
    p.k = k;
    p.blk = blk;
    p.bpr = nparts_in;
    p.part = k * pstride;
    p.pcoff = 0;
    p.mparts = p.rparts = 0;
    return p;
}

// Where a CG march workgroup works: its lattice, cut, band and segment, its unit record, and
// the partial count the previous kernel left per unit.
struct MarchWork {
    Lat lat;
    MarchPlan mp;
    MarchPos mpos;
    UPos pos;
    int nparts_in;
};

// One lattice: the vectors of a solve cut alike, workgroups vector-major.
struct MGeoOne {
    Lat lat;
    MarchPlan mp;
    int nparts_in;
    int pstride;
    __device__ __forceinline__ MarchWork at(int wg) const {
        MarchWork w;
        w.lat = lat;
        w.mp = mp;
        w.mpos = march_pos(lat, mp, wg);
        const int per_vec = mp.nseg * mp.nband;
        w.pos = march_unit(lat, w.mpos.k, wg - w.mpos.k * per_vec, nparts_in, pstride);
        w.nparts_in = nparts_in;
        return w;
    }
};

// A batch of lattices: blocks[wg] = (unit, workgroup within the unit), each unit with its own
// cut (step A's, or with ru the reliable update's FP64 one).
struct MGeoBatch {
    const UnitDesc* units;
    const int2* blocks;
    int ru;
    __device__ __forceinline__ MarchWork at(int wg) const {
        const int2 e = blocks[wg];
        const UnitDesc& u = units[e.x];
        MarchWork w;
        w.lat = u.lat;
        w.mp = ru ? u.rmp : u.mp;
        w.mpos = march_pos_in(u.lat, w.mp, e.x, e.y);
        w.pos = GeoBatch{units, blocks}.unit(e.x, e.y);
        w.nparts_in = u.bpr;
        return w;
    }
};

template <class MG, bool NN2>
__global__ __launch_bounds__(kMarchCgThreads) void k_cg_a2_march(CgCtl ctl, MG mg, CgVecs<float> v,
                                                                 const float* __restrict__ phi_base, Coef<float> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    const MarchWork w = mg.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = w.lat;
    const MarchPlan& mp = w.mp;
    const MarchPos& mpos = w.mpos;
    const UPos& pos = w.pos;
    const float* phi = phi_base + pos.phioff;
    const int L = lat.L, Lt = lat.Lt, LL = lat.LL, vol = lat.vol, P = L / 2, rowc = 4 * L;
    constexpr int H = NN2 ? 2 : 1;    // rows beside the band on either side
    const size_t off = pos.voff;
    const float2* z = v.z + off;
    // this thread's element: row lr of the band buffer (0 and nr + 1 are the rows beside the band)
    const int e = threadIdx.x, nh = (mpos.nr + 2 * H) * P;
    const bool act = e < nh;
    const int lr = act ? e / P : 0, py = act ? e - lr * P : 0, y = 2 * py;
    const int xrow = wrap_row(mpos.x0 - H + lr, L);
    const bool inner = act && lr >= H && lr < mpos.nr + H;
    const int ro = xrow * L + y;                      // offset of the element within a slice
    const int t0 = mpos.t0, t1 = mpos.t1;
    float4 rz[4], rp[4], rx[4], rq[4];
    float2 f1 = make_float2(0.f, 0.f), f2 = f1, f3 = f1;
    auto load_phi = [&](int tq) {
        if (inner) {
            const size_t i = size_t(tq) * LL + ro;
            f1 = *reinterpret_cast<const float2*>(phi + i);
            f2 = *reinterpret_cast<const float2*>(phi + vol + i);
            f3 = *reinterpret_cast<const float2*>(phi + 2 * vol + i);
        }
    };
    // the first slice's z and phi do not depend on the record: in flight while it is reduced
    if (act) {
#pragma unroll
        for (int c = 0; c < 4; ++c) rz[c] = ld4(z, size_t(c) * vol + size_t(t0) * LL + ro);
    }
    load_phi(t0);
    cg_finalize(ctl, pos, w.nparts_in);
    const CgState& S = cg_shared();
    if (S.mode != CG_ACTIVE) {
        cg_publish(ctl, pos);
        return;
    }
    const float alpha = float(S.alpha), alpha_old = float(S.alpha_old), beta = float(S.beta);
    const bool fold = S.alpha_old != 0.0;   // x += both pending steps this iteration (see k_cg_a)
    const double defer = S.alpha;
    const int pb = S.pbuf;
    const float2* pin = (pb ? v.p1 : v.p0) + off;
    float2* pout = (pb ? v.p0 : v.p1) + off;
    float2* x = v.x + off;
    float2* t = v.t + off;
    float2* cur = reinterpret_cast<float2*>(march_smem);
    float2* nxt = cur + size_t(mp.R + 2 * H) * rowc;
    // slice tq of z and p_old (and x and the older direction when the solution update is due);
    // the slice after the segment (own false) is needed only at the band's own sites, for the
    // time link, and its solution update belongs to the next segment
    auto load_slab = [&](int tq, bool with_z, bool own) {
        if (own ? act : inner) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = size_t(c) * vol + size_t(tq) * LL + ro;
                if (with_z) rz[c] = ld4(z, i);
                rp[c] = ld4(pin, i);
            }
        }
        if (inner && fold && own) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = size_t(c) * vol + size_t(tq) * LL + ro;
                rx[c] = ld4(x, i);
                rq[c] = ld4(pout, i);
            }
        }
    };
    // p_new at slice tq from the loaded z, p_old (into buf, and stored with the x update when own)
    auto form = [&](int tq, float2* buf, bool own, float4 (&pn)[4]) {
#pragma unroll
        for (int c = 0; c < 4; ++c) pn[c] = f4axpy(beta, rp[c], rz[c]);
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) *reinterpret_cast<float4*>(buf + lr * rowc + c * L + y) = pn[c];
        }
        if (inner && own) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = size_t(c) * vol + size_t(tq) * LL + ro;
                st4(pout, i, pn[c]);
                if (fold) st4(x, i, f4axpy(alpha, rp[c], f4axpy(alpha_old, rq[c], rx[c])));
            }
        }
    };
    float4 pn[4];
    load_slab(t0, false, true);
    form(t0, cur, true, pn);
    load_slab(t0 + 1 == Lt ? 0 : t0 + 1, true, t0 + 1 < t1);
    double part = 0.0;
    for (int tau = t0; tau < t1; ++tau) {
        const int tn = tau + 1 == Lt ? 0 : tau + 1;
        const bool own_next = tau + 1 < t1;
        float4 pnx[4];
        form(tn, nxt, own_next, pnx);
        const float2 g1 = f1, g2 = f2, g3 = f3;
        if (own_next) {
            load_slab(tn + 1 == Lt ? 0 : tn + 1, true, tau + 2 < t1);
            load_phi(tn);
        }
        __syncthreads();
        if (inner) {
            float4 o[4], cen[4];
            stencil_pair_lds<NN2>(cur, lr, xrow, y, L, g1, g2, g3, cf, tau == Lt - 1 ? -1.f : 1.f, pnx, o, cen);
            float acc = 0.f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                st4(t, size_t(c) * vol + size_t(tau) * LL + ro, o[c]);
                acc += f4norm2(o[c]);
            }
            part += double(acc);
        }
        __syncthreads();
        float2* sw = cur;
        cur = nxt;
        nxt = sw;
    }
    store_partial(ctl, PEND_TT, pos, part);
    if (threadIdx.x == 0) {
        CgState& W = cg_shared();
        W.alpha_old = fold ? 0.0 : defer;
        W.alpha = 0.0;
        W.pbuf = 1 - pb;
        W.pending = PEND_TT;
    }
    cg_publish(ctl, pos);
}

template <class MG, bool NN2>
__global__ __launch_bounds__(kMarchCgThreads) void k_cg_a_march(CgCtl ctl, MG mg, CgVecs<double> v,
                                                                const double* __restrict__ phi_base, Coef<double> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    const MarchWork w = mg.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = w.lat;
    const MarchPlan& mp = w.mp;
    const MarchPos& mpos = w.mpos;
    const UPos& pos = w.pos;
    const double* phi = phi_base + pos.phioff;
    const int L = lat.L, Lt = lat.Lt, LL = lat.LL, vol = lat.vol, rowc = 4 * L;
    constexpr int H = NN2 ? 2 : 1;    // rows beside the band on either side
    const size_t off = pos.voff;
    const double2* z = v.z + off;
    const int e = threadIdx.x, nh = (mpos.nr + 2 * H) * L;
    const bool act = e < nh;
    const int lr = act ? e / L : 0, y = act ? e - lr * L : 0;
    const int xrow = wrap_row(mpos.x0 - H + lr, L);
    const bool inner = act && lr >= H && lr < mpos.nr + H;
    const int ro = xrow * L + y;
    const int t0 = mpos.t0, t1 = mpos.t1;
    double2 rz[4], rp[4], rx[4], rq[4];
    double f1 = 0.0, f2 = 0.0, f3 = 0.0;
    auto load_phi = [&](int tq) {
        if (inner) {
            const size_t i = size_t(tq) * LL + ro;
            f1 = phi[i];
            f2 = phi[vol + i];
            f3 = phi[2 * vol + i];
        }
    };
    // the first slice's z and phi do not depend on the record: in flight while it is reduced
    if (act) {
#pragma unroll
        for (int c = 0; c < 4; ++c) rz[c] = z[size_t(c) * vol + size_t(t0) * LL + ro];
    }
    load_phi(t0);
    cg_finalize(ctl, pos, w.nparts_in);
    const CgState& S = cg_shared();
    if (S.mode != CG_ACTIVE) {
        cg_publish(ctl, pos);
        return;
    }
    const double alpha = S.alpha, alpha_old = S.alpha_old, beta = S.beta;
    const bool fold = alpha_old != 0.0;     // x += both pending steps this iteration (see k_cg_a)
    const double defer = S.alpha;
    const int pb = S.pbuf;
    const double2* pin = (pb ? v.p1 : v.p0) + off;
    double2* pout = (pb ? v.p0 : v.p1) + off;
    double2* x = v.x + off;
    double2* t = v.t + off;
    double2* cur = reinterpret_cast<double2*>(march_smem);
    double2* nxt = cur + size_t(mp.R + 2 * H) * rowc;
    // slice tq of z and p_old (and x and the older direction when the solution update is due);
    // the slice after the segment (own false) is needed only at the band's own sites, for the
    // time link, and its solution update belongs to the next segment
    auto load_slab = [&](int tq, bool with_z, bool own) {
        if (own ? act : inner) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = size_t(c) * vol + size_t(tq) * LL + ro;
                if (with_z) rz[c] = z[i];
                rp[c] = pin[i];
            }
        }
        if (inner && fold && own) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = size_t(c) * vol + size_t(tq) * LL + ro;
                rx[c] = x[i];
                rq[c] = pout[i];
            }
        }
    };
    auto form = [&](int tq, double2* buf, bool own, double2 (&pn)[4]) {
#pragma unroll
        for (int c = 0; c < 4; ++c) pn[c] = axpy<double>(beta, rp[c], rz[c]);
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) buf[lr * rowc + c * L + y] = pn[c];
        }
        if (inner && own) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = size_t(c) * vol + size_t(tq) * LL + ro;
                pout[i] = pn[c];
                if (fold) x[i] = axpy<double>(alpha, rp[c], axpy<double>(alpha_old, rq[c], rx[c]));
            }
        }
    };
    double2 pn[4];
    load_slab(t0, false, true);
    form(t0, cur, true, pn);
    load_slab(t0 + 1 == Lt ? 0 : t0 + 1, true, t0 + 1 < t1);
    double part = 0.0;
    for (int tau = t0; tau < t1; ++tau) {
        const int tn = tau + 1 == Lt ? 0 : tau + 1;
        const bool own_next = tau + 1 < t1;
        double2 pnx[4];
        form(tn, nxt, own_next, pnx);
        const double g1 = f1, g2 = f2, g3 = f3;
        if (own_next) {
            load_slab(tn + 1 == Lt ? 0 : tn + 1, true, tau + 2 < t1);
            load_phi(tn);
        }
        __syncthreads();
        if (inner) {
            double2 o[4], cen[4];
            stencil_site_lds<NN2>(cur, lr, xrow, y, L, g1, g2, g3, cf, tau == Lt - 1 ? -1.0 : 1.0, pnx, o, cen);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                t[size_t(c) * vol + size_t(tau) * LL + ro] = o[c];
                part += norm2<double>(o[c]);
            }
        }
        __syncthreads();
        double2* sw = cur;
        cur = nxt;
        nxt = sw;
    }
    store_partial(ctl, PEND_TT, pos, part);
    if (threadIdx.x == 0) {
        CgState& W = cg_shared();
        W.alpha_old = fold ? 0.0 : defer;
        W.alpha = 0.0;
        W.pbuf = 1 - pb;
        W.pending = PEND_TT;
    }
    cg_publish(ctl, pos);
}

// ------------------------------------------------------------------------------------
// CG step B as a march with step A's cut: r -= alpha_k M^dagger t, partial |r|^2 (PEND_RR, one
// per workgroup; the next kernel is told the count).  M^dagger needs t(tau - 1) only at the
// site itself, kept in registers from the slice before; LDS holds t(tau) on the band's rows and
// the rows beside it, alternating between two buffers (one barrier per slice), the next
// slice's loads in flight meanwhile.  The arithmetic per site is that of k_cg_b / k_cg_b2.
template <class MG, bool NN2>
__global__ __launch_bounds__(kMarchCgThreads) void k_cg_b2_march(CgCtl ctl, MG mg, CgVecs<float> v,
                                                                 const float* __restrict__ phi_base, Coef<float> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    const MarchWork w = mg.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = w.lat;
    const MarchPlan& mp = w.mp;
    const MarchPos& mpos = w.mpos;
    const UPos& pos = w.pos;
    const float* phi = phi_base + pos.phioff;
    const int L = lat.L, Lt = lat.Lt, LL = lat.LL, vol = lat.vol, P = L / 2, rowc = 4 * L;
    constexpr int H = NN2 ? 2 : 1;
    const size_t off = pos.voff;
    const float2* tin = v.t + off;
    float2* r = v.r + off;
    float2* buf0 = reinterpret_cast<float2*>(march_smem);
    float2* buf1 = buf0 + size_t(mp.R + 2 * H) * rowc;
    const int e = threadIdx.x, nh = (mpos.nr + 2 * H) * P;
    const bool act = e < nh;
    const int lr = act ? e / P : 0, py = act ? e - lr * P : 0, y = 2 * py;
    const int xrow = wrap_row(mpos.x0 - H + lr, L);
    const bool inner = act && lr >= H && lr < mpos.nr + H;
    const int ro = xrow * L + y;
    // defined on every thread (a conditionally loaded array would be kept in scratch memory)
    float4 rv[4], rs[4], prev[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rv[c] = rs[c] = prev[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    float2 f1 = make_float2(0.f, 0.f), f2 = f1, f3 = f1;
    auto load_slab = [&](int tq) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) rv[c] = ld4(tin, size_t(c) * vol + size_t(tq) * LL + ro);
        }
    };
    auto load_site = [&](int tq) {
        if (inner) {
            const size_t i = size_t(tq) * LL + ro;
            f1 = *reinterpret_cast<const float2*>(phi + i);
            f2 = *reinterpret_cast<const float2*>(phi + vol + i);
            f3 = *reinterpret_cast<const float2*>(phi + 2 * vol + i);
#pragma unroll
            for (int c = 0; c < 4; ++c) rs[c] = ld4(r, size_t(c) * vol + i);
        }
    };
    const int t0 = mpos.t0, t1 = mpos.t1;
    if (inner) {
        const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) prev[c] = ld4(tin, size_t(c) * vol + size_t(tp) * LL + ro);
    }
    // the first slice's loads do not depend on the record: in flight while it is reduced
    load_slab(t0);
    load_site(t0);
    cg_finalize(ctl, pos, w.nparts_in);
    const CgState& S = cg_shared();
    if (S.mode != CG_ACTIVE) {
        cg_publish(ctl, pos);
        return;
    }
    const float alpha = float(S.alpha_cur);
    double part = 0.0;
    for (int tau = t0; tau < t1; ++tau) {
        float2* cur = (tau - t0) & 1 ? buf1 : buf0;
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) *reinterpret_cast<float4*>(cur + lr * rowc + c * L + y) = rv[c];
        }
        const float2 g1 = f1, g2 = f2, g3 = f3;
        float4 rt[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) rt[c] = rs[c];
        if (tau + 1 < t1) {
            load_slab(tau + 1);
            load_site(tau + 1);
        }
        __syncthreads();
        if (inner) {
            float4 o[4], cen[4];
            stencil_pair_lds<NN2>(cur, lr, xrow, y, L, g1, g2, g3, cf, tau == 0 ? -1.f : 1.f, prev, o, cen);
            float acc = 0.f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float4 rn = f4axpy(-alpha, o[c], rt[c]);
                st4(r, size_t(c) * vol + size_t(tau) * LL + ro, rn);
                acc += f4norm2(rn);
                prev[c] = cen[c];
            }
            part += double(acc);
        }
    }
    store_partial(ctl, PEND_RR, pos, part);
    if (threadIdx.x == 0) cg_shared().pending = PEND_RR;
    cg_publish(ctl, pos);
}

template <class MG, bool NN2>
__global__ __launch_bounds__(kMarchCgThreads) void k_cg_b_march(CgCtl ctl, MG mg, CgVecs<double> v,
                                                                const double* __restrict__ phi_base, Coef<double> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    const MarchWork w = mg.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = w.lat;
    const MarchPlan& mp = w.mp;
    const MarchPos& mpos = w.mpos;
    const UPos& pos = w.pos;
    const double* phi = phi_base + pos.phioff;
    const int L = lat.L, Lt = lat.Lt, LL = lat.LL, vol = lat.vol, rowc = 4 * L;
    constexpr int H = NN2 ? 2 : 1;
    const size_t off = pos.voff;
    const double2* tin = v.t + off;
    double2* r = v.r + off;
    double2* buf0 = reinterpret_cast<double2*>(march_smem);
    double2* buf1 = buf0 + size_t(mp.R + 2 * H) * rowc;
    const int e = threadIdx.x, nh = (mpos.nr + 2 * H) * L;
    const bool act = e < nh;
    const int lr = act ? e / L : 0, y = act ? e - lr * L : 0;
    const int xrow = wrap_row(mpos.x0 - H + lr, L);
    const bool inner = act && lr >= H && lr < mpos.nr + H;
    const int ro = xrow * L + y;
    double2 rv[4], rs[4], prev[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rv[c] = rs[c] = prev[c] = make_double2(0.0, 0.0);
    double f1 = 0.0, f2 = 0.0, f3 = 0.0;
    auto load_slab = [&](int tq) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) rv[c] = tin[size_t(c) * vol + size_t(tq) * LL + ro];
        }
    };
    auto load_site = [&](int tq) {
        if (inner) {
            const size_t i = size_t(tq) * LL + ro;
            f1 = phi[i];
            f2 = phi[vol + i];
            f3 = phi[2 * vol + i];
#pragma unroll
            for (int c = 0; c < 4; ++c) rs[c] = r[size_t(c) * vol + i];
        }
    };
    const int t0 = mpos.t0, t1 = mpos.t1;
    if (inner) {
        const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) prev[c] = tin[size_t(c) * vol + size_t(tp) * LL + ro];
    }
    // the first slice's loads do not depend on the record: in flight while it is reduced
    load_slab(t0);
    load_site(t0);
    cg_finalize(ctl, pos, w.nparts_in);
    const CgState& S = cg_shared();
    if (S.mode != CG_ACTIVE) {
        cg_publish(ctl, pos);
        return;
    }
    const double alpha = S.alpha_cur;
    double part = 0.0;
    for (int tau = t0; tau < t1; ++tau) {
        double2* cur = (tau - t0) & 1 ? buf1 : buf0;
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) cur[lr * rowc + c * L + y] = rv[c];
        }
        const double g1 = f1, g2 = f2, g3 = f3;
        double2 rt[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) rt[c] = rs[c];
        if (tau + 1 < t1) {
            load_slab(tau + 1);
            load_site(tau + 1);
        }
        __syncthreads();
        if (inner) {
            double2 o[4], cen[4];
            stencil_site_lds<NN2>(cur, lr, xrow, y, L, g1, g2, g3, cf, tau == 0 ? -1.0 : 1.0, prev, o, cen);
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double2 rn = axpy<double>(-alpha, o[c], rt[c]);
                r[size_t(c) * vol + size_t(tau) * LL + ro] = rn;
                acc += norm2<double>(rn);
                prev[c] = cen[c];
            }
            part += acc;
        }
    }
    store_partial(ctl, PEND_RR, pos, part);
    if (threadIdx.x == 0) cg_shared().pending = PEND_RR;
    cg_publish(ctl, pos);
}

// ------------------------------------------------------------------------------------
// The FP64 reliable update of the conjugate-gradient solve (after the elementwise fold of the
// pending step into x64) as two marches with the FP64 step-A march's cut and thread layout:
// t64 = M x64, then r = b - M^dagger t64 with the FP64 partial |r|^2.  They replace the two
// FP64 tile stencils, which read their inputs again from L2 for every neighbour.

// t64 = M x64 for the units in `filter` (Eq. 17): each slice, x64(tau + 1) on the band's rows
// and the rows beside it goes to LDS while M at tau is formed from the previous slice's copy,
// the time link taken from the thread's own element of tau + 1.  Reads x64 and phi once (plus
// the rows beside each band and one slice per segment), writes t64 once.
template <class MG>
__global__ __launch_bounds__(kMarchCgThreads) void k_ru_apply_march(CgCtl ctl, MG mg, const double2* __restrict__ x64,
                                                                    double2* __restrict__ t64,
                                                                    const double* __restrict__ phi_base,
                                                                    Coef<double> cf, int filter) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    const MarchWork w = mg.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = w.lat;
    const MarchPlan& mp = w.mp;
    const MarchPos& mpos = w.mpos;
    const UPos& pos = w.pos;
    const double* phi = phi_base + pos.phioff;
    const int L = lat.L, Lt = lat.Lt, LL = lat.LL, vol = lat.vol, rowc = 4 * L;
    cg_finalize(ctl, pos, w.nparts_in);
    const int mode = cg_shared().mode;
    cg_publish(ctl, pos);
    if (!((1 << mode) & filter)) return;
    const size_t off = pos.voff;
    const double2* xin = x64 + off;
    double2* t = t64 + off;
    double2* cur = reinterpret_cast<double2*>(march_smem);
    double2* nxt = cur + size_t(mp.R + 2) * rowc;
    const int e = threadIdx.x, nh = (mpos.nr + 2) * L;
    const bool act = e < nh;
    const int lr = act ? e / L : 0, y = act ? e - lr * L : 0;
    const int xrow = wrap_row(mpos.x0 - 1 + lr, L);
    const bool inner = act && lr >= 1 && lr <= mpos.nr;
    const int ro = xrow * L + y;
    double2 rv[4];
    double f1 = 0.0, f2 = 0.0, f3 = 0.0;
    auto load_slab = [&](int tq) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) rv[c] = xin[size_t(c) * vol + size_t(tq) * LL + ro];
        }
    };
    auto load_phi = [&](int tq) {
        if (inner) {
            const size_t i = size_t(tq) * LL + ro;
            f1 = phi[i];
            f2 = phi[vol + i];
            f3 = phi[2 * vol + i];
        }
    };
    auto place = [&](double2* buf, double2 (&v)[4]) {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = rv[c];
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) buf[lr * rowc + c * L + y] = v[c];
        }
    };
    const int t0 = mpos.t0, t1 = mpos.t1;
    double2 v0[4];
    load_slab(t0);
    place(cur, v0);
    load_slab(t0 + 1 == Lt ? 0 : t0 + 1);
    load_phi(t0);
    for (int tau = t0; tau < t1; ++tau) {
        const int tn = tau + 1 == Lt ? 0 : tau + 1;
        double2 vn[4];
        place(nxt, vn);
        const double g1 = f1, g2 = f2, g3 = f3;
        if (tau + 1 < t1) {
            load_slab(tn + 1 == Lt ? 0 : tn + 1);
            load_phi(tn);
        }
        __syncthreads();
        if (inner) {
            double2 o[4], cen[4];
            stencil_site_lds(cur, lr, xrow, y, L, g1, g2, g3, cf, tau == Lt - 1 ? -1.0 : 1.0, vn, o, cen);
#pragma unroll
            for (int c = 0; c < 4; ++c) t[size_t(c) * vol + size_t(tau) * LL + ro] = o[c];
        }
        __syncthreads();
        double2* sw = cur;
        cur = nxt;
        nxt = sw;
    }
}

// r = b - M^dagger t64 in FP64, stored in the Krylov precision, with the FP64 partial |r|^2
// (PEND_RU, one per workgroup) for the units in `filter`.  M^dagger needs t64(tau - 1) only at
// the site itself: each slice's own element is kept in registers for the next.  LDS holds
// t64(tau) on the band's rows and the rows beside it, alternating between two buffers so that
// one barrier per slice suffices; the next slice's loads are in flight meanwhile.
template <typename R, class MG>
__global__ __launch_bounds__(kMarchCgThreads) void k_ru_resid_march(CgCtl ctl, MG mg, const double2* __restrict__ b,
                                                                    const double2* __restrict__ t64,
                                                                    const double* __restrict__ phi_base,
                                                                    Coef<double> cf, C2<R>* __restrict__ r, int filter) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    const MarchWork w = mg.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = w.lat;
    const MarchPlan& mp = w.mp;
    const MarchPos& mpos = w.mpos;
    const UPos& pos = w.pos;
    const double* phi = phi_base + pos.phioff;
    const int L = lat.L, Lt = lat.Lt, LL = lat.LL, vol = lat.vol, rowc = 4 * L;
    cg_finalize(ctl, pos, w.nparts_in);
    if (!((1 << cg_shared().mode) & filter)) {
        cg_publish(ctl, pos);
        return;
    }
    const size_t off = pos.voff;
    const double2* tin = t64 + off;
    const double2* bb = b + off;
    C2<R>* rr = r + off;
    double2* buf0 = reinterpret_cast<double2*>(march_smem);
    double2* buf1 = buf0 + size_t(mp.R + 2) * rowc;
    const int e = threadIdx.x, nh = (mpos.nr + 2) * L;
    const bool act = e < nh;
    const int lr = act ? e / L : 0, y = act ? e - lr * L : 0;
    const int xrow = wrap_row(mpos.x0 - 1 + lr, L);
    const bool inner = act && lr >= 1 && lr <= mpos.nr;
    const int ro = xrow * L + y;
    // defined on every thread (a conditionally loaded array would be kept in scratch memory)
    double2 rv[4], bv[4], prev[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rv[c] = bv[c] = prev[c] = make_double2(0.0, 0.0);
    double f1 = 0.0, f2 = 0.0, f3 = 0.0;
    auto load_slab = [&](int tq) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) rv[c] = tin[size_t(c) * vol + size_t(tq) * LL + ro];
        }
    };
    auto load_site = [&](int tq) {
        if (inner) {
            const size_t i = size_t(tq) * LL + ro;
            f1 = phi[i];
            f2 = phi[vol + i];
            f3 = phi[2 * vol + i];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = bb[size_t(c) * vol + i];
        }
    };
    const int t0 = mpos.t0, t1 = mpos.t1;
    if (inner) {
        const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) prev[c] = tin[size_t(c) * vol + size_t(tp) * LL + ro];
    }
    load_slab(t0);
    load_site(t0);
    double part = 0.0;
    for (int tau = t0; tau < t1; ++tau) {
        double2* cur = (tau - t0) & 1 ? buf1 : buf0;
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) cur[lr * rowc + c * L + y] = rv[c];
        }
        const double g1 = f1, g2 = f2, g3 = f3;
        double2 bt[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bt[c] = bv[c];
        if (tau + 1 < t1) {
            load_slab(tau + 1);
            load_site(tau + 1);
        }
        __syncthreads();
        if (inner) {
            double2 o[4], cen[4];
            stencil_site_lds(cur, lr, xrow, y, L, g1, g2, g3, cf, tau == 0 ? -1.0 : 1.0, prev, o, cen);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double2 d = sub<double>(bt[c], o[c]);
                part += norm2<double>(d);
                rr[size_t(c) * vol + size_t(tau) * LL + ro] = mk<R>(R(d.x), R(d.y));
                prev[c] = cen[c];
            }
        }
    }
    store_partial(ctl, PEND_RU, pos, part);
    if (threadIdx.x == 0) cg_shared().pending = PEND_RU;
    cg_publish(ctl, pos);
}

// ------------------------------------------------------------------------------------
// M^dagger M in one pass as a march with the loads one slice ahead (the structure of the CG
// step-A march): a workgroup owns a band of R rows of one vector and the two rows on either
// side of it, and walks a segment of slices.  chi(tau) = A_tau psi(tau) + s_tau psi(tau + 1) is
// formed on the R + 2 rows that M^dagger reaches, and (M^dagger chi)(tau) = A_tau chi(tau) +
// s_{tau-1} chi(tau - 1) on the band's R rows, chi(tau - 1) kept in registers.  The two are
// software-pipelined: while slice tau's M^dagger reads chi(tau) from LDS, chi(tau + 1) is formed
// from psi(tau + 1) in LDS and written to a second chi buffer, and psi(tau + 2) to a second psi
// buffer, so one barrier per slice separates every LDS write from its reads (two slices of psi
// on R + 4 rows and two of chi on R + 2 in LDS); the next slice's psi and phi are loaded while
// the current one is computed.  A segment starts by forming chi(t0 - 1) at the band's rows and
// chi(t0).  HBM: psi and phi read once (plus the rows beside each band, which its neighbours
// read too, and one slice per segment), the result written once.
// Most threads of a one-pass M^dagger M march workgroup (one per element of its rows).  The
// kernels are instantiated for at most 512 threads (up to 256 VGPRs each), 768 (168 VGPRs,
// enough for both precisions) and 1024 (128 VGPRs, a few spilled): a band takes the smallest
// that holds it.
constexpr int kMdmMidThreads = 768;
constexpr int kMdmMarchThreads = 1024;

template <typename R>
__host__ __device__ inline size_t mdm_march_lds(int Rrows, int L) {
    return size_t(4 * Rrows + 12) * 4 * size_t(L) * sizeof(C2<R>);
}

template <int MAXT>
__global__ __launch_bounds__(MAXT) void k_mdm2_march(Lat lat, MarchPlan mp, const float2* __restrict__ in,
                                                                float2* __restrict__ out,
                                                                const float* __restrict__ phi, Coef<float> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    const int L = lat.L, Lt = lat.Lt, LL = lat.LL, vol = lat.vol, P = L / 2, rowc = 4 * L;
    const MarchPos mpos = march_pos(lat, mp, xcd_remap(blockIdx.x, gridDim.x));
    const size_t voff = size_t(mpos.k) * 4 * vol;
    const float2* psi = in + voff;
    float2* dst = out + voff;
    // psi of a slice (rows x0 - 2 .. x0 + nr + 1) and chi of a slice (rows x0 - 1 .. x0 + nr), two
    // of each
    float2* pa = reinterpret_cast<float2*>(march_smem);
    float2* pb = pa + size_t(mp.R + 4) * rowc;
    float2* ca = pb + size_t(mp.R + 4) * rowc;
    float2* cb = ca + size_t(mp.R + 2) * rowc;
    const int e = threadIdx.x, nh = (mpos.nr + 4) * P;
    const bool act = e < nh;
    const int lr = act ? e / P : 0, py = act ? e - lr * P : 0, y = 2 * py;
    const int xrow = wrap_row(mpos.x0 - 2 + lr, L);
    const bool chirow = act && lr >= 1 && lr <= mpos.nr + 2;     // M psi is formed here
    const bool inner = act && lr >= 2 && lr <= mpos.nr + 1;      // M^dagger M psi is written here
    const int ro = xrow * L + y;
    float4 rv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rv[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    float2 f1 = make_float2(0.f, 0.f), f2 = f1, f3 = f1;
    auto load_psi = [&](int tq) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) rv[c] = ld4(psi, size_t(c) * vol + size_t(tq) * LL + ro);
        }
    };
    auto load_phi = [&](int tq) {
        if (chirow) {
            const size_t i = size_t(tq) * LL + ro;
            f1 = *reinterpret_cast<const float2*>(phi + i);
            f2 = *reinterpret_cast<const float2*>(phi + vol + i);
            f3 = *reinterpret_cast<const float2*>(phi + 2 * vol + i);
        }
    };
    auto put = [&](float2* buf, const float4 (&v)[4]) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) *reinterpret_cast<float4*>(buf + lr * rowc + c * L + y) = v[c];
        }
    };
    const int t0 = mpos.t0, t1 = mpos.t1;
    const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
    auto wrapt = [&](int t) { return t >= Lt ? t - Lt : t; };
    float4 prev[4], own[4], cen[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) prev[c] = own[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    // chi(t0 - 1) at the band's rows, from psi(t0 - 1) (LDS) and psi(t0) (own site)
    load_psi(tm);
    load_phi(tm);
    put(pa, rv);
    const float2 h1 = f1, h2 = f2, h3 = f3;
    load_psi(t0);
    __syncthreads();
    float4 pv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) pv[c] = rv[c];
    put(pb, pv);
    load_psi(wrapt(t0 + 1));
    load_phi(t0);
    if (inner) stencil_pair_lds(pa, lr, xrow, y, L, h1, h2, h3, cf, tm == Lt - 1 ? -1.f : 1.f, pv, prev, cen);
    __syncthreads();
    // chi(t0) on the R + 2 rows, from psi(t0) (LDS) and psi(t0 + 1) (own site)
#pragma unroll
    for (int c = 0; c < 4; ++c) pv[c] = rv[c];
    float2 c1 = f1, c2 = f2, c3 = f3;
    put(pa, pv);
    if (t0 + 1 < t1) {
        load_psi(wrapt(t0 + 2));
        load_phi(t0 + 1);
    }
    if (chirow) {
        stencil_pair_lds(pb, lr, xrow, y, L, c1, c2, c3, cf, t0 == Lt - 1 ? -1.f : 1.f, pv, own, cen);
#pragma unroll
        for (int c = 0; c < 4; ++c) *reinterpret_cast<float4*>(ca + (lr - 1) * rowc + c * L + y) = own[c];
    }
    __syncthreads();
    // slice tau: psi(tau + 1) and chi(tau) are in LDS; chi(tau + 1) and (M^dagger chi)(tau) do not
    // depend on each other, so one barrier per slice separates the writes from the next reads
    float2 *pcur = pa, *pnxt = pb, *ccur = ca, *cnxt = cb;
    for (int tau = t0; tau < t1; ++tau) {
        const bool more = tau + 1 < t1;
        float4 pn[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) pn[c] = rv[c];                  // psi(tau + 2)
        const float2 g1 = f1, g2 = f2, g3 = f3;                      // phi(tau + 1)
        if (tau + 2 < t1) {
            load_psi(wrapt(tau + 3));
            load_phi(tau + 2);
        }
        if (more) {
            put(pnxt, pn);
            if (chirow) {
                stencil_pair_lds(pcur, lr, xrow, y, L, g1, g2, g3, cf, tau + 1 == Lt - 1 ? -1.f : 1.f, pn, own, cen);
#pragma unroll
                for (int c = 0; c < 4; ++c) *reinterpret_cast<float4*>(cnxt + (lr - 1) * rowc + c * L + y) = own[c];
            }
        }
        if (inner) {
            float4 o[4];
            stencil_pair_lds(ccur, lr - 1, xrow, y, L, c1, c2, c3, cf, tau == 0 ? -1.f : 1.f, prev, o, cen);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                st4(dst, size_t(c) * vol + size_t(tau) * LL + ro, o[c]);
                prev[c] = cen[c];
            }
        }
        c1 = g1;
        c2 = g2;
        c3 = g3;
        __syncthreads();
        float2* sw = pcur;
        pcur = pnxt;
        pnxt = sw;
        sw = ccur;
        ccur = cnxt;
        cnxt = sw;
    }
}

template <int MAXT>
__global__ __launch_bounds__(MAXT) void k_mdm_march(Lat lat, MarchPlan mp, const double2* __restrict__ in,
                                                               double2* __restrict__ out,
                                                               const double* __restrict__ phi, Coef<double> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    const int L = lat.L, Lt = lat.Lt, LL = lat.LL, vol = lat.vol, rowc = 4 * L;
    const MarchPos mpos = march_pos(lat, mp, xcd_remap(blockIdx.x, gridDim.x));
    const size_t voff = size_t(mpos.k) * 4 * vol;
    const double2* psi = in + voff;
    double2* dst = out + voff;
    double2* pa = reinterpret_cast<double2*>(march_smem);
    double2* pb = pa + size_t(mp.R + 4) * rowc;
    double2* ca = pb + size_t(mp.R + 4) * rowc;
    double2* cb = ca + size_t(mp.R + 2) * rowc;
    const int e = threadIdx.x, nh = (mpos.nr + 4) * L;
    const bool act = e < nh;
    const int lr = act ? e / L : 0, y = act ? e - lr * L : 0;
    const int xrow = wrap_row(mpos.x0 - 2 + lr, L);
    const bool chirow = act && lr >= 1 && lr <= mpos.nr + 2;
    const bool inner = act && lr >= 2 && lr <= mpos.nr + 1;
    const int ro = xrow * L + y;
    double2 rv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rv[c] = make_double2(0.0, 0.0);
    double f1 = 0.0, f2 = 0.0, f3 = 0.0;
    auto load_psi = [&](int tq) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) rv[c] = psi[size_t(c) * vol + size_t(tq) * LL + ro];
        }
    };
    auto load_phi = [&](int tq) {
        if (chirow) {
            const size_t i = size_t(tq) * LL + ro;
            f1 = phi[i];
            f2 = phi[vol + i];
            f3 = phi[2 * vol + i];
        }
    };
    auto put = [&](double2* buf, const double2 (&v)[4]) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) buf[lr * rowc + c * L + y] = v[c];
        }
    };
    const int t0 = mpos.t0, t1 = mpos.t1;
    const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
    auto wrapt = [&](int t) { return t >= Lt ? t - Lt : t; };
    double2 prev[4], own[4], cen[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) prev[c] = own[c] = make_double2(0.0, 0.0);
    // chi(t0 - 1) at the band's rows, from psi(t0 - 1) (LDS) and psi(t0) (own site)
    load_psi(tm);
    load_phi(tm);
    put(pa, rv);
    const double h1 = f1, h2 = f2, h3 = f3;
    load_psi(t0);
    __syncthreads();
    double2 pv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) pv[c] = rv[c];
    put(pb, pv);
    load_psi(wrapt(t0 + 1));
    load_phi(t0);
    if (inner) stencil_site_lds(pa, lr, xrow, y, L, h1, h2, h3, cf, tm == Lt - 1 ? -1.0 : 1.0, pv, prev, cen);
    __syncthreads();
    // chi(t0) on the R + 2 rows, from psi(t0) (LDS) and psi(t0 + 1) (own site)
#pragma unroll
    for (int c = 0; c < 4; ++c) pv[c] = rv[c];
    double c1 = f1, c2 = f2, c3 = f3;
    put(pa, pv);
    if (t0 + 1 < t1) {
        load_psi(wrapt(t0 + 2));
        load_phi(t0 + 1);
    }
    if (chirow) {
        stencil_site_lds(pb, lr, xrow, y, L, c1, c2, c3, cf, t0 == Lt - 1 ? -1.0 : 1.0, pv, own, cen);
#pragma unroll
        for (int c = 0; c < 4; ++c) ca[(lr - 1) * rowc + c * L + y] = own[c];
    }
    __syncthreads();
    // slice tau: as in k_mdm2_march, chi(tau + 1) and (M^dagger chi)(tau) between two barriers
    double2 *pcur = pa, *pnxt = pb, *ccur = ca, *cnxt = cb;
    for (int tau = t0; tau < t1; ++tau) {
        const bool more = tau + 1 < t1;
        double2 pn[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) pn[c] = rv[c];                  // psi(tau + 2)
        const double g1 = f1, g2 = f2, g3 = f3;                      // phi(tau + 1)
        if (tau + 2 < t1) {
            load_psi(wrapt(tau + 3));
            load_phi(tau + 2);
        }
        if (more) {
            put(pnxt, pn);
            if (chirow) {
                stencil_site_lds(pcur, lr, xrow, y, L, g1, g2, g3, cf, tau + 1 == Lt - 1 ? -1.0 : 1.0, pn, own, cen);
#pragma unroll
                for (int c = 0; c < 4; ++c) cnxt[(lr - 1) * rowc + c * L + y] = own[c];
            }
        }
        if (inner) {
            double2 o[4];
            stencil_site_lds(ccur, lr - 1, xrow, y, L, c1, c2, c3, cf, tau == 0 ? -1.0 : 1.0, prev, o, cen);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                dst[size_t(c) * vol + size_t(tau) * LL + ro] = o[c];
                prev[c] = cen[c];
            }
        }
        c1 = g1;
        c2 = g2;
        c3 = g3;
        __syncthreads();
        double2* sw = pcur;
        pcur = pnxt;
        pnxt = sw;
        sw = ccur;
        ccur = cnxt;
        cnxt = sw;
    }
}

}  // namespace hmc
