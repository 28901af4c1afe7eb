// march.h -- the normal operator M^dagger M of Eq. (22) in one pass over HBM.
//
// With chi = M psi (Eq. 17):  (M^dagger M psi)(tau) = A_tau chi(tau) + s_{tau-1} chi(tau - 1),
// where A_tau is the time-local part of M (diagonal, hopping, Yukawa coupling to phi(tau)) and
// s_{tau-1} the sign of the time link (-1 across the antiperiodic wrap at tau = 0).  Applying
// A_tau needs chi(tau) at the spatial neighbours, so chi(tau) = A_tau psi(tau) + s_tau psi(tau+1)
// is formed one row beyond the rows a workgroup writes, and chi(tau - 1) is the previous slice of
// the same workgroup.
//
// A workgroup owns a band of R whole rows (x0 .. x0 + R - 1, every y) of one vector and marches
// through a segment of time slices.  Per slice it computes chi on the R + 2 rows of its band and
// the two rows beside it into LDS (psi and phi come through the cache hierarchy: the rows beside
// a band are the neighbour bands' own rows, read by the workgroups next to it on the same XCD),
// then forms M^dagger M psi on its R rows from LDS and from chi(tau - 1), which each thread keeps
// in registers for the sites it writes.  The first slice of a segment forms chi(t0 - 1) at those
// sites first.  HBM sees psi and phi read once and the result written once: 76 B per site in
// FP32 (complex64 spinors, FP32 phi), 152 B in FP64, against twice that for two passes.
// Workgroups are ordered segment-major, so with the XCD remap each XCD sweeps every band of a
// run of consecutive segments: the rows beside a band and the slice before a segment are read
// through the same L2.
//
// The nearest-neighbour operator only (the two-site hops need a band two rows wider); the
// arithmetic per site is that of the two-pass kernels, in the same order.
#pragma once

#include "kernels.h"

namespace hmc {

// Most threads of a marching workgroup (8 waves: up to 256 VGPRs per thread).
constexpr int kMarchMaxThreads = 512;

// Cut of one lattice into bands of rows and segments of time slices.
struct MarchPlan {
    int R;        // rows per band (the last band may have fewer)
    int nband;    // bands: ceil(L / R)
    int seglen;   // slices per segment (the last segment may have fewer)
    int nseg;     // segments: ceil(L_tau / seglen)
};

__host__ __device__ inline MarchPlan make_march_plan(int L, int Lt, int R, int seglen) {
    MarchPlan p;
    p.R = R < L ? R : L;
    p.nband = (L + p.R - 1) / p.R;
    p.seglen = seglen < Lt ? seglen : Lt;
    p.nseg = (Lt + p.seglen - 1) / p.seglen;
    return p;
}

// The workgroup's vector, band and segment.
struct MarchPos {
    int k, x0, nr, t0, t1;
};
__device__ __forceinline__ MarchPos march_pos(const Lat& lat, const MarchPlan& mp, int wg) {
    const int per_vec = mp.nseg * mp.nband;
    MarchPos p;
    p.k = wg / per_vec;
    const int rem = wg - p.k * per_vec;
    const int seg = rem / mp.nband, band = rem - seg * mp.nband;
    p.x0 = band * mp.R;
    p.nr = lat.L - p.x0 < mp.R ? lat.L - p.x0 : mp.R;
    p.t0 = seg * mp.seglen;
    p.t1 = lat.Lt - p.t0 < mp.seglen ? lat.Lt : p.t0 + mp.seglen;
    return p;
}

__device__ __forceinline__ int wrap_row(int x, int L) { return x < 0 ? x + L : (x >= L ? x - L : x); }

// Dynamic LDS of a marching workgroup: chi on R + 2 rows, 4 components, L sites.
template <typename R>
__host__ __device__ inline size_t march_lds(int Rrows, int L) {
    return size_t(Rrows + 2) * 4 * size_t(L) * sizeof(C2<R>);
}

// M^dagger at the pair (x, y) of slice tau (flat index s) from chi(tau) in LDS (row r of the
// band buffer, [row][component][y]) and chi(tau - 1) in registers (tt), with the time link's
// sign ts: the stencil arithmetic of the two-pass kernels in their order.  cen receives
// chi(tau) at the pair.
__device__ __forceinline__ void mdag_pair_lds(const float2* __restrict__ chi, int r, int x, int y, int s,
                                              const Lat& lat, const float* __restrict__ phi,
                                              const Coef<float>& cf, float ts, const float4 (&tt)[4],
                                              float4 (&o)[4], float4 (&cen)[4]) {
    const int L = lat.L, vol = lat.vol, rowc = 4 * L;
    auto lds4 = [&](int rr, int c, int yy) { return *reinterpret_cast<const float4*>(chi + rr * rowc + c * L + yy); };
    const int yl = y == 0 ? L - 1 : y - 1, yr = y + 2 == L ? 0 : y + 2;
#pragma unroll
    for (int c = 0; c < 4; ++c) cen[c] = lds4(r, c, y);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int a = c >> 1;
        const float4 xp = lds4(r + 1, c, y), xm = lds4(r - 1, c, y), t4 = tt[c];
        const float2 lo = chi[r * rowc + c * L + yl], hi = chi[r * rowc + c * L + yr];
        const float4 ce = cen[c];
        const float dg = cf.diag[a], h0 = cf.hop[a][0], h1 = cf.hop[a][1];
        float4 v;
        v.x = dg * ce.x + h0 * (xp.x + xm.x) + h1 * (lo.x + ce.z) + ts * t4.x;
        v.y = dg * ce.y + h0 * (xp.y + xm.y) + h1 * (lo.y + ce.w) + ts * t4.y;
        v.z = dg * ce.z + h0 * (xp.z + xm.z) + h1 * (ce.x + hi.x) + ts * t4.z;
        v.w = dg * ce.w + h0 * (xp.w + xm.w) + h1 * (ce.y + hi.y) + ts * t4.w;
        o[c] = v;
    }
    const float g0 = cf.cpl * float((x & 1) ? -1 : 1), g1 = -g0;   // (-1)^(x+y), y even
    const float2 P1 = *reinterpret_cast<const float2*>(phi + s);
    const float2 P2 = *reinterpret_cast<const float2*>(phi + vol + s);
    const float2 P3 = *reinterpret_cast<const float2*>(phi + 2 * vol + s);
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

// FP32: an element is a pair of neighbouring sites (y even), as in the pair kernels.
// EPT: pairs of the band's rows per thread (the launch has at least R * L / (2 EPT) threads,
// at most kMarchMaxThreads).
template <int EPT>
__global__ __launch_bounds__(kMarchMaxThreads) void k_mdm2(Lat lat, MarchPlan mp, const float2* __restrict__ in,
                                               float2* __restrict__ out, const float* __restrict__ phi,
                                               Coef<float> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    float2* chi = reinterpret_cast<float2*>(march_smem);      // [row][component][y]
    const int L = lat.L, vol = lat.vol, P = L / 2, rowc = 4 * L;
    const MarchPos mpos = march_pos(lat, mp, xcd_remap(blockIdx.x, gridDim.x));
    const size_t voff = size_t(mpos.k) * 4 * vol;
    const SrcPlain2 src{in + voff, vol};
    float2* dst = out + voff;
    const int nint = mpos.nr * P, nhalo = (mpos.nr + 2) * P;

    // chi(t0 - 1) at this thread's pairs
    float4 prev[EPT][4];
    {
        const int tm = mpos.t0 == 0 ? lat.Lt - 1 : mpos.t0 - 1;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = threadIdx.x + j * blockDim.x;
            if (e < nint) {
                const int lr = e / P, py = e - lr * P;
                const int s = (tm * L + mpos.x0 + lr) * L + 2 * py;
                float4 cen[4];
                dslash_pair<false, false>(src, phi, lat, cf, neighbours(lat, s), s, prev[j], cen);
            }
        }
    }
    for (int tau = mpos.t0; tau < mpos.t1; ++tau) {
        // chi(tau) = M psi on the band's rows and the row on either side
        for (int e = threadIdx.x; e < nhalo; e += blockDim.x) {
            const int lr = e / P, py = e - lr * P;
            const int s = (tau * L + wrap_row(mpos.x0 - 1 + lr, L)) * L + 2 * py;
            float4 o[4], cen[4];
            dslash_pair<false, false>(src, phi, lat, cf, neighbours(lat, s), s, o, cen);
#pragma unroll
            for (int c = 0; c < 4; ++c) *reinterpret_cast<float4*>(chi + lr * rowc + c * L + 2 * py) = o[c];
        }
        __syncthreads();
        // M^dagger chi on the band's rows: A_tau chi(tau) from LDS, the time link from chi(tau - 1)
        const float ts = tau == 0 ? -1.f : 1.f;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = threadIdx.x + j * blockDim.x;
            if (e < nint) {
                const int lr = e / P, py = e - lr * P, y = 2 * py;
                const int x = mpos.x0 + lr;
                const int s = (tau * L + x) * L + y;
                float4 cen[4], o[4];
                mdag_pair_lds(chi, lr + 1, x, y, s, lat, phi, cf, ts, prev[j], o, cen);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    st4(dst, size_t(c) * vol + s, o[c]);
                    prev[j][c] = cen[c];
                }
            }
        }
        __syncthreads();
    }
}

// FP64 form of mdag_pair_lds at the site (x, y).
__device__ __forceinline__ void mdag_site_lds(const double2* __restrict__ chi, int r, int x, int y, int s,
                                              const Lat& lat, const double* __restrict__ phi,
                                              const Coef<double>& cf, double ts, const double2 (&tt)[4],
                                              double2 (&o)[4], double2 (&cen)[4]) {
    const int L = lat.L, vol = lat.vol, rowc = 4 * L;
    const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
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
        o[c] = v;
    }
    const double g = cf.cpl * double(((x + y) & 1) ? -1 : 1);
    const double q1 = g * phi[s], q2 = g * phi[vol + s], q3 = g * phi[2 * vol + s];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const double2 u = cen[2 * (1 - a)], w = cen[2 * (1 - a) + 1];
        o[2 * a].x += q3 * u.x + q1 * w.x + q2 * w.y;
        o[2 * a].y += q3 * u.y + q1 * w.y - q2 * w.x;
        o[2 * a + 1].x += q1 * u.x - q2 * u.y - q3 * w.x;
        o[2 * a + 1].y += q1 * u.y + q2 * u.x - q3 * w.y;
    }
}

// FP64: an element is one site.
template <int EPT>
__global__ __launch_bounds__(kMarchMaxThreads) void k_mdm(Lat lat, MarchPlan mp, const double2* __restrict__ in,
                                              double2* __restrict__ out, const double* __restrict__ phi,
                                              Coef<double> cf) {
    extern __shared__ __align__(16) unsigned char march_smem[];
    double2* chi = reinterpret_cast<double2*>(march_smem);    // [row][component][y]
    const int L = lat.L, vol = lat.vol, rowc = 4 * L;
    const MarchPos mpos = march_pos(lat, mp, xcd_remap(blockIdx.x, gridDim.x));
    const size_t voff = size_t(mpos.k) * 4 * vol;
    const SrcPlain<double> src{in + voff, vol};
    double2* dst = out + voff;
    const int nint = mpos.nr * L, nhalo = (mpos.nr + 2) * L;

    double2 prev[EPT][4];
    {
        const int tm = mpos.t0 == 0 ? lat.Lt - 1 : mpos.t0 - 1;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = threadIdx.x + j * blockDim.x;
            if (e < nint) {
                const int lr = e / L, y = e - lr * L;
                const int s = (tm * L + mpos.x0 + lr) * L + y;
                double2 cen[4];
                dslash_site<double, false, false>(src, phi, lat, cf, neighbours(lat, s), s, prev[j], cen);
            }
        }
    }
    for (int tau = mpos.t0; tau < mpos.t1; ++tau) {
        for (int e = threadIdx.x; e < nhalo; e += blockDim.x) {
            const int lr = e / L, y = e - lr * L;
            const int s = (tau * L + wrap_row(mpos.x0 - 1 + lr, L)) * L + y;
            double2 o[4], cen[4];
            dslash_site<double, false, false>(src, phi, lat, cf, neighbours(lat, s), s, o, cen);
#pragma unroll
            for (int c = 0; c < 4; ++c) chi[lr * rowc + c * L + y] = o[c];
        }
        __syncthreads();
        const double ts = tau == 0 ? -1.0 : 1.0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = threadIdx.x + j * blockDim.x;
            if (e < nint) {
                const int lr = e / L, y = e - lr * L;
                const int x = mpos.x0 + lr;
                const int s = (tau * L + x) * L + y;
                double2 cen[4], o[4];
                mdag_site_lds(chi, lr + 1, x, y, s, lat, phi, cf, ts, prev[j], o, cen);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    dst[size_t(c) * vol + s] = o[c];
                    prev[j][c] = cen[c];
                }
            }
        }
        __syncthreads();
    }
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

}  // namespace hmc
