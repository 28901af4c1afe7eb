// lattice.h -- lattice geometry, index arithmetic and operator coefficients shared by
// the host driver and the gfx950 kernels of libhmc.
//
// Site order is the row-major (tau, x, y) of the fermion-matrix labels of Eq. (17);
// a spinor stores its four components (c = 2*band + spin) as four planes of
// L_tau*L*L complex numbers, one vector after another.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmc {

constexpr int kMaxL = 256;
constexpr int kMaxVolLog2 = 26;    // exactness bound of FastDiv below
constexpr int kNumXcd = 8;          // MI355X: 8 XCDs, workgroups dispatched round-robin

// Exact unsigned division n / d for n < 2^26 and d <= 2^16 by a 42-bit reciprocal:
// with m = floor(2^42 / d) + 1 = (2^42 + e) / d, 0 < e <= d, floor(n m / 2^42) equals
// floor(n / d) whenever n e < 2^42, which the two bounds guarantee.
struct FastDiv {
    uint32_t d;
    uint64_t m;
    __host__ __device__ void init(uint32_t dd) {
        d = dd;
        m = (uint64_t(1) << 42) / dd + 1;
    }
    __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
        return uint32_t((uint64_t(n) * m) >> 42);
    }
};

struct Lat {
    int L, Lt, LL, vol;
    FastDiv dL, dLL;
};

inline Lat make_lat(int L, int Lt) {
    Lat l;
    l.L = L;
    l.Lt = Lt;
    l.LL = L * L;
    l.vol = Lt * L * L;
    l.dL.init(L);
    l.dLL.init(L * L);
    return l;
}

// Per-site geometry: coordinates, the six neighbours and the two time-link signs.
struct Nbr {
    int tau, x, y;
    int xp, xm, yp, ym, tp, tm;
    int sfwd;   // coefficient of psi(tau+1) in M: -1 on the last slice (antiperiodic)
    int sbwd;   // coefficient of psi(tau-1) in M^dagger: -1 on the first slice
    int stag;   // (-1)^(x+y), the phase exp(i Q_AF . r) with Q_AF = (pi, pi)
};

__host__ __device__ __forceinline__ Nbr neighbours(const Lat& lat, int s) {
    Nbr n;
    const int L = lat.L;
    const uint32_t q = lat.dL.div(uint32_t(s));        // s / L = tau*L + x
    n.y = s - int(q) * L;
    n.tau = int(lat.dLL.div(uint32_t(s)));
    n.x = int(q) - n.tau * L;
    n.xp = (n.x == L - 1) ? s - (L - 1) * L : s + L;
    n.xm = (n.x == 0) ? s + (L - 1) * L : s - L;
    n.yp = (n.y == L - 1) ? s - (L - 1) : s + 1;
    n.ym = (n.y == 0) ? s + (L - 1) : s - 1;
    n.tp = (n.tau == lat.Lt - 1) ? s - (lat.Lt - 1) * lat.LL : s + lat.LL;
    n.tm = (n.tau == 0) ? s + (lat.Lt - 1) * lat.LL : s - lat.LL;
    n.sfwd = (n.tau == lat.Lt - 1) ? -1 : 1;
    n.sbwd = (n.tau == 0) ? -1 : 1;
    n.stag = ((n.x + n.y) & 1) ? -1 : 1;
    return n;
}

// Sites two steps along each spatial axis (periodic): x +- 2 and y +- 2.
struct Nbr2 {
    int xpp, xmm, ypp, ymm;
};
__host__ __device__ __forceinline__ Nbr2 neighbours2(const Lat& lat, const Nbr& nb, int s) {
    const int L = lat.L;
    Nbr2 n;
    n.xpp = nb.x + 2 < L ? s + 2 * L : s + 2 * L - L * L;
    n.xmm = nb.x >= 2 ? s - 2 * L : s - 2 * L + L * L;
    n.ypp = nb.y + 2 < L ? s + 2 : s + 2 - L;
    n.ymm = nb.y >= 2 ? s - 2 : s - 2 + L;
    return n;
}

// Hardware workgroup id -> logical tile id.  Workgroups go round-robin to the 8 XCDs
// (bid % 8); this hands XCD j a contiguous range of logical tiles so that stencil
// neighbours (the rows above/below and the next/previous time slice) are read through
// the same L2.  Bijective on [0, nb).
__host__ __device__ __forceinline__ int xcd_remap(int bid, int nb) {
    const int q = nb / kNumXcd, rem = nb % kNumXcd;
    const int xcd = bid % kNumXcd, local = bid / kNumXcd;
    const int base = (xcd < rem) ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
    return base + local;
}

// ------------------------------------------------------------------------------------
// complex helpers (interleaved re, im), usable on the host and the device
template <typename R> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };
template <typename R> using C2 = typename CT<R>::T;

template <typename R>
__host__ __device__ __forceinline__ C2<R> mk(R re, R im) { C2<R> z; z.x = re; z.y = im; return z; }
template <typename R>
__host__ __device__ __forceinline__ C2<R> add(C2<R> a, C2<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R>
__host__ __device__ __forceinline__ C2<R> sub(C2<R> a, C2<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <typename R>
__host__ __device__ __forceinline__ C2<R> scl(R s, C2<R> a) { return mk<R>(s * a.x, s * a.y); }
// a + s*b
template <typename R>
__host__ __device__ __forceinline__ C2<R> axpy(R s, C2<R> b, C2<R> a) { return mk<R>(a.x + s * b.x, a.y + s * b.y); }
template <typename R>
__host__ __device__ __forceinline__ R norm2(C2<R> a) { return a.x * a.x + a.y * a.y; }
// a * b and a * conj(b)
template <typename R>
__host__ __device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) { return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <typename R>
__host__ __device__ __forceinline__ C2<R> cmulc(C2<R> a, C2<R> b) { return mk<R>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }

// Coefficients of M in the arithmetic precision R (Eq. 17).
template <typename R>
struct Coef {
    R diag[2];      // -(1 + dtau mu_band)
    R hop[2][2];    // -dtau t[band][direction]
    R cpl;          // dtau * lambda (Yukawa)
    R hop2[2][2];   // -dtau tn[band][direction]: hop by two sites along the axis
    int nn2;        // some hop2 is nonzero (the stencils then read the distance-2 sites)
};

// Boson-action coefficients (Eq. 2, time term 1/(2 c^2)).
struct BosonCoef {
    double kt;      // 1/(c^2 dtau): time-gradient stiffness after the dtau * 1/dtau^2
    double ks;      // dtau: spatial-gradient stiffness
    double kr;      // dtau * r
    double ku;      // dtau * u
};

}  // namespace hmc
