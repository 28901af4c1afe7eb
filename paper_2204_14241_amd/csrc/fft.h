// fft.h -- the twisted Fourier preconditioner P = (K K^dagger)^{-1} of Methods C (Eq. 23-26)
// and the in-place mixed-radix FFT it runs on.
//
// K, the phi-independent part of the fermion matrix, is diagonal on twisted plane waves
// exp(i w_n tau + 2 pi i (kx x + ky y) / L) with w_n = pi (2 n + 1) / N_tau (the twist
// exp(i pi tau / N_tau) turns periodic functions of tau into antiperiodic ones).  Its eigenvalue
// is exp(i w_n) - b with b = 1 + dtau (mu_band + 2 t[band][0] cos k_x + 2 t[band][1] cos k_y),
// so P multiplies each Fourier coefficient of the untwisted field by
// 1 / |exp(i w_n) - b|^2 = 1 / ((1 - b)^2 + 4 b sin^2(w_n / 2)).
//
// The transforms are split into three passes over a spinor so that each pass holds a whole
// line set in LDS: (1) the 2-D (x, y) transform of every (component, tau) slice; (2) per group
// of (x, y) columns of one component, twist, transform along tau, multiply by the symbol,
// inverse along tau, untwist; (3) the inverse 2-D transform of every slice.
//
// FFT: forward is a decimation-in-frequency sequence of radix stages done in place, so its
// output sits in mixed-radix digit-reversed order (position p holds frequency fft_freq(p));
// the inverse applies the conjugate transposes of the same stages in reverse order, which
// takes that order back to natural order.  No permutation pass is ever needed: the symbol is
// applied at permuted positions, and every position knows its frequency.  Radices 4, 2, 3,
// 5, 7, 11, 13; lengths with a larger prime factor are rejected.  The functions are
// __host__ __device__: the host build serves the CPU tests of this code.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.h"

namespace hmc {

constexpr int kFftMaxStages = 24;
constexpr int kFftMaxRadix = 13;

struct FftPlan {
    int n;                      // transform length
    int nst;                    // number of radix stages
    int radix[kFftMaxStages];   // radix of stage 0 (outermost) ... nst - 1
};

__host__ __device__ inline bool make_fft_plan(int n, FftPlan& p) {
    p.n = n;
    p.nst = 0;
    if (n < 1) return false;
    int m = n;
    while (m % 4 == 0) {
        if (p.nst == kFftMaxStages) return false;
        p.radix[p.nst++] = 4;
        m /= 4;
    }
    const int primes[6] = {2, 3, 5, 7, 11, 13};
    for (int f : primes) {
        while (m % f == 0) {
            if (p.nst == kFftMaxStages) return false;
            p.radix[p.nst++] = f;
            m /= f;
        }
    }
    return m == 1;
}

// Frequency held at position pos after the forward transform.
__host__ __device__ inline int fft_freq(const FftPlan& pl, int pos) {
    int k = 0, mult = 1, rem = pl.n;
    for (int i = 0; i < pl.nst; ++i) {
        const int M = rem / pl.radix[i];
        const int d = pos / M;
        pos -= d * M;
        k += d * mult;
        mult *= pl.radix[i];
        rem = M;
    }
    return k;
}

// Small DFT of radix r in place on v: v_k <- sum_m v_m W^{(+-) m k}, W = exp(-2 pi i / r)
// read from the length-n table (W_r^e = tw[e * n / r]).
template <typename R, bool INV>
__host__ __device__ inline void small_dft(C2<R> (&v)[kFftMaxRadix], int r, const C2<R>* tw, int n) {
    if (r == 2) {
        const C2<R> a = v[0], b = v[1];
        v[0] = add<R>(a, b);
        v[1] = sub<R>(a, b);
        return;
    }
    if (r == 4) {
        const C2<R> a = v[0], b = v[1], c = v[2], d = v[3];
        const C2<R> s0 = add<R>(a, c), d0 = sub<R>(a, c), s1 = add<R>(b, d), d1 = sub<R>(b, d);
        // forward: -i * d1; inverse: +i * d1
        const C2<R> jd1 = INV ? mk<R>(-d1.y, d1.x) : mk<R>(d1.y, -d1.x);
        v[0] = add<R>(s0, s1);
        v[1] = add<R>(d0, jd1);
        v[2] = sub<R>(s0, s1);
        v[3] = sub<R>(d0, jd1);
        return;
    }
    C2<R> o[kFftMaxRadix];
    const int step = n / r;
    for (int k = 0; k < r; ++k) {
        C2<R> acc = v[0];
        for (int m = 1; m < r; ++m) {
            const C2<R> w = tw[((m * k) % r) * step];
            acc = add<R>(acc, INV ? cmulc<R>(v[m], w) : cmul<R>(v[m], w));
        }
        o[k] = acc;
    }
    for (int k = 0; k < r; ++k) v[k] = o[k];
}

// One butterfly j of stage st (sub-length ni) on the line at `line`, element stride es.
// Forward (DIF): v_q = x[base + M q]; small DFT; times W_N^{(N/ni) n1 k}; store in place.
// Inverse: the conjugate transpose of that map.
template <typename R, bool INV>
__host__ __device__ inline void fft_butterfly(C2<R>* line, int es, const FftPlan& pl, int st, int ni,
                                              int j, const C2<R>* tw) {
    const int r = pl.radix[st];
    const int M = ni / r;
    const int b = j / M, n1 = j - b * M;
    const int base = b * ni + n1;
    const int s = pl.n / ni;
    C2<R> v[kFftMaxRadix];
    for (int q = 0; q < r; ++q) v[q] = line[(base + M * q) * es];
    if (!INV) {
        small_dft<R, false>(v, r, tw, pl.n);
        for (int k = 1; k < r; ++k) v[k] = cmul<R>(v[k], tw[(s * n1 * k) % pl.n]);
    } else {
        for (int k = 1; k < r; ++k) v[k] = cmulc<R>(v[k], tw[(s * n1 * k) % pl.n]);
        small_dft<R, true>(v, r, tw, pl.n);
    }
    for (int q = 0; q < r; ++q) line[(base + M * q) * es] = v[q];
}

// Execution policies: the device one spreads work over the workgroup and synchronises it; the
// host one runs sequentially (CPU tests).
struct ExDevice {
    template <class F>
    __device__ __forceinline__ void for_each(int n, F f) const {
        for (int i = threadIdx.x; i < n; i += blockDim.x) f(i);
    }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
};
struct ExHost {
    template <class F>
    void for_each(int n, F f) const {
        for (int i = 0; i < n; ++i) f(i);
    }
    void sync() const {}
};

// All stages on cnt lines (line l starts at buf + l * ls, element stride es).
template <typename R, bool INV, class Ex>
__host__ __device__ inline void fft_lines(const Ex& ex, C2<R>* buf, int es, int ls, int cnt,
                                          const FftPlan& pl, const C2<R>* tw) {
    int ni[kFftMaxStages];
    int len = pl.n;
    for (int st = 0; st < pl.nst; ++st) {
        ni[st] = len;
        len /= pl.radix[st];
    }
    for (int q = 0; q < pl.nst; ++q) {
        const int st = INV ? pl.nst - 1 - q : q;
        const int nb = pl.n / pl.radix[st];
        const int nist = ni[st];
        ex.for_each(cnt * nb, [=](int j) {
            const int l = j / nb;
            fft_butterfly<R, INV>(buf + l * ls, es, pl, st, nist, j - l * nb, tw);
        });
        ex.sync();
    }
}

// 2-D transform of one L x L slice (row-major x, y) in place: forward along y then x; inverse
// along x then y.
template <typename R, bool INV, class Ex>
__host__ __device__ inline void fft_slice(const Ex& ex, C2<R>* buf, const FftPlan& pl, const C2<R>* tw) {
    const int L = pl.n;
    if (!INV) {
        fft_lines<R, false>(ex, buf, 1, L, L, pl, tw);
        fft_lines<R, false>(ex, buf, L, 1, L, pl, tw);
    } else {
        fft_lines<R, true>(ex, buf, L, 1, L, pl, tw);
        fft_lines<R, true>(ex, buf, 1, L, L, pl, tw);
    }
}

// Symbol 1/|K_hat|^2 of the preconditioner for one band, from b and sin^2(w_n / 2).
__host__ __device__ __forceinline__ double pc_symbol(double b, double s2) {
    const double d = 1.0 - b;
    return 1.0 / (d * d + 4.0 * b * s2);
}

// Per-lattice tables, computed once on the host in FP64 (pc_table_blob) and read by every pass:
//   twl[j]   = exp(-2 pi i j / L)          FFT twiddles of length L
//   twT[j]   = exp(-2 pi i j / N_tau)      FFT twiddles of length N_tau
//   twt[tau] = exp(-i pi tau / N_tau)      the conjugate twist
//   s2[p]    = sin^2(w_n / 2) for the frequency n held at tau-position p
//   cosx[p]  = cos(2 pi k / L) for the frequency k held at x (or y) position p
template <typename R>
struct PcTables {
    C2<R>* twt;
    double* s2;
    double* cosx;
    C2<R>* twl;
    C2<R>* twT;
};

// Offsets (in doubles) of the tables in the flat blob: twl, twT, twt (complex), s2, cosx.
struct PcBlob {
    int twl, twT, twt, s2, cosx, size;
};
__host__ __device__ __forceinline__ PcBlob pc_blob_layout(int L, int Lt) {
    PcBlob b;
    b.twl = 0;
    b.twT = 2 * L;
    b.twt = b.twT + 2 * Lt;
    b.s2 = b.twt + 2 * Lt;
    b.cosx = b.s2 + Lt;
    b.size = b.cosx + L;
    return b;
}

// The tau pass on one group of `ncol` (x, y) columns of one component of band `band`, held in
// buf as [N_tau][ncol] (column j at buf + j, stride ncol), starting at xy-position col0.
// Input: the (x, y)-transformed field; output: the same after twist, tau transform, symbol,
// inverse tau transform and untwist, scaled by 1 / (N_tau L^2).  Returns the workgroup's share
// of <r, P r> = (1 / N) sum |Y|^2 / |K_hat|^2 (Parseval), valid in every thread's own terms
// (the caller reduces).
template <typename R, class Ex>
__host__ __device__ inline double pc_tau_pass(const Ex& ex, C2<R>* buf, int ncol, int col0, int band,
                                              const PcTables<R>& t, const FftPlan& pt, const FftPlan& pl,
                                              const Coef<double>& cf64) {
    const int Lt = pt.n, L = pl.n;
    const double inv_n = 1.0 / (double(Lt) * double(L) * double(L));
    ex.for_each(Lt * ncol, [=](int i) {
        const int tau = i / ncol;
        buf[i] = cmul<R>(buf[i], t.twt[tau]);
    });
    ex.sync();
    fft_lines<R, false>(ex, buf, ncol, 1, ncol, pt, t.twT);
    double part = 0.0;
    double* pp = &part;
    ex.for_each(Lt * ncol, [=](int i) {
        const int p = i / ncol, j = i - p * ncol;
        const int col = col0 + j;
        const int px = col / L, py = col - px * L;
        // b = 1 + dtau (mu + 2 t_x cos kx + 2 t_y cos ky), with diag = -1 - dtau mu, hop = -dtau t
        const double b = -cf64.diag[band] - 2.0 * (cf64.hop[band][0] * t.cosx[px] + cf64.hop[band][1] * t.cosx[py]);
        const double w = pc_symbol(b, t.s2[p]) * inv_n;
        const C2<R> y = buf[i];
        *pp += w * double(norm2<R>(y));
        buf[i] = scl<R>(R(w), y);
    });
    ex.sync();
    fft_lines<R, true>(ex, buf, ncol, 1, ncol, pt, t.twT);
    ex.for_each(Lt * ncol, [=](int i) {
        const int tau = i / ncol;
        buf[i] = cmulc<R>(buf[i], t.twt[tau]);
    });
    ex.sync();
    return part;
}

}  // namespace hmc
