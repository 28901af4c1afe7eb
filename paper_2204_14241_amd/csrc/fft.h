// fft.h -- the twisted Fourier preconditioner P = (K K^dagger)^{-1} of Methods C (Eq. 23-26)
// and the in-place mixed-radix FFT it runs on.
//
// K, the phi-independent part of the fermion matrix, is diagonal on twisted plane waves
// exp(i w_n tau + 2 pi i (kx x + ky y) / L) with w_n = pi (2 n + 1) / N_tau (the twist
// exp(i pi tau / N_tau) turns periodic functions of tau into antiperiodic ones).  Its eigenvalue
// is exp(i w_n) - b with b = 1 + dtau (mu_band + 2 t[band][0] cos k_x + 2 t[band][1] cos k_y
// + 2 tn[band][0] cos 2k_x + 2 tn[band][1] cos 2k_y), the tn terms being the hops by two
// sites of the production model, so P multiplies each Fourier coefficient of the untwisted
// field by 1 / |exp(i w_n) - b|^2 = 1 / ((1 - b)^2 + 4 b sin^2(w_n / 2)).
//
// The preconditioner runs in three passes over a spinor: (1) the 2-D (x, y) transform of
// every (component, tau) slice, held in LDS; (2) per (x, y) frequency column, the exact
// inverse of K K^dagger along tau as two first-order recurrences in registers (precond.h),
// which is what the twisted tau transform and the symbol compute; (3) the inverse 2-D
// transform of every slice.  This header holds the transforms and the tables.
//
// FFT: forward is a decimation-in-frequency sequence of radix stages done in place, so its
// output sits in mixed-radix digit-reversed order (position p holds frequency fft_freq(p));
// the inverse applies the conjugate transposes of the same stages in reverse order, which
// takes that order back to natural order.  No permutation pass is ever needed: the symbol is
// applied at permuted positions, and every position knows its frequency.  Radices 4, 2, 3,
// 5, 7; lengths with a larger prime factor are rejected.  The functions are
// __host__ __device__: the host build serves the CPU tests of this code.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.h"

namespace hmc {

constexpr int kFftMaxStages = 12;   // 4^12 > any lattice extent accepted
constexpr int kFftMaxRadix = 7;

struct FftPlan {
    int n;                      // transform length
    int nst;                    // number of radix stages
    int radix[kFftMaxStages];   // radix of stage 0 (outermost) ... nst - 1
    int ni[kFftMaxStages];      // sub-length a stage works on (n for stage 0)
    FastDiv dM[kFftMaxStages];  // division by ni / radix (butterfly -> block, offset)
    FastDiv dnb[kFftMaxStages]; // division by n / radix (work item -> line, butterfly)
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
    const int primes[4] = {2, 3, 5, 7};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int f = primes[i];
        while (m % f == 0) {
            if (p.nst == kFftMaxStages) return false;
            p.radix[p.nst++] = f;
            m /= f;
        }
    }
    int len = n;
    for (int st = 0; st < p.nst; ++st) {
        p.ni[st] = len;
        p.dM[st].init(uint32_t(len / p.radix[st]));
        p.dnb[st].init(uint32_t(n / p.radix[st]));
        len /= p.radix[st];
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

// Small DFT of radix 2, 3, 4 or 5 in place on v: v_k <- sum_m v_m W^{(+-) m k},
// W = exp(-2 pi i / RAD).  Radix 2 and 4 exactly; radix 3 and 5 in their symmetric forms with
// the powers of W read from the length-n table (W_RAD^e = tw[e * n / RAD]).
template <typename R, bool INV, int RAD>
__host__ __device__ __forceinline__ void small_dft(C2<R> (&v)[RAD], const C2<R>* tw, int n) {
    if constexpr (RAD == 2) {
        const C2<R> a = v[0], b = v[1];
        v[0] = add<R>(a, b);
        v[1] = sub<R>(a, b);
    } else if constexpr (RAD == 4) {
        const C2<R> a = v[0], b = v[1], c = v[2], d = v[3];
        const C2<R> s0 = add<R>(a, c), d0 = sub<R>(a, c), s1 = add<R>(b, d), d1 = sub<R>(b, d);
        // forward: -i * d1; inverse: +i * d1
        const C2<R> jd1 = INV ? mk<R>(-d1.y, d1.x) : mk<R>(d1.y, -d1.x);
        v[0] = add<R>(s0, s1);
        v[1] = add<R>(d0, jd1);
        v[2] = sub<R>(s0, s1);
        v[3] = sub<R>(d0, jd1);
    } else if constexpr (RAD == 3) {
        // W = c - i s with c = -1/2, s = sin(2 pi / 3), both taken from the table
        const C2<R> w = tw[n / 3];
        const R hs = INV ? -w.y : w.y;                    // -s forward, +s inverse
        const C2<R> a = v[0], b = v[1], c = v[2];
        const C2<R> t1 = add<R>(b, c);
        const C2<R> t2 = axpy<R>(w.x, t1, a);             // a + c t1 (c = -1/2)
        const C2<R> d = sub<R>(b, c);
        const C2<R> t3 = mk<R>(-hs * d.y, hs * d.x);       // i * hs * (b - c)
        v[0] = add<R>(a, t1);
        v[1] = add<R>(t2, t3);
        v[2] = sub<R>(t2, t3);
    } else if constexpr (RAD == 5) {
        // W = c1 - i s1, W^2 = c2 - i s2 from the table; the symmetric 5-point form
        const C2<R> w1 = tw[n / 5], w2 = tw[2 * (n / 5)];
        const R c1 = w1.x, s1 = -w1.y, c2 = w2.x, s2 = -w2.y;
        const C2<R> t1 = add<R>(v[1], v[4]), t2 = add<R>(v[2], v[3]);
        const C2<R> t3 = sub<R>(v[1], v[4]), t4 = sub<R>(v[2], v[3]);
        const C2<R> a1 = axpy<R>(c2, t2, axpy<R>(c1, t1, v[0]));
        const C2<R> a2 = axpy<R>(c1, t2, axpy<R>(c2, t1, v[0]));
        const C2<R> b1 = axpy<R>(s2, t4, scl<R>(s1, t3));
        const C2<R> b2 = axpy<R>(-s1, t4, scl<R>(s2, t3));
        // forward: X1 = a1 - i b1, X4 = a1 + i b1, X2 = a2 - i b2, X3 = a2 + i b2; inverse: i -> -i
        const R sg = INV ? R(-1) : R(1);
        const C2<R> ib1 = mk<R>(-sg * b1.y, sg * b1.x), ib2 = mk<R>(-sg * b2.y, sg * b2.x);
        v[0] = add<R>(v[0], add<R>(t1, t2));
        v[1] = sub<R>(a1, ib1);
        v[4] = add<R>(a1, ib1);
        v[2] = sub<R>(a2, ib2);
        v[3] = add<R>(a2, ib2);
    }
}

// Butterfly j of a radix-RAD stage with sub-length ni, transform length n: its inputs sit at
// positions base + M q (q < RAD) of the line, and its twiddles are W_n^{e1 k}.
struct BflyPos {
    int base, M, e1;
};
__host__ __device__ __forceinline__ BflyPos bfly_pos(int n, int ni, const FastDiv& dM, int j) {
    const int M = int(dM.d);
    const int b = int(dM.div(uint32_t(j))), n1 = j - b * M;
    return BflyPos{b * ni + n1, M, (n / ni) * n1};
}
template <typename R, int RAD>
__host__ __device__ __forceinline__ void bfly_load(const C2<R>* src, int es, const BflyPos& p, C2<R> (&v)[RAD]) {
#pragma unroll
    for (int q = 0; q < RAD; ++q) v[q] = src[(p.base + p.M * q) * es];
}

// The butterfly on its loaded inputs v, stored at the same positions of the line at `line`.
// Forward (DIF): small DFT, then times W_n^{e1 k}.  Inverse: the conjugate transpose of that
// map.  The twiddle exponent e1 k stays below n because n1 < ni/RAD and k < RAD.
template <typename R, bool INV, int RAD>
__host__ __device__ __forceinline__ void bfly_store(C2<R>* line, int es, int n, const BflyPos& p, C2<R> (&v)[RAD],
                                                    const C2<R>* tw) {
    const int base = p.base, M = p.M, e1 = p.e1;
    if constexpr (RAD <= 5) {
        // W^{e1 k} as powers of the one table entry W^{e1} (one LDS read per butterfly instead
        // of RAD - 1, whose per-lane addresses also collide in the banks)
        const C2<R> w1 = tw[e1];
        if constexpr (!INV) {
            small_dft<R, false, RAD>(v, tw, n);
            C2<R> w = w1;
#pragma unroll
            for (int k = 1; k < RAD; ++k) {
                v[k] = cmul<R>(v[k], w);
                if (k + 1 < RAD) w = cmul<R>(w, w1);
            }
        } else {
            C2<R> w = w1;
#pragma unroll
            for (int k = 1; k < RAD; ++k) {
                v[k] = cmulc<R>(v[k], w);
                if (k + 1 < RAD) w = cmul<R>(w, w1);
            }
            small_dft<R, true, RAD>(v, tw, n);
        }
#pragma unroll
        for (int q = 0; q < RAD; ++q) line[(base + M * q) * es] = v[q];
    } else {
        // radix 7: each output is summed from the inputs held in registers and stored at once
        // (no output array), the powers of W read from the table as they are needed
        const int step = n / RAD;
        if constexpr (INV) {
#pragma unroll
            for (int k = 1; k < RAD; ++k) v[k] = cmulc<R>(v[k], tw[e1 * k]);
        }
#pragma unroll
        for (int k = 0; k < RAD; ++k) {
            C2<R> acc = v[0];
#pragma unroll
            for (int m = 1; m < RAD; ++m) {
                const C2<R> w = tw[((m * k) % RAD) * step];
                acc = add<R>(acc, INV ? cmulc<R>(v[m], w) : cmul<R>(v[m], w));
            }
            if constexpr (!INV) {
                if (k > 0) acc = cmul<R>(acc, tw[e1 * k]);
            }
            line[(base + M * k) * es] = acc;
        }
    }
}


// One butterfly j, from the line at `src` to the same positions of the line at `line` (in
// place when they coincide).
template <typename R, bool INV, int RAD>
__host__ __device__ __forceinline__ void butterfly(const C2<R>* src, C2<R>* line, int es, int n, int ni,
                                                   const FastDiv& dM, int j, const C2<R>* tw) {
    const BflyPos p = bfly_pos(n, ni, dM, j);
    C2<R> v[RAD];
    bfly_load<R, RAD>(src, es, p, v);
    bfly_store<R, INV, RAD>(line, es, n, p, v, tw);
}

// One radix-RAD stage on cnt lines: every butterfly of every line, spread over the executor,
// from the lines at src to the same positions at dst.  Consecutive work items take
// consecutive lines when lines are closer together than the elements of a line, consecutive
// butterflies otherwise (LDS bank spread, and whole rows of a slice when src or dst is in
// global memory).  Divisions by the stage's counts use the plan's precomputed reciprocals.
template <typename R, bool INV, int RAD, class Ex>
__host__ __device__ __forceinline__ void fft_stage(const Ex& ex, const C2<R>* src, C2<R>* buf, int es, int ls,
                                                   int cnt, const FastDiv& dcnt, int n, int ni, const FastDiv& dM,
                                                   const FastDiv& dnb, const C2<R>* tw) {
    const int nb = n / RAD;
    const bool lines_fast = ls < es;
    ex.for_each(cnt * nb, [&](int j) {
        int l, jj;
        if (lines_fast) {
            jj = int(dcnt.div(uint32_t(j)));
            l = j - jj * cnt;
        } else {
            l = int(dnb.div(uint32_t(j)));
            jj = j - l * nb;
        }
        butterfly<R, INV, RAD>(src + l * ls, buf + l * ls, es, n, ni, dM, jj, tw);
    });
}

// The same stage with the inputs of NB butterflies per thread loaded before any is computed,
// for a stage that reads global memory (more loads in flight than one butterfly's).
template <typename R, bool INV, int RAD, int NB, class Ex>
__host__ __device__ __forceinline__ void fft_stage_nb(const Ex& ex, const C2<R>* src, C2<R>* buf, int es, int ls,
                                                      int cnt, const FastDiv& dcnt, int n, int ni, const FastDiv& dM,
                                                      const FastDiv& dnb, const C2<R>* tw) {
    const int nb = n / RAD, total = cnt * nb, stride = ex.stride();
    const bool lines_fast = ls < es;
#pragma unroll 1
    for (int j0 = ex.first(); j0 < total; j0 += NB * stride) {
        C2<R> v[NB][RAD];
        BflyPos p[NB];
        int lo[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * stride;
            if (j < total) {
                int l, jj;
                if (lines_fast) {
                    jj = int(dcnt.div(uint32_t(j)));
                    l = j - jj * cnt;
                } else {
                    l = int(dnb.div(uint32_t(j)));
                    jj = j - l * nb;
                }
                lo[u] = l * ls;
                p[u] = bfly_pos(n, ni, dM, jj);
                bfly_load<R, RAD>(src + lo[u], es, p[u], v[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u)
            if (j0 + u * stride < total) bfly_store<R, INV, RAD>(buf + lo[u], es, n, p[u], v[u], tw);
    }
}

// Execution policies: the device one spreads work over the workgroup and synchronises it; the
// host one runs sequentially (CPU tests).  sum_each adds up what f returns, per thread.
struct ExDevice {
    __device__ __forceinline__ int first() const { return int(threadIdx.x); }
    __device__ __forceinline__ int stride() const { return int(blockDim.x); }
    template <class F>
    __device__ __forceinline__ void for_each(int n, F f) const {
#pragma unroll 1
        for (int i = threadIdx.x; i < n; i += blockDim.x) f(i);
    }
    template <class F>
    __device__ __forceinline__ double sum_each(int n, F f) const {
        double a = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) a += f(i);
        return a;
    }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
};
struct ExHost {
    int first() const { return 0; }
    int stride() const { return 1; }
    template <class F>
    void for_each(int n, F f) const {
        for (int i = 0; i < n; ++i) f(i);
    }
    template <class F>
    double sum_each(int n, F f) const {
        double a = 0.0;
        for (int i = 0; i < n; ++i) a += f(i);
        return a;
    }
    void sync() const {}
};

// Stage st of the plan on cnt lines (line l starts at src + l * ls and dst + l * ls, element
// stride es), no synchronisation.  MAXR is the largest radix compiled in (5 or 7): a kernel's
// register allocation covers every stage it can reach, and the radix-7 stage needs many more
// than the others, so kernels for lattices without a factor 7 leave it out.
template <typename R, bool INV, int MAXR = 7, int NB = 1, class Ex>
__host__ __device__ __forceinline__ void fft_one_stage(const Ex& ex, const C2<R>* src, C2<R>* dst, int es, int ls,
                                                       int cnt, const FastDiv& dcnt, const FftPlan& pl, int st,
                                                       const C2<R>* tw) {
    const int n = pl.n, ni = pl.ni[st];
    const FastDiv& dM = pl.dM[st];
    const FastDiv& dnb = pl.dnb[st];
#define HMC_FFT_STAGE(RAD)                                                                       \
    if constexpr (NB > 1) fft_stage_nb<R, INV, RAD, NB>(ex, src, dst, es, ls, cnt, dcnt, n, ni, dM, dnb, tw); \
    else fft_stage<R, INV, RAD>(ex, src, dst, es, ls, cnt, dcnt, n, ni, dM, dnb, tw);
    switch (pl.radix[st]) {
        case 4: { HMC_FFT_STAGE(4) } break;
        case 2: { HMC_FFT_STAGE(2) } break;
        case 3: { HMC_FFT_STAGE(3) } break;
        case 5: { HMC_FFT_STAGE(5) } break;
        default:
            if constexpr (MAXR >= 7) { HMC_FFT_STAGE(7) }
            break;
    }
#undef HMC_FFT_STAGE
}

// Stages in place on cnt lines of buf, in transform order (stage 0 first forward, last first
// inverse), leaving out the first `skip0` and the last `skip1` of that order; each followed by
// a synchronisation.  The plan may live in LDS: it is only read, stage by stage.
template <typename R, bool INV, int MAXR = 7, class Ex>
__host__ __device__ __forceinline__ void fft_lines(const Ex& ex, C2<R>* buf, int es, int ls, int cnt,
                                                   const FftPlan& pl, const C2<R>* tw, int skip0 = 0,
                                                   int skip1 = 0) {
    const int nst = pl.nst;
    FastDiv dcnt;
    dcnt.init(uint32_t(cnt));
    for (int q = skip0; q < nst - skip1; ++q) {
        fft_one_stage<R, INV, MAXR>(ex, buf, buf, es, ls, cnt, dcnt, pl, INV ? nst - 1 - q : q, tw);
        ex.sync();
    }
}

// 2-D transform of one L x L slice (row-major x, y) in place: forward along y then x; inverse
// along x then y.
template <typename R, bool INV, int MAXR = 7, class Ex>
__host__ __device__ __forceinline__ void fft_slice(const Ex& ex, C2<R>* buf, const FftPlan& pl, const C2<R>* tw) {
    const int L = pl.n;
    if (!INV) {
        fft_lines<R, false, MAXR>(ex, buf, 1, L, L, pl, tw);
        fft_lines<R, false, MAXR>(ex, buf, L, 1, L, pl, tw);
    } else {
        fft_lines<R, true, MAXR>(ex, buf, L, 1, L, pl, tw);
        fft_lines<R, true, MAXR>(ex, buf, 1, L, L, pl, tw);
    }
}

// The same 2-D transform from the slice at src to the slice at dst, with buf (the size of a
// slice) as the working copy: the first stage reads src and writes buf, the last reads buf and
// writes dst, so src and dst (which may coincide) are each touched once, by a stage, with no
// separate copy in or out.
template <typename R, bool INV, int MAXR = 7, class Ex>
__host__ __device__ __forceinline__ void fft_slice_io(const Ex& ex, const C2<R>* src, C2<R>* buf, C2<R>* dst,
                                                      const FftPlan& pl, const C2<R>* tw) {
    const int L = pl.n, nst = pl.nst;
    FastDiv dL;
    dL.init(uint32_t(L));
    // forward: rows (es 1, ls L) then columns (es L, ls 1); inverse: columns then rows
    const int es0 = INV ? L : 1, ls0 = INV ? 1 : L;
    // the stage that reads src keeps several butterflies' loads in flight per thread (2 FP32,
    // which keeps three slice workgroups per CU; 4 FP64, where one slice fills the LDS anyway)
    fft_one_stage<R, INV, MAXR, sizeof(R) == 4 ? 2 : 4>(ex, src, buf, es0, ls0, L, dL, pl, INV ? nst - 1 : 0, tw);
    ex.sync();
    fft_lines<R, INV, MAXR>(ex, buf, es0, ls0, L, pl, tw, 1, 0);
    fft_lines<R, INV, MAXR>(ex, buf, ls0, es0, L, pl, tw, 0, 1);
    fft_one_stage<R, INV, MAXR>(ex, buf, dst, ls0, es0, L, dL, pl, INV ? 0 : nst - 1, tw);
}

// Largest radix a plan uses.
__host__ __device__ inline int fft_max_radix(const FftPlan& pl) {
    int m = 1;
    for (int i = 0; i < pl.nst; ++i) m = pl.radix[i] > m ? pl.radix[i] : m;
    return m;
}

// Per-lattice tables, computed once on the host in FP64 (pc_table_blob) and read by the
// passes of the preconditioner and of the metric:
//   twl[j]   = exp(-2 pi i j / L)          FFT twiddles of length L
//   twT[j]   = exp(-2 pi i j / N_tau)      FFT twiddles of length N_tau
//   cosx[p]  = cos(2 pi k / L) for the frequency k held at x (or y) position p
// Offsets (in doubles) of the tables in the flat blob.
struct PcBlob {
    int twl, twT, cosx, size;
};
__host__ __device__ __forceinline__ PcBlob pc_blob_layout(int L, int Lt) {
    PcBlob b;
    b.twl = 0;
    b.twT = 2 * L;
    b.cosx = b.twT + 2 * Lt;
    b.size = b.cosx + L;
    return b;
}

}  // namespace hmc
