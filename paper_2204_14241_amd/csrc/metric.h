// Kernels of the Fourier-diagonal HMC metric ("Scale-invariant sampling": Eq. 30 and the
// momentum draw and kinetic energy stated with it).  They reuse the FFT of the Fourier
// preconditioner (fft.h) and the staging and reduction helpers of kernels.h.
//
// On a real boson-shaped field v (3 components of
// N_tau x L x L) the passes compute, per component, the unitary transform F v and from it
// per-frequency work against a caller table sigma of the same shape in natural frequency
// order: y = Re F(s . F^* v) with s = sigma or sigma^(-1/2), the sums sum_k w(k) |(F v)(k)|^2
// with w = sigma, 1/sigma or 1, and acc(k) += |(F v)(k)|^2 (one term of Eq. 30).  A null
// sigma reads as sigma = 1.  FP64, three passes shaped like the preconditioner's: the slice
// FFT of (v, 0) into a complex scratch field, the tau pass, the inverse slice FFT that writes
// or adds the real part.
#pragma once

#include "precond.h"

namespace hmc {

enum MetricMul : int { MUL_SIGMA = 1, MUL_RSQRT = 2 };
enum MetricRed : int { RED_NONE = 0, RED_SIGMA = 1, RED_INV = 2, RED_PLAIN = 3 };

struct MetricGeo {
    int L, Lt, LL, vol;
};

// One workgroup per (component, slice).  Forward: scr = FFT2(in, 0).  Inverse: the inverse
// FFT2 of scr, then out = Re (add == 0) or out += h Re (add == 1).
template <bool INV, int MAXR>
__global__ __launch_bounds__(kPcBlock) void k_mt_xy(MetricGeo g, const double* __restrict__ in,
                                                  double2* __restrict__ scr, double* __restrict__ out, int add,
                                                  double h, const double* __restrict__ blob) {
    extern __shared__ __align__(16) unsigned char pc_smem[];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int L = g.L, LL = g.LL;
    double2* buf = reinterpret_cast<double2*>(pc_smem);
    double2* tw = buf + LL;
    const PcBlob bl = pc_blob_layout(L, g.Lt);
    for (int i = threadIdx.x; i < L; i += kPcBlock) tw[i] = make_double2(blob[bl.twl + 2 * i], blob[bl.twl + 2 * i + 1]);
    __shared__ FftPlan pl;
    if (threadIdx.x == 0) make_fft_plan(L, pl);
    const size_t o = size_t(b) * LL;   // slice tau of component l: b = l N_tau + tau
    if (!INV) {
        for (int i = threadIdx.x; i < LL; i += kPcBlock) buf[i] = make_double2(in[o + i], 0.0);
    } else {
        stage_in<double>(buf, LL, [&](int i) { return scr + o + i; });
    }
    __syncthreads();
    fft_slice<double, INV, MAXR>(ExDevice(), buf, pl, tw);
    if (!INV) {
        stage_out<double>(buf, LL, [&](int i) { return scr + o + i; });
    } else if (add) {
        for (int i = threadIdx.x; i < LL; i += kPcBlock) out[o + i] = out[o + i] + h * buf[i].x;
    } else {
        for (int i = threadIdx.x; i < LL; i += kPcBlock) out[o + i] = buf[i].x;
    }
}

// One workgroup per (component, group of 16 consecutive positions of a slice): the tau FFT
// of the group's columns of scr, the per-frequency work (positions are in digit-reversed
// order; each knows its frequency), and with `mul` != 0 the scaling by s / V and the inverse
// tau FFT back into scr.  part[workgroup] receives rs times the workgroup's share of the sum;
// acc(k) receives |(F v)(k)|^2, added (acc_add) or stored.
template <int MAXR>
__global__ __launch_bounds__(kPcBlock) void k_mt_t(MetricGeo g, double2* __restrict__ scr,
                                                 const double* __restrict__ sigma, int mul, int red, double rs,
                                                 double* __restrict__ acc, int acc_add, double* __restrict__ part,
                                                 const double* __restrict__ blob) {
    extern __shared__ __align__(16) unsigned char pc_smem[];
    constexpr int NC = pc_ncol<double>();
    const int L = g.L, Lt = g.Lt, LL = g.LL;
    const int ng = pc_groups(LL, NC);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int l = b / ng, grp = b - l * ng;
    const int col0 = grp * NC, ncol = min(NC, LL - col0);
    double2* buf = reinterpret_cast<double2*>(pc_smem);
    double2* twT = buf + Lt * NC;
    int* fT = reinterpret_cast<int*>(twT + Lt);
    int* fL = fT + Lt;
    const PcBlob bl = pc_blob_layout(L, Lt);
    for (int i = threadIdx.x; i < Lt; i += kPcBlock) twT[i] = make_double2(blob[bl.twT + 2 * i], blob[bl.twT + 2 * i + 1]);
    __shared__ FftPlan pt, pl;
    if (threadIdx.x == 0) make_fft_plan(Lt, pt);
    if (threadIdx.x == 1) make_fft_plan(L, pl);
    __syncthreads();
    for (int i = threadIdx.x; i < Lt; i += kPcBlock) fT[i] = fft_freq(pt, i);
    for (int i = threadIdx.x; i < L; i += kPcBlock) fL[i] = fft_freq(pl, i);
    FastDiv dc, dL;
    dc.init(uint32_t(ncol));
    dL.init(uint32_t(L));
    const size_t o = size_t(l) * g.vol + size_t(col0);
    auto at = [&](int i) {
        const int tau = int(dc.div(uint32_t(i)));
        return scr + o + size_t(tau) * LL + (i - tau * ncol);
    };
    stage_in<double>(buf, Lt * ncol, at);
    __syncthreads();
    fft_lines<double, false, MAXR>(ExDevice(), buf, ncol, 1, ncol, pt, twT);
    const double inv_v = 1.0 / double(g.vol);
    const double* sg = sigma ? sigma + size_t(l) * g.vol : nullptr;
    double* ac = acc ? acc + size_t(l) * g.vol : nullptr;
    double sum[1] = {0.0};
    for (int i = threadIdx.x; i < Lt * ncol; i += kPcBlock) {
        const int p = int(dc.div(uint32_t(i))), j = i - p * ncol;
        const int col = col0 + j;
        const int px = int(dL.div(uint32_t(col))), py = col - px * L;
        const size_t k = (size_t(fT[p]) * L + fL[px]) * L + fL[py];
        const double sv = sg ? sg[k] : 1.0;
        const double2 y = buf[i];
        const double n2 = (y.x * y.x + y.y * y.y) * inv_v;
        if (red == RED_SIGMA) sum[0] += sv * n2;
        else if (red == RED_INV) sum[0] += n2 / sv;
        else if (red == RED_PLAIN) sum[0] += n2;
        if (ac) ac[k] = acc_add ? ac[k] + n2 : n2;
        if (mul) {
            const double m = (mul == MUL_SIGMA ? sv : 1.0 / sqrt(sv)) * inv_v;
            buf[i] = make_double2(m * y.x, m * y.y);
        }
    }
    block_reduce<1>(sum);   // ends with a barrier
    if (part != nullptr && threadIdx.x == 0) part[b] = rs * sum[0];
    if (mul) {
        fft_lines<double, true, MAXR>(ExDevice(), buf, ncol, 1, ncol, pt, twT);
        stage_out<double>(buf, Lt * ncol, at);
    }
}

// chi(k) += scale ((t0(k) + t1(k)) + t2(k)) for the three component planes of t (each vol
// long): one term of the SDW susceptibility of Eq. (34) from the per-component spectra.
__global__ __launch_bounds__(kBlock) void k_mt_sum3(const double* __restrict__ t, double* __restrict__ chi,
                                                    double scale, int vol) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < vol) chi[i] = chi[i] + scale * ((t[i] + t[vol + i]) + t[2 * vol + i]);
}

// Per-workgroup partial sums of each component of a boson-shaped field: part[l * nb + b] for
// component l and workgroup b of nb (the order parameter Phi = sum over sites of phi).
__global__ __launch_bounds__(kBlock) void k_mt_csum(const double* __restrict__ phi, double* __restrict__ part,
                                                    int vol, int nb) {
    const int l = blockIdx.x / nb, b = blockIdx.x - l * nb;
    double v[1] = {0.0};
    for (int i = b * kBlock + threadIdx.x; i < vol; i += nb * kBlock) v[0] += phi[size_t(l) * vol + i];
    block_reduce<1>(v);
    if (threadIdx.x == 0) part[size_t(l) * nb + b] = v[0];
}

}  // namespace hmc
