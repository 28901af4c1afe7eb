/*
 * hmc_testing.h -- host-callable helpers of libhmc, exported so that the lattice indexing and
 * the FFT the kernels use can be checked on a machine without a GPU.
 *
 * They run the same __host__ __device__ functions the kernels call, compiled for the host.
 * Arguments are plain integers and host arrays; nothing here touches a device, except
 * hmc_test_apply_precond (the preconditioner applied once on the GPU, for parity tests).
 */
#ifndef HMC_TESTING_H
#define HMC_TESTING_H

#include "hmc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Decompose a site index s = (tau*L + x)*L + y of an L x L x L_tau lattice into
 * (tau, x, y) and its six neighbours in the order x+1, x-1, y+1, y-1, tau+1, tau-1
 * (periodic wrap), plus the signs of the two time links as the kernels apply them:
 * sign_fwd is the coefficient of psi(tau+1) in M (-1 on the last slice, +1 otherwise,
 * Eq. 17), sign_bwd that of psi(tau-1) in M^dagger (-1 on the first slice).
 * out[0..2] = tau, x, y; out[3..8] = neighbours; out[9] = sign_fwd; out[10] = sign_bwd;
 * out[11] = the staggered phase (-1)^(x+y).  Returns 0, or -1 for an argument the
 * kernels reject (odd L, L < 4, L > 256, L_tau < 2, volume >= 2^26, s out of range). */
int hmc_test_site(int L, int L_tau, int s, int out[12]);

/* The block-index permutation the kernels use to keep neighbouring lattice tiles on one
 * of the MI355X's 8 XCDs: maps a hardware workgroup id (dispatched round-robin over the
 * XCDs) to a logical tile id.  A bijection on [0, nblocks). */
int hmc_test_xcd_remap(int bid, int nblocks);

/* The tiles a CG or apply workgroup works on: workgroup blk of the bpr workgroups of one
 * right-hand side, over nt tiles, takes tiles out[0], out[0] + out[2], ... below out[1].
 * Over blk in [0, bpr) these sets partition [0, nt).  Returns 0, or -1 for blk outside
 * [0, bpr), bpr < 1 or nt < 0. */
int hmc_test_tile_span(int blk, int bpr, int nt, int out[3]);

/* The in-place mixed-radix FFT of the preconditioner (fft.h), run on the host in FP64 on one
 * line of n complex numbers (interleaved re, im).  Forward (inverse = 0): the unnormalised
 * transform sum_m x_m exp(-2 pi i m k / n), frequency k left at the position p with
 * hmc_test_fft_freq(n, p) = k.  Inverse: the conjugate transpose of the forward map, so that
 * inverse(forward(x)) = n x.  Returns 0, or -1 if n has a prime factor above 7. */
int hmc_test_fft(int n, int inverse, const double* in, double* out);
int hmc_test_fft_freq(int n, int pos);

/* The Fourier preconditioner P = (K K^dagger)^{-1} of Methods C (Eq. 26) applied on the host
 * in FP64 to one spinor (complex128, [4][L_tau][L][L]) by the same three passes the kernels
 * run (2-D transforms per slice; per frequency column the two tau recurrences, chunked as the
 * FP64 kernel chunks them; inverse 2-D).  rz (optional) receives <in, P in> = sum |K^{-1} r|^2.
 * Returns 0, or -1 for a lattice the preconditioner does not support. */
int hmc_test_precond(int L, int L_tau, double dtau, const hmc_params* params, const double* in,
                     double* out, double* rz);

/* One application z = P r of the Fourier preconditioner P = (K K^dagger)^{-1} of Methods C
 * (Eq. 23-26) ON THE GPU, by the kernels a preconditioned solve runs (it is the only entry
 * point here that touches a device).  ctx: a one-lattice context with its workspace set (its
 * params need not ask for the preconditioner, but the lattice must support it in
 * `precision`).  in: n <= max_rhs complex128 spinors (device); out: n spinors (device) in the
 * Krylov precision of `precision`: complex128 for HMC_FP64, complex64 for HMC_MIXED (then r is
 * in rounded to FP32 first, as the mixed solver holds it).  rz (optional, host, n doubles):
 * <r, P r> reduced in FP64.  Uses the context's workspace; synchronises the stream.  Errors:
 * HMC_ERR_INVALID_ARG (NULL, alignment, n, batch context, unsupported lattice),
 * HMC_ERR_WORKSPACE, HMC_ERR_NONFINITE, HMC_ERR_HIP. */
int hmc_test_apply_precond(hmc_ctx* ctx, int precision, const void* in, void* out, int n, double* rz,
                           void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HMC_TESTING_H */
