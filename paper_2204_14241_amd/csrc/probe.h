// probe.h -- plain streaming kernels that measure what HBM bandwidth this GPU sustains for a
// given mix of reads and writes.  They are the achievable-rate reference against which the
// stencil kernels are read: a kernel that streams r reads and w writes per site is compared
// with the probe that streams the same mix, not only with the nominal 8 TB/s.
//
// Each thread moves 16-byte vectors in a grid-stride loop, U of them in flight per stream
// before the first store (the stencil kernels keep about as many loads outstanding).  The
// nontemporal read form (NT) keeps eight loads in flight and marks them as streaming, so that
// they do not displace cached lines: the highest read rate found on this GPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "kernels.h"

namespace hmc {

enum ProbeKind : int { PROBE_READ = 0, PROBE_WRITE = 1, PROBE_COPY = 2, PROBE_3R3W = 3, PROBE_READ_NT = 4 };

typedef float probe_v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 probe_ld(const float4* p, bool nt) {
    if (!nt) return *p;
    const probe_v4f x = __builtin_nontemporal_load(reinterpret_cast<const probe_v4f*>(p));
    return make_float4(x.x, x.y, x.z, x.w);
}

// NR source streams and NW destination streams of n4 16-byte vectors each, stream k of the
// sources at src + k * n4 (likewise dst).  NR > 0, NW = 0: the reads are summed and one
// partial per workgroup is written to part (so the loads cannot be dropped).  NR = 0: every
// destination vector is written with its index.  Otherwise destination k receives source k
// scaled by 1.5 (NR = NW).  NT: nontemporal loads (read-only form).
template <int NR, int NW, bool NT = false>
__global__ __launch_bounds__(kBlock) void k_stream(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   size_t n4, double* __restrict__ part) {
    static_assert(!NT || (NR == 1 && NW == 0), "the nontemporal form reads one stream");
    constexpr int U = NT ? 8 : (NR == 0 ? 4 : (NR == 1 ? 4 : 2));
    const size_t stride = size_t(gridDim.x) * kBlock;
    float acc = 0.f;
    for (size_t i0 = size_t(blockIdx.x) * kBlock + threadIdx.x; i0 < n4; i0 += stride * U) {
        float4 v[NR > 0 ? NR : 1][U];
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t i = i0 + size_t(u) * stride;
                v[k][u] = i < n4 ? probe_ld(src + size_t(k) * n4 + i, NT) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        if constexpr (NW == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) acc += (v[0][u].x + v[0][u].y) + (v[0][u].z + v[0][u].w);
        } else {
#pragma unroll
            for (int k = 0; k < NW; ++k)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const size_t i = i0 + size_t(u) * stride;
                    if (i >= n4) continue;
                    float4 w;
                    if constexpr (NR == 0) {
                        const float f = float(i);
                        w = make_float4(f, f, f, f);
                    } else {
                        const float4 a = v[k][u];
                        w = make_float4(1.5f * a.x, 1.5f * a.y, 1.5f * a.z, 1.5f * a.w);
                    }
                    dst[size_t(k) * n4 + i] = w;
                }
        }
    }
    if constexpr (NW == 0) {
        double a[1] = {double(acc)};
        block_reduce<1>(a);
        if (threadIdx.x == 0) part[blockIdx.x] = a[0];
    }
}

}  // namespace hmc
