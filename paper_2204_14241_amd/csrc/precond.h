// The Fourier preconditioner of Methods C (Eq. 23-26) on the GPU: the passes that produce
// z = P r inside CG (transforms and tables in fft.h).
#pragma once

#include "fft.h"
#include "kernels.h"

namespace hmc {

// Fourier preconditioner passes (Methods C, Eq. 23-26), run for the units whose residual has
// just changed, producing z = P r with P = (K K^dagger)^{-1}, K the phi-independent part of
// the fermion matrix:
//   pass 1 (k_pc_xy, forward): 2-D (x, y) transform of one (component, tau) slice, r -> z;
//   pass 2 (k_pc_t): for each (x, y) frequency of one component, the exact solve of
//          K_k K_k^dagger z = r along tau (see below), in place on z; partial <r, z>;
//   pass 3 (k_pc_xy, inverse): inverse 2-D transform of one slice, in place on z.
// Pass 1 consumes the new residual norm (or the first |b|^2, or a true residual), pass 3 the
// <r, z> partials of pass 2.
// Columns of a tau-transform workgroup that keeps its column block in LDS (the metric's tau
// pass): 256 bytes of each slice row, 32 FP32 or 16 FP64 values.
template <typename R>
__host__ __device__ constexpr int pc_ncol() { return int(256 / sizeof(C2<R>)); }

__host__ __device__ __forceinline__ int pc_groups(int LL, int ncol) { return (LL + ncol - 1) / ncol; }

// Workgroup size of the slice passes: a slice is one workgroup's LDS, and only a few fit a
// CU, so each gets more threads (more loads in flight, shorter FFT phase).
constexpr int kPcBlock = 512;

constexpr int kPcCols = 64;     // columns per tau-pass workgroup

// Longest chunk a thread holds in registers (40 FP32, 32 FP64 values) and most chunks per
// column, i.e. wavefronts of a 512-thread workgroup: N_tau <= 320 (FP32) or 256 (FP64).
template <typename R>
__host__ __device__ constexpr int pc_chunk_max() { return sizeof(R) == 4 ? 40 : 32; }
template <typename R>
__host__ __device__ constexpr int pc_max_chunks() { return 8; }

// Chunks per column for N_tau (the fewest that keep chunks within pc_chunk_max); 0 if more
// than pc_max_chunks would be needed.
template <typename R>
__host__ __device__ inline int pc_chunks(int Lt) {
    const int q = (Lt + pc_chunk_max<R>() - 1) / pc_chunk_max<R>();
    return q > pc_max_chunks<R>() ? 0 : (q < 1 ? 1 : q);
}

// Stage n complex elements between global memory and LDS: element i of the set lives at g(i)
// in global memory and at lds[i].  Up to 64 bytes of loads are in flight per thread before
// their LDS writes (a plain loop would wait out the memory latency once per element).  The
// components are kept in separate arrays so that they stay in registers.
template <typename R, class G>
__device__ __forceinline__ void stage_in(C2<R>* __restrict__ lds, int n, G g) {
    constexpr int U = sizeof(R) == 4 ? 8 : 4;
    const int nt = blockDim.x;
    for (int i0 = threadIdx.x; i0 < n; i0 += nt * U) {
        R vx[U], vy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * nt;
            if (i < n) {
                const C2<R> v = *g(i);
                vx[u] = v.x;
                vy[u] = v.y;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * nt;
            if (i < n) lds[i] = mk<R>(vx[u], vy[u]);
        }
    }
}
template <typename R, class G>
__device__ __forceinline__ void stage_out(const C2<R>* __restrict__ lds, int n, G g) {
    constexpr int U = sizeof(R) == 4 ? 8 : 4;
    const int nt = blockDim.x;
    for (int i0 = threadIdx.x; i0 < n; i0 += nt * U) {
        R vx[U], vy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * nt;
            if (i < n) {
                const C2<R> v = lds[i];
                vx[u] = v.x;
                vy[u] = v.y;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * nt;
            if (i < n) *g(i) = mk<R>(vx[u], vy[u]);
        }
    }
}

template <typename R, bool INV, class Geo, int MAXR>
__global__ __launch_bounds__(kPcBlock) void k_pc_xy(CgCtl ctl, Geo geo, const C2<R>* src, C2<R>* dst,
                                                  const double* __restrict__ blob) {
    extern __shared__ __align__(16) unsigned char pc_smem[];
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const int L = lat.L, LL = lat.LL;
    const int nparts = INV ? 4 * pc_groups(LL, kPcCols) : pos.bpr;
    const int got = cg_finalize(ctl, pos, nparts);
    CgState& S = cg_shared();
    const bool work = S.pc && S.mode == CG_ACTIVE &&
                      (INV ? got == PEND_RZ : (got == PEND_RR || got == PEND_RU || got == PEND_BB));
    if (!work) {
        cg_publish(ctl, pos);
        return;
    }
    if (!INV && threadIdx.x == 0) S.zstage = 1;
    C2<R>* buf = reinterpret_cast<C2<R>*>(pc_smem);
    C2<R>* tw = buf + LL;
    const PcBlob bl = pc_blob_layout(L, lat.Lt);
    const double* B = blob + pos.pcoff;
    for (int i = threadIdx.x; i < L; i += kPcBlock) tw[i] = mk<R>(R(B[bl.twl + 2 * i]), R(B[bl.twl + 2 * i + 1]));
    const int c = pos.blk / lat.Lt, tau = pos.blk - c * lat.Lt;
    const size_t o = pos.voff + size_t(c) * lat.vol + size_t(tau) * LL;
    __shared__ FftPlan pl;
    if (threadIdx.x == 0) make_fft_plan(L, pl);
    __syncthreads();
    // the first stage reads the slice from src, the last writes it to dst
    fft_slice_io<R, INV, MAXR>(ExDevice(), src + o, buf, dst + o, pl, tw);
    cg_publish(ctl, pos);
}

// Pass 2.  For the (x, y) frequency k of a column, K acts along tau as
//   (K y)(tau) = -b y(tau) + s_tau y(tau + 1),  b = 1 + dtau (mu + 2 t_x cos kx + 2 t_y cos ky),
// with s_tau = -1 on the antiperiodic wrap (tau = N_tau - 1, where y(N_tau) is y(0)) and +1
// elsewhere; (K^dagger z)(tau) = -b z(tau) + s_{tau-1} z(tau - 1).  The twisted tau transform
// diagonalises both, which is how Eq. (24)-(26) apply P; here P_k = K_k^{-dagger} K_k^{-1} is
// applied directly as two first-order recurrences, y = K^{-1} r then z = K^{-dagger} y, each
// run in the direction in which it contracts: K^{-1} forward for |b| <= 1 (y(t+1) =
// s_t (r(t) + b y(t))) and backward otherwise (y(t) = (s_t y(t+1) - r(t)) / b); K^{-dagger}
// the other way round.  <r, P r> = sum |y|^2 (over the unnormalised 2-D transform, 1 / L^2).
//
// A workgroup takes 64 columns (one per lane) and cuts each into Q chunks, one per wavefront;
// a thread holds its chunk in registers.  Each recurrence: every thread reduces its chunk to
// an affine map of the value entering it, one lane per column composes the Q maps around the
// cycle (closing it through the wrap) and hands each chunk its entering value, and the
// threads rerun their chunks from it.
// Signs of the two recurrences at tau: s_tau (K) and s_{tau-1} (K^dagger).
struct SignK {
    int Lt;
    __host__ __device__ int operator()(int t) const { return t == Lt - 1 ? -1 : 1; }
};
struct SignKd {
    __host__ __device__ int operator()(int t) const { return t == 0 ? -1 : 1; }
};

// A thread's chunk: positions t0 .. t0 + n - 1 of its column in registers, v[j] holding
// t0 + j, or t0 + n - 1 - j when rev (a lane whose K^{-1} runs backward keeps its chunk in
// that order).  Both recurrences then walk the registers in a fixed order, K^{-1} up and
// K^{-dagger} down, with compile-time register positions: the direction never depends on
// the lane (a per-lane choice of register would put the chunk in scratch memory).
// One step at position t with entering value x: before, x' = sg(t) (b x + v(t)) and the value
// kept at t is x (K^{-1} forward, K^{-dagger} backward); else x' = (sg(t) x - v(t)) / b and the
// value kept is x' (K^{-1} backward, K^{-dagger} forward).
// chunk_map: the chunk as the affine map x_out = a x_in + c.
// One step; the sign is applied to chain values only (a select on the chunk's own values
// could be hoisted ahead of the chain and hold a second copy of the chunk).
template <typename R>
__host__ __device__ __forceinline__ C2<R> rec_step(C2<R> x, C2<R> v, R b, R ib, bool neg, bool before) {
    if (before) {   // sg (b x + v)
        const C2<R> w = mk<R>(b * x.x + v.x, b * x.y + v.y);
        return neg ? mk<R>(-w.x, -w.y) : w;
    }
    const C2<R> xs = neg ? mk<R>(-x.x, -x.y) : x;   // (sg x - v) / b
    return mk<R>(ib * (xs.x - v.x), ib * (xs.y - v.y));
}
template <typename R, int MC, bool ASC, class Sg>
__host__ __device__ __forceinline__ void chunk_map(const C2<R> (&v)[MC], int n, int t0, bool rev, R b, R ib, Sg sg,
                                                   bool before, R& a, C2<R>& c) {
    // a: the product of the steps' multipliers (b or 1/b, signed); c: the chunk run from 0
    a = R(1);
    c = mk<R>(R(0), R(0));
    const R mb = before ? b : ib;
#pragma unroll
    for (int k = 0; k < MC; ++k) {
        const int j = ASC ? k : MC - 1 - k;
        if (j < n) {
            const bool neg = sg(rev ? t0 + n - 1 - j : t0 + j) < 0;
            a = neg ? -(mb * a) : mb * a;
            c = rec_step<R>(c, v[j], b, ib, neg, before);
        }
    }
}
// The same chunk run from the entering value x, replacing v by the recurrence's values.
template <typename R, int MC, bool ASC, class Sg>
__host__ __device__ __forceinline__ void chunk_apply(C2<R> (&v)[MC], int n, int t0, bool rev, R b, R ib, Sg sg,
                                                     bool before, C2<R> x) {
#pragma unroll
    for (int k = 0; k < MC; ++k) {
        const int j = ASC ? k : MC - 1 - k;
        if (j < n) {
            const bool neg = sg(rev ? t0 + n - 1 - j : t0 + j) < 0;
            const C2<R> y = rec_step<R>(x, v[j], b, ib, neg, before);
            v[j] = before ? x : y;
            x = y;
        }
    }
}
// Compose the Q chunk maps of one column (a[q * st], c[q * st]) around the cycle and write
// the value entering each chunk: ascending chunks map x_q -> x_{q+1}, descending ones
// x_{q+1} -> x_q, and x_Q is x_0 (the wrap).  x[q * st] for q = 0 .. Q (x_Q = x_0); chunk q
// enters with x_q (ascending) or x_{q+1} (descending).
template <typename R>
__host__ __device__ inline void chunk_close(const R* a, const C2<R>* c, C2<R>* x, int Q, int st, bool up) {
    R A = R(1);
    C2<R> C = mk<R>(R(0), R(0));
    for (int k = 0; k < Q; ++k) {
        const int q = up ? k : Q - 1 - k;
        const R aq = a[q * st];
        A = aq * A;
        C = mk<R>(aq * C.x + c[q * st].x, aq * C.y + c[q * st].y);
    }
    const R inv = R(1) / (R(1) - A);
    C2<R> v = mk<R>(C.x * inv, C.y * inv);
    x[0] = v;
    x[Q * st] = v;
    for (int k = 0; k + 1 < Q; ++k) {
        const int q = up ? k : Q - 1 - k;   // map applied: x_{q+1} from x_q, or x_q from x_{q+1}
        const R aq = a[q * st];
        v = mk<R>(aq * v.x + c[q * st].x, aq * v.y + c[q * st].y);
        x[(up ? q + 1 : q) * st] = v;
    }
}

// b of the column at slice position col (positions hold frequencies in digit-reversed order,
// cosx is indexed by position).
__host__ __device__ inline double pc_column_b(int col, int L, int band, const double* cosx, const Coef<double>& cf) {
    const int px = col / L, py = col - px * L;
    const double cx = cosx[px], cy = cosx[py];
    return -cf.diag[band] - 2.0 * (cf.hop[band][0] * cx + cf.hop[band][1] * cy) -
           2.0 * (cf.hop2[band][0] * (2.0 * cx * cx - 1.0) + cf.hop2[band][1] * (2.0 * cy * cy - 1.0));
}

// Both recurrences on one thread's chunk, with the workgroup's map exchange in LDS (a, c, x:
// Q x 64 entries, x one row more).  Returns sum |y|^2 over the chunk (y = K^{-1} r).
template <typename R, int MC>
__device__ __forceinline__ double pc_tau_solve(C2<R> (&v)[MC], int n, int t0, int Lt, R b, R* sa, C2<R>* sc,
                                               C2<R>* sx, int q, int lane, int Q) {
    const R ib = R(1) / b;
    const bool small = b <= R(1) && b >= R(-1);
    const SignK sk{Lt};
    const SignKd skd{};
    R a;
    C2<R> c;
    // y = K^{-1} r: forward (kept value entering each step) for |b| <= 1, else backward; the
    // registers hold the chunk in the order this recurrence walks it (rev = !small)
    chunk_map<R, MC, true>(v, n, t0, !small, b, ib, sk, small, a, c);
    sa[q * kPcCols + lane] = a;
    sc[q * kPcCols + lane] = c;
    __syncthreads();
    if (q == 0) chunk_close<R>(sa + lane, sc + lane, sx + lane, Q, kPcCols, small);
    __syncthreads();
    chunk_apply<R, MC, true>(v, n, t0, !small, b, ib, sk, small, sx[(small ? q : q + 1) * kPcCols + lane]);
    double part = 0.0;
#pragma unroll
    for (int i = 0; i < MC; ++i)
        if (i < n) part += double(v[i].x) * double(v[i].x) + double(v[i].y) * double(v[i].y);
    __syncthreads();   // the exchange arrays are reused
    // z = K^{-dagger} y: backward for |b| <= 1, else forward, i.e. the registers walked down
    chunk_map<R, MC, false>(v, n, t0, !small, b, ib, skd, small, a, c);
    sa[q * kPcCols + lane] = a;
    sc[q * kPcCols + lane] = c;
    __syncthreads();
    if (q == 0) chunk_close<R>(sa + lane, sc + lane, sx + lane, Q, kPcCols, !small);
    __syncthreads();
    chunk_apply<R, MC, false>(v, n, t0, !small, b, ib, skd, small, sx[(small ? q + 1 : q) * kPcCols + lane]);
    return part;
}

// Dynamic LDS of the tau pass for Q chunks per column.
template <typename R>
__host__ __device__ inline size_t pc_tau_lds(int Q) {
    return size_t(Q) * kPcCols * (sizeof(R) + sizeof(C2<R>)) + size_t(Q + 1) * kPcCols * sizeof(C2<R>);
}

// Pass 2: one workgroup per (component, group of 64 columns) of a unit, 64 Q threads (lane:
// column, wavefront: chunk), Q = blockDim / 64 at least each lattice's pc_chunks.
template <typename R, class Geo>
__global__ __launch_bounds__(kPcCols * pc_max_chunks<R>()) void k_pc_t(CgCtl ctl, Geo geo, C2<R>* z,
                                                            const double* __restrict__ blob, Coef<double> cf) {
    extern __shared__ __align__(16) unsigned char pc_smem[];
    constexpr int MC = pc_chunk_max<R>();
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const int L = lat.L, Lt = lat.Lt, LL = lat.LL;
    cg_finalize(ctl, pos, 0);
    CgState& S = cg_shared();
    const bool work = S.pc && S.mode == CG_ACTIVE && S.zstage == 1;
    if (!work) {
        cg_publish(ctl, pos);
        return;
    }
    const int ng = pc_groups(LL, kPcCols);
    const int comp = pos.blk / ng, grp = pos.blk - comp * ng;
    // the chunk is the wavefront's (a scalar), the column the lane's
    const int lane = threadIdx.x & (kPcCols - 1), Q = blockDim.x / kPcCols;
    const int q = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kPcCols);
    const int col = grp * kPcCols + lane;
    const bool on = col < LL;
    // the lattice's own chunk count (a batch launch has the largest of its lattices; chunks
    // beyond a lattice's count are empty, identity maps, so each lattice is cut the same way
    // in a batch as on its own)
    const int ql = pc_chunks<R>(Lt), m = (Lt + ql - 1) / ql;
    const int t0 = min(q * m, Lt), n = min(m, Lt - t0);
    const PcBlob bl = pc_blob_layout(L, Lt);
    const R b = on ? R(pc_column_b(col, L, comp >> 1, blob + pos.pcoff + bl.cosx, cf)) : R(1);
    const bool rev = !(b <= R(1) && b >= R(-1));   // K^{-1} runs backward: chunk held reversed
    // element j of the chunk at zc + j * st (one pointer and one stride per lane)
    C2<R>* zc = z + pos.voff + size_t(comp) * lat.vol + size_t(t0) * LL + size_t(col) +
                (rev && n > 0 ? ptrdiff_t(n - 1) * LL : ptrdiff_t(0));
    ptrdiff_t st = rev ? -ptrdiff_t(LL) : ptrdiff_t(LL);
    C2<R> v[MC];
#pragma unroll
    for (int j = 0; j < MC; ++j) v[j] = (j < n && on) ? zc[j * st] : mk<R>(R(0), R(0));
    // the stores recompute their addresses rather than keep the loads' live through the solve
    asm volatile("" : "+v"(st));
    R* sa = reinterpret_cast<R*>(pc_smem);
    C2<R>* sc = reinterpret_cast<C2<R>*>(sa + Q * kPcCols);
    C2<R>* sx = sc + Q * kPcCols;
    const double part = pc_tau_solve<R, MC>(v, n, t0, Lt, b, sa, sc, sx, q, lane, Q);
    const R inv = R(1) / R(LL);
#pragma unroll
    for (int j = 0; j < MC; ++j)
        if (j < n && on) zc[j * st] = mk<R>(v[j].x * inv, v[j].y * inv);
    store_partial(ctl, PEND_RZ, pos, part / double(LL));
    if (threadIdx.x == 0) {
        S.zstage = 2;
        S.pending = PEND_RZ;
    }
    cg_publish(ctl, pos);
}

}  // namespace hmc
