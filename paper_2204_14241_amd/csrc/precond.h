// The Fourier preconditioner of Methods C (Eq. 23-26) on the GPU: the passes that produce
// z = P r inside CG (transforms and tables in fft.h).
#pragma once

#include <type_traits>

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

// Longest chunk a thread holds in registers (20 FP32, 32 FP64 values) and most chunks per
// column, i.e. wavefronts of a workgroup (1024 or 512 threads): N_tau <= 320 (FP32) or 256
// (FP64).  Short FP32 chunks give a column more wavefronts and each a shorter chain (at
// 80x80x200 the pass takes 19 us with chunks of 20 against 26 us with 40); FP64 chunks of 20
// would spill under the 1024-thread bound.
template <typename R>
__host__ __device__ constexpr int pc_chunk_max() { return sizeof(R) == 4 ? 20 : 32; }
template <typename R>
__host__ __device__ constexpr int pc_max_chunks() { return sizeof(R) == 4 ? 16 : 8; }

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
// A thread's chunk: positions t0 .. t0 + n - 1 of its column in registers, v[j] holding
// t0 + j, or t0 + n - 1 - j when rev (a lane whose K^{-1} runs backward keeps its chunk in
// that order).  Both recurrences then walk the registers in a fixed order, K^{-1} up and
// K^{-dagger} down, with compile-time register positions (a per-lane choice of register would
// put the chunk in scratch memory).
// Away from the wrap, every step of either recurrence is x' = A x + B v(t) with the lane's own
// A and B.  A lane with |b| <= 1 runs both "before": the step keeps its entering value x
// (K^{-1} forward, K^{-dagger} backward), A = b, B = 1.  Otherwise the step keeps x' (K^{-1}
// backward, K^{-dagger} forward), A = 1/b, B = -1/b.  The wrap's sign s = -1 falls on one step
// of one chunk (tau = N_tau - 1 for K^{-1}, tau = 0 for K^{-dagger}): the last step a before-lane
// takes there, whose leaving value it negates, or the first step of any other lane, whose
// entering value it negates.  It is therefore applied to that chunk's map and entering value
// (wrap_map, wrap_entry) rather than inside the loop.
template <typename R>
struct RecCoef {
    R A, B;
    bool before;
};
template <typename R>
__host__ __device__ __forceinline__ RecCoef<R> rec_coef(R b) {
    const bool before = b <= R(1) && b >= R(-1);
    const R ib = R(1) / b;
    return {before ? b : ib, before ? R(1) : -ib, before};
}

// Chunk q of a column of N_tau positions: chunks of pc_chunk_max from tau = 0, the last one
// shorter, the ones beyond the column empty (n = 0).  Full chunks make a reversed lane's rows
// the mirror image of a forward lane's, so loads and stores can be issued in mirrored pairs.
struct ChunkSpan {
    int t0, n;
};
template <typename R>
__host__ __device__ __forceinline__ ChunkSpan pc_chunk_span(int q, int Lt) {
    constexpr int MC = pc_chunk_max<R>();
    const int t0 = q * MC < Lt ? q * MC : Lt;
    return {t0, Lt - t0 < MC ? Lt - t0 : MC};
}

// A chunk's length: the runtime count, or FixedLen when every chunk of the launch is full, so
// that the walks carry no per-step predicates.
template <int N>
struct FixedLen {
    __host__ __device__ constexpr FixedLen() {}
    __host__ __device__ constexpr explicit FixedLen(int) {}   // the runtime count, known to be N
    __host__ __device__ constexpr operator int() const { return N; }
};

// x^n by repeated squaring (n >= 0).
template <typename R>
__host__ __device__ __forceinline__ R ipow(R x, int n) {
    R r = R(1);
    for (; n > 0; n >>= 1) {
        if (n & 1) r *= x;
        x *= x;
    }
    return r;
}

// The chunk's values are scaled by B once (chunk_scale), so that each step is one multiply-add
// per component, x' = A x + u(t) with u = B v.  (Computing B v inside the steps lets the
// compiler keep those products live from one walk to the next: a second copy of the chunk.)
// Registers beyond the chunk hold zeros, which scaling keeps, so it needs no predicate.
template <typename R, int MC>
__host__ __device__ __forceinline__ void chunk_scale(C2<R> (&v)[MC], R B) {
#pragma unroll
    for (int j = 0; j < MC; ++j) v[j] = mk<R>(B * v[j].x, B * v[j].y);
}
// chunk_map: the chunk (scaled values u) as the affine map x_out = a x_in + c (a = A^n, c the
// chunk run from 0).
template <typename R, int MC, bool ASC, class N>
__host__ __device__ __forceinline__ void chunk_map(const C2<R> (&u)[MC], N n, RecCoef<R> k, R& a, C2<R>& c) {
    a = ipow(k.A, int(n));
    c = mk<R>(R(0), R(0));
#pragma unroll
    for (int s = 0; s < MC; ++s) {
        const int j = ASC ? s : MC - 1 - s;
        if (j < n) c = mk<R>(k.A * c.x + u[j].x, k.A * c.y + u[j].y);
    }
}
// The same chunk run from the entering value x, replacing u by the recurrence's values.
template <typename R, int MC, bool ASC, class N>
__host__ __device__ __forceinline__ void chunk_apply(C2<R> (&u)[MC], N n, RecCoef<R> k, C2<R> x) {
#pragma unroll
    for (int s = 0; s < MC; ++s) {
        const int j = ASC ? s : MC - 1 - s;
        if (j < n) {
            const C2<R> y = mk<R>(k.A * x.x + u[j].x, k.A * x.y + u[j].y);
            u[j] = mk<R>(k.before ? x.x : y.x, k.before ? x.y : y.y);
            x = y;
        }
    }
}
// The wrap's sign on the chunk that holds it: a before-lane's leaving value is negated
// (a, c -> -a, -c), another lane's entering value (a -> -a, and x_in -> -x_in on the rerun).
template <typename R>
__host__ __device__ __forceinline__ void wrap_map(bool wrap, bool before, R& a, C2<R>& c) {
    a = wrap ? -a : a;
    const bool nc = wrap && before;
    c = mk<R>(nc ? -c.x : c.x, nc ? -c.y : c.y);
}
template <typename R>
__host__ __device__ __forceinline__ C2<R> wrap_entry(bool wrap, bool before, C2<R> x) {
    const bool nx = wrap && !before;
    return mk<R>(nx ? -x.x : x.x, nx ? -x.y : x.y);
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

// sum |v|^2 over a chunk, accumulated in R.
template <typename R, int MC, class N>
__host__ __device__ __forceinline__ R chunk_norm2(const C2<R> (&v)[MC], N n) {
    R s = R(0);
#pragma unroll
    for (int j = 0; j < MC; ++j)
        if (j < n) s += v[j].x * v[j].x + v[j].y * v[j].y;
    return s;
}
// Makes b available only after a has been computed (an empty asm that takes and returns both).
template <typename R>
__host__ __device__ __forceinline__ void order_pin(R& a, R& b) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(a), "+v"(b));
#else
    (void)a;
    (void)b;
#endif
}

// Both recurrences on one thread's chunk (n values from tau = sp.t0), with the workgroup's map
// exchange in LDS (a, c, x: Q x 64 entries, x one row more).  z comes out scaled by `scale`.
// Returns sum |y|^2 over the chunk (y = K^{-1} r).  Between the barriers: the maps are written
// before the first, read by the closing wave before the second; the entering values are read
// after the second, and the next closing wave writes them only after the third, which every
// wave reaches after its reads.
template <typename R, int MC, class N>
__device__ __forceinline__ double pc_tau_solve(C2<R> (&v)[MC], N n, ChunkSpan sp, int Lt, R b, R scale, R* sa,
                                               C2<R>* sc, C2<R>* sx, int q, int lane, int Q) {
    const RecCoef<R> k = rec_coef(b);
    const bool wk = sp.n > 0 && sp.t0 + sp.n == Lt;   // holds tau = N_tau - 1 (K's wrap)
    const bool wkd = sp.n > 0 && sp.t0 == 0;          // holds tau = 0 (K^dagger's wrap)
    R a;
    C2<R> c;
    // y = K^{-1} r: the registers walked up
    chunk_scale<R, MC>(v, k.B);
    chunk_map<R, MC, true>(v, n, k, a, c);
    wrap_map<R>(wk, k.before, a, c);
    sa[q * kPcCols + lane] = a;
    sc[q * kPcCols + lane] = c;
    __syncthreads();
    if (q == 0) chunk_close<R>(sa + lane, sc + lane, sx + lane, Q, kPcCols, k.before);
    __syncthreads();
    const C2<R> x1 = wrap_entry<R>(wk, k.before, sx[(k.before ? q : q + 1) * kPcCols + lane]);
    chunk_apply<R, MC, true>(v, n, k, x1);
    // then z = K^{-dagger} y, scaled: the registers walked down.  The norm is taken before the
    // values are scaled (deferred, it would hold y and B y at once).
    R nrm = chunk_norm2<R, MC>(v, n);
    R B2 = k.B * scale;
    order_pin(nrm, B2);
    chunk_scale<R, MC>(v, B2);
    chunk_map<R, MC, false>(v, n, k, a, c);
    wrap_map<R>(wkd, k.before, a, c);
    sa[q * kPcCols + lane] = a;
    sc[q * kPcCols + lane] = c;
    __syncthreads();
    if (q == 0) chunk_close<R>(sa + lane, sc + lane, sx + lane, Q, kPcCols, !k.before);
    __syncthreads();
    const C2<R> x2 = wrap_entry<R>(wkd, k.before, sx[(k.before ? q + 1 : q) * kPcCols + lane]);
    chunk_apply<R, MC, false>(v, n, k, x2);
    return double(nrm);
}

// Dynamic LDS of the tau pass for Q chunks per column.
template <typename R>
__host__ __device__ inline size_t pc_tau_lds(int Q) {
    return size_t(Q) * kPcCols * (sizeof(R) + sizeof(C2<R>)) + size_t(Q + 1) * kPcCols * sizeof(C2<R>);
}

// Pass 2: one workgroup per (component, group of 64 columns) of a unit, 64 Q threads (lane:
// column, wavefront: chunk), Q = blockDim / 64 at least each lattice's pc_chunks.  FULL: every
// lattice of the launch has N_tau = Q pc_chunk_max, so every chunk is full.
template <typename R, class Geo, bool FULL>
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
    // the lattice's own chunks (a batch launch has as many as the longest of its lattices needs;
    // chunks beyond a lattice's own are empty, identity maps, so each lattice is cut the same
    // way in a batch as on its own)
    const ChunkSpan sp = pc_chunk_span<R>(q, Lt);
    using N = typename std::conditional<FULL, FixedLen<MC>, int>::type;
    const N n = N(sp.n);
    const PcBlob bl = pc_blob_layout(L, Lt);
    const R b = on ? R(pc_column_b(col, L, comp >> 1, blob + pos.pcoff + bl.cosx, cf)) : R(1);
    const bool rev = !(b <= R(1) && b >= R(-1));   // K^{-1} runs backward: chunk held reversed
    // Element j of the chunk at byte offset o0 + j * ob from the chunk's first row (a base shared
    // by the wavefront), in 32 bits: at most pc_chunk_max rows of an L x L slice.
    const char* zb = reinterpret_cast<const char*>(z + pos.voff + size_t(comp) * lat.vol + size_t(sp.t0) * LL);
    const int rowb = LL * int(sizeof(C2<R>));
    // a lane past the slice's last column runs a copy of that column (b = 1; its results are
    // neither stored nor counted), so that the loads need no lane mask
    const unsigned o0 = unsigned(on ? col : LL - 1) * unsigned(sizeof(C2<R>)) +
                        (rev && n > 0 ? unsigned(int(n) - 1) * unsigned(rowb) : 0u);
    int ob = rev ? -rowb : rowb;
    auto at = [&](int j) { return reinterpret_cast<C2<R>*>(const_cast<char*>(zb) + (o0 + unsigned(j * ob))); };
    // Registers j and MC - 1 - j are loaded and stored back to back: in a full chunk they cover
    // the same two rows between the forward and the reversed lanes, so each pair writes whole
    // cache lines while they are still in L2.
    C2<R> v[MC];
#pragma unroll
    for (int i = 0; i < MC; ++i) {
        const int j = (i & 1) ? MC - 1 - (i >> 1) : (i >> 1);
        v[j] = j < n ? *at(j) : mk<R>(R(0), R(0));
    }
    // the stores recompute their addresses rather than keep the loads' live through the solve
    asm volatile("" : "+v"(ob));
    R* sa = reinterpret_cast<R*>(pc_smem);
    C2<R>* sc = reinterpret_cast<C2<R>*>(sa + Q * kPcCols);
    C2<R>* sx = sc + Q * kPcCols;
    // z is stored with the inverse transform's 1 / L^2
    const double pl = pc_tau_solve<R, MC>(v, n, sp, Lt, b, R(1) / R(LL), sa, sc, sx, q, lane, Q);
    const double part = on ? pl : 0.0;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
        const int j = (i & 1) ? MC - 1 - (i >> 1) : (i >> 1);
        if (j < n && on) *at(j) = v[j];
    }
    store_partial(ctl, PEND_RZ, pos, part / double(LL));
    if (threadIdx.x == 0) {
        S.zstage = 2;
        S.pending = PEND_RZ;
    }
    cg_publish(ctl, pos);
}

}  // namespace hmc
