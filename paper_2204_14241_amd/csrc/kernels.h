// kernels.h -- gfx950 kernels of libhmc: the fermion-matrix stencil (Eq. 17) and its
// adjoint, the fused conjugate-gradient steps on M^dagger M (Eq. 22), FP64 reliable
// updates, deterministic FP64 reductions, the pseudofermion and boson gradients and the
// leapfrog updates (Methods D).
//
// Work decomposition: one thread per lattice site handles all four spinor components
// (the Yukawa term couples them); a 256-thread tile covers 256 consecutive sites in
// (tau, x, y) order.  Workgroup ids are permuted so each of the 8 XCDs sweeps a
// contiguous slab of the lattice (stencil neighbours then hit its L2).  Every operation
// here is a bandwidth-bound sparse stencil or vector update, so no matrix cores are used.
//
// Global reductions never use fences or atomics: on the multi-XCD gfx950 an agent-scope
// release writes back the whole L2, which would serialise thousands of workgroups.
// Instead each workgroup stores one partial sum, and the consumer -- the next kernel in
// the stream -- sums the partials in index order at its start (every workgroup obtains
// the bit-identical total), or a one-workgroup kernel does.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"

namespace hmc {

constexpr int kBlock = 256;

__device__ __forceinline__ bool finite(double x) { return x - x == 0.0; }

// ------------------------------------------------------------------------------------
// Deterministic block reduction of NQ doubles: butterfly within each 64-wide wavefront,
// then a fixed-order sum over the wavefronts.  Totals are valid in thread 0.
template <int NQ>
__device__ __forceinline__ void block_reduce(double (&v)[NQ]) {
    __shared__ double sh[NQ][16];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double a = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        v[q] = a;
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) sh[q][w] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double a = 0.0;
            for (int i = 0; i < nw; ++i) a += sh[q][i];
            v[q] = a;
        }
    }
    __syncthreads();
}

// Sum n partials in a fixed order (strided by thread, then block_reduce); valid in thread 0.
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int n) {
    double v[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += blockDim.x) v[0] += p[j];
    block_reduce<1>(v);
    return v[0];
}

// ------------------------------------------------------------------------------------
// CG bookkeeping kept on the device, one record per right-hand side, double-buffered:
// kernel number s of a solve reads records[s % 2] and (workgroup 0) writes
// records[(s + 1) % 2], so no workgroup ever sees a record changed by its own launch.
enum CgMode : int {
    CG_ACTIVE = 0,      // iterating
    CG_CONV_ITER = 1,   // iterated residual reached the stop, or fell by the factor that calls
                        // for a reliable update; waits for the FP64 true residual
    CG_MAXIT = 2,       // iteration cap reached; x not yet finalised
    CG_DONE = 3,        // true residual passed
    CG_STOPPED = 4,     // iteration cap reached, x finalised
    CG_FAILED = 5,      // a reduction was not finite
};
enum : int {
    F_ACTIVE = 1 << CG_ACTIVE,
    F_CONV_ITER = 1 << CG_CONV_ITER,
    F_MAXIT = 1 << CG_MAXIT,
};
// Which partial sums the previous kernel left to be reduced.
enum CgPending : int { PEND_NONE = 0, PEND_BB = 1, PEND_TT = 2, PEND_RR = 3, PEND_RU = 4, PEND_RZ = 5 };
constexpr int kPendKinds = 5;

struct CgState {
    double bb;          // |b|^2
    double tol2;        // tol^2
    double stop_rr;     // tol^2 |b|^2
    double rr;          // current iterated |r|^2
    double rr_prev;     // |r|^2 of the previous iteration
    double alpha;       // step still to be added to x along the current p (pending)
    double alpha_old;   // step still to be added along the previous p, held in the other
                        // direction buffer (0: none; step A adds both every second iteration)
    double alpha_cur;   // step of the iteration in flight
    double beta;        // coefficient of the next direction update p <- r + beta p
    double rr_true;     // last FP64 true residual |b - A x|^2
    double drop2;       // reliable update once |r|^2 falls below drop2 times its value at the
                        // last true residual (0: only at the stop)
    double ru_rr;       // that threshold
    double rz;          // <r, z> of the current residual, z = P r (z = r without preconditioner)
    double rz_prev;     // <r, z> of the previous residual
    int mode;
    int iters;
    int pbuf;           // which of the two direction buffers holds the current p
    int n_ru;           // FP64 true-residual recomputations
    int maxit;
    int pending;        // CgPending
    int pc;             // 1: Fourier-preconditioned (z = P r computed by the three pc passes)
    int zstage;         // pc: 0 z current; 1 forward (x, y) transform done; 2 tau pass done
    int zinit;          // pc: the next <r, z> is the first of the solve (no direction to keep)
    int pad;
};

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

// One right-hand side of one lattice: the unit the CG state machine tracks.  A solve on a
// single lattice has one unit per right-hand side; a batch of independent lattices (chains)
// of different sizes has one per (chain, right-hand side), all in one launch.
struct UnitDesc {
    Lat lat;            // geometry of the unit's lattice
    long long voff;     // first complex element of the unit's vector in the spinor arrays
    long long phioff;   // first element of its lattice's boson field
    int bpr;            // workgroups on the unit; workgroup b takes tiles b, b + bpr, ...
    int part;           // first partial-sum slot of the unit (within one kind)
    int chain;          // lattice the unit belongs to
    int pcoff;          // first double of its lattice's preconditioner tables
    MarchPlan mp;       // step A as a march in this launch shape's precision (march.h)
    int mparts;         // its workgroups (bands x segments); 0: the tile kernels
    MarchPlan rmp;      // the reliable update's FP64 marches
    int rparts;         // their workgroups; 0: the tile kernels
};

// Where a workgroup works: its unit and its rank within the unit.
struct UPos {
    Lat lat;
    size_t voff, phioff;
    int k;              // unit (state record index)
    int blk;            // workgroup within the unit
    int bpr;            // CG workgroups on the unit (the count of its step partials)
    int part;           // first partial slot of the unit
    int pcoff;          // first double of the preconditioner tables of its lattice
    int mparts;         // batch: workgroups of the unit's step-A march (0 for one lattice)
    int rparts;         // batch: workgroups of the unit's reliable-update marches
};

// One lattice: unit k = right-hand side k; a launch runs nblk workgroups per unit in k-major
// order (nblk = bpr for the CG steps, the slice or column-group count for the preconditioner
// passes); each unit owns pstride partial slots per kind.
struct GeoOne {
    Lat lat;
    int bpr;
    int nblk;
    int pstride;
    __device__ __forceinline__ UPos unit(int k, int blk) const {
        UPos p;
        p.lat = lat;
        p.voff = size_t(k) * 4 * lat.vol;
        p.phioff = 0;
        p.k = k;
        p.blk = blk;
        p.bpr = bpr;
        p.part = k * pstride;
        p.pcoff = 0;
        p.mparts = p.rparts = 0;
        return p;
    }
    __device__ __forceinline__ UPos at(int logical) const {
        const int k = logical / nblk;
        return unit(k, logical - k * nblk);
    }
};

// A ragged batch: blocks[logical] = (unit, workgroup within the unit).
struct GeoBatch {
    const UnitDesc* units;
    const int2* blocks;
    __device__ __forceinline__ UPos unit(int k, int blk) const {
        const UnitDesc& u = units[k];
        UPos p;
        p.lat = u.lat;
        p.voff = size_t(u.voff);
        p.phioff = size_t(u.phioff);
        p.k = k;
        p.blk = blk;
        p.bpr = u.bpr;
        p.part = u.part;
        p.pcoff = u.pcoff;
        p.mparts = u.mparts;
        p.rparts = u.rparts;
        return p;
    }
    __device__ __forceinline__ UPos at(int logical) const {
        const int2 e = blocks[logical];
        return unit(e.x, e.y);
    }
};

// Tiles of workgroup blk among the bpr workgroups of a unit with nt tiles.  When bpr is a
// multiple of the XCD count, the tiles are cut into kNumXcd contiguous regions and the
// bpr / kNumXcd workgroups of region g stride through it together (with the XCD remap, the
// workgroups of a region share an XCD when the unit's workgroups are XCD-aligned): the
// time-slice neighbours of the tiles a region is working on are then the tiles it has just
// done or does next, still in that XCD's L2.  Otherwise workgroup b takes tiles b, b + bpr, ...
// Either way the workgroups partition [0, nt).
struct TileSpan {
    int first, end, step;
};
__host__ __device__ __forceinline__ TileSpan tile_span(int blk, int bpr, int nt) {
    TileSpan t;
    if (bpr % kNumXcd == 0) {
        const int per = bpr / kNumXcd;
        const int g = blk / per, m = blk - g * per;
        const int lo = int((long long)g * nt / kNumXcd), hi = int((long long)(g + 1) * nt / kNumXcd);
        t.first = lo + m;
        t.end = hi;
        t.step = per;
    } else {
        t.first = blk;
        t.end = nt;
        t.step = bpr;
    }
    return t;
}

__device__ __forceinline__ int tiles1(const Lat& l) { return (l.vol + kBlock - 1) / kBlock; }
__device__ __forceinline__ int tiles2(const Lat& l) { return (l.vol / 2 + kBlock - 1) / kBlock; }

// State records and partial sums of the CG kernels.
struct CgCtl {
    const CgState* st_in;
    CgState* st_out;
    double* part;       // partial sums [kPendKinds][nslots]
    int nslots;         // partial slots per kind
    int expect;         // the only partial kind that can be pending at this launch
    int nparts;         // > 0: partials the previous kernel left per unit (when its workgroup
                        // count differs from the caller's default); kPartsMarch / kPartsRu:
                        // each unit's own march workgroup count (a batch's march launches)
};
constexpr int kPartsMarch = -1;
constexpr int kPartsRu = -2;

__device__ __forceinline__ double* part_slot(const CgCtl& c, int kind, const UPos& p) {
    return c.part + size_t(kind - 1) * c.nslots + p.part;
}

constexpr int kStateWords = int(sizeof(CgState) / 4);
static_assert(sizeof(CgState) % 4 == 0 && kStateWords <= kBlock, "state record layout");

// The workgroup's copy of its right-hand side's record (one per kernel).
__device__ __forceinline__ CgState& cg_shared() {
    __shared__ CgState sh;
    return sh;
}

// Reduce the pending partials of right-hand side k (nparts of them, as many as the producing
// kernel ran workgroups on the unit) and advance its state machine into cg_shared().  Every
// workgroup computes the same record (deterministic order).  The record (one dword per lane)
// and the partials the host expects to be pending are loaded in the same memory round trip;
// the partials are used only if the record says so.  Returns the kind consumed (PEND_NONE if
// nothing was pending).  A pending kind other than the expected one (a sequencing error of
// the host) fails the right-hand side instead of using foreign partials.
__device__ __forceinline__ int cg_finalize(const CgCtl& c, const UPos& pos, int nparts) {
    const int k = pos.k;
    CgState& sh = cg_shared();
    __shared__ int consumed;
    const int t = threadIdx.x;
    unsigned w = 0u;
    if (t < kStateWords) w = reinterpret_cast<const unsigned*>(c.st_in + k)[t];
    double tot = 0.0;
    if (c.expect != PEND_NONE) {
        const int np = c.nparts > 0 ? c.nparts
                       : c.nparts == kPartsMarch ? pos.mparts
                       : c.nparts == kPartsRu ? pos.rparts : nparts;
        tot = sum_partials(part_slot(c, c.expect, pos), np);
    }
    if (t < kStateWords) reinterpret_cast<unsigned*>(&sh)[t] = w;
    __syncthreads();
    if (t == 0) {
        CgState& s = sh;
        consumed = s.pending;
        if (s.pending != PEND_NONE && s.pending != c.expect) {
            s.mode = CG_FAILED;
        } else {
            switch (s.pending) {
                case PEND_BB:
                    s.bb = tot;
                    s.stop_rr = s.tol2 * tot;
                    s.rr = s.rr_prev = s.rr_true = tot;
                    s.rz = s.rz_prev = tot;
                    s.ru_rr = s.drop2 * tot;
                    s.zinit = 1;
                    s.zstage = 0;
                    s.mode = !finite(tot) ? CG_FAILED : (tot > 0.0 ? CG_ACTIVE : CG_DONE);
                    break;
                case PEND_TT:
                    if (s.mode == CG_ACTIVE) {
                        if (!(tot > 0.0) || !finite(tot)) s.mode = CG_FAILED;
                        else s.alpha_cur = s.rz / tot;
                    }
                    break;
                case PEND_RR:
                    if (s.mode == CG_ACTIVE) {
                        if (!finite(tot)) {
                            s.mode = CG_FAILED;
                        } else {
                            s.rz_prev = s.rz;
                            if (!s.pc) {
                                s.beta = tot / s.rz;
                                s.rz = tot;
                            }
                            s.rr_prev = s.rr;
                            s.rr = tot;
                            s.alpha = s.alpha_cur;
                            s.iters += 1;
                            if (tot <= s.stop_rr || tot <= s.ru_rr) s.mode = CG_CONV_ITER;
                            else if (s.iters >= s.maxit) s.mode = CG_MAXIT;
                        }
                    }
                    break;
                case PEND_RU:
                    s.rr_true = tot;
                    s.n_ru += 1;
                    s.alpha = 0.0;
                    s.alpha_old = 0.0;
                    if (!finite(tot)) {
                        s.mode = CG_FAILED;
                    } else if (tot <= s.stop_rr) {
                        s.mode = CG_DONE;
                    } else if (s.mode == CG_MAXIT) {
                        s.mode = CG_STOPPED;
                    } else {
                        if (!s.pc) {
                            s.beta = tot / s.rz_prev;
                            s.rz = tot;
                        }
                        s.rr = tot;
                        s.ru_rr = s.drop2 * tot;
                        s.mode = CG_ACTIVE;
                    }
                    break;
                case PEND_RZ:
                    if (s.mode == CG_ACTIVE) {
                        if (!(tot > 0.0) || !finite(tot)) {
                            s.mode = CG_FAILED;
                        } else if (s.zinit) {
                            s.beta = 0.0;
                            s.rz = tot;
                            s.zinit = 0;
                        } else {
                            s.beta = tot / s.rz_prev;
                            s.rz = tot;
                        }
                    }
                    s.zstage = 0;
                    break;
            }
        }
        s.pending = PEND_NONE;
    }
    __syncthreads();
    return consumed;
}

// Workgroup 0 of a right-hand side publishes the record for the next kernel (all threads
// of the workgroup call this; changes made by thread 0 before it are included).
__device__ __forceinline__ void cg_publish(const CgCtl& c, const UPos& pos) {
    __syncthreads();
    if (pos.blk == 0 && threadIdx.x < kStateWords)
        reinterpret_cast<unsigned*>(c.st_out + pos.k)[threadIdx.x] =
            reinterpret_cast<const unsigned*>(&cg_shared())[threadIdx.x];
}

// ------------------------------------------------------------------------------------
// The stencil of Eq. (17) at one site.  Src(c, i) yields component c of the input at
// site i (a plain load, or an expression such as r + beta p evaluated on the fly).
//   (M psi)_c     = diag_b psi_c + sum_d hop_bd [psi_c(r+d) + psi_c(r-d)]
//                   + sfwd psi_c(tau+1) + Yukawa_c
//   (M^+ psi)_c   = the same with sbwd psi_c(tau-1)
//   Yukawa (band a, spin s) = dtau lambda (-1)^(x+y) sum_s' (phi . Pauli)_{s s'} psi_{other band, s'}
// with phi . Pauli = [[phi3, phi1 - i phi2], [phi1 + i phi2, -phi3]].
template <typename R, bool DAG, bool NN2, class Src>
__device__ __forceinline__ void dslash_site(const Src& src, const R* __restrict__ phi,
                                            const Lat& lat, const Coef<R>& cf, const Nbr& nb,
                                            int s, C2<R> (&out)[4], C2<R> (&cen)[4]) {
    const int vol = lat.vol;
#pragma unroll
    for (int c = 0; c < 4; ++c) cen[c] = src(c, s);
    const int st = DAG ? nb.tm : nb.tp;
    const R ts = R(DAG ? nb.sbwd : nb.sfwd);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int a = c >> 1;
        const C2<R> hx = add<R>(src(c, nb.xp), src(c, nb.xm));
        const C2<R> hy = add<R>(src(c, nb.yp), src(c, nb.ym));
        const C2<R> tt = src(c, st);
        C2<R> o = scl<R>(cf.diag[a], cen[c]);
        o = axpy<R>(cf.hop[a][0], hx, o);
        o = axpy<R>(cf.hop[a][1], hy, o);
        o = axpy<R>(ts, tt, o);
        out[c] = o;
    }
    if constexpr (NN2) {   // hops by two sites along each axis (the production model's NNN terms)
        const Nbr2 n2 = neighbours2(lat, nb, s);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int a = c >> 1;
            out[c] = axpy<R>(cf.hop2[a][0], add<R>(src(c, n2.xpp), src(c, n2.xmm)), out[c]);
            out[c] = axpy<R>(cf.hop2[a][1], add<R>(src(c, n2.ypp), src(c, n2.ymm)), out[c]);
        }
    }
    const R g = cf.cpl * R(nb.stag);
    const R q1 = g * phi[s], q2 = g * phi[vol + s], q3 = g * phi[2 * vol + s];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const C2<R> u = cen[2 * (1 - a)], w = cen[2 * (1 - a) + 1];
        // spin up:   q3 u + (q1 - i q2) w
        out[2 * a].x += q3 * u.x + q1 * w.x + q2 * w.y;
        out[2 * a].y += q3 * u.y + q1 * w.y - q2 * w.x;
        // spin down: (q1 + i q2) u - q3 w
        out[2 * a + 1].x += q1 * u.x - q2 * u.y - q3 * w.x;
        out[2 * a + 1].y += q1 * u.y + q2 * u.x - q3 * w.y;
    }
}

template <typename R>
struct SrcPlain {
    const C2<R>* __restrict__ v;
    int vol;
    __device__ __forceinline__ C2<R> operator()(int c, int i) const { return v[c * vol + i]; }
};

// p_new = r + beta * p_old, formed at every stencil point
template <typename R>
struct SrcXpay {
    const C2<R>* __restrict__ r;
    const C2<R>* __restrict__ p;
    R beta;
    int vol;
    __device__ __forceinline__ C2<R> operator()(int c, int i) const {
        return axpy<R>(beta, p[c * vol + i], r[c * vol + i]);
    }
};

// ------------------------------------------------------------------------------------
// out = M in (or M^dagger) for every unit of the geometry; workgroup b of a unit takes its
// 256-site tiles b, b + bpr, ...
template <typename R, bool DAG, class Geo, bool NN2>
__global__ __launch_bounds__(kBlock) void k_apply(Geo geo, const C2<R>* __restrict__ in,
                                                  C2<R>* __restrict__ out,
                                                  const R* __restrict__ phi_base, Coef<R> cf) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const R* phi = phi_base + pos.phioff;
    SrcPlain<R> src{in + pos.voff, lat.vol};
    C2<R>* dst = out + pos.voff;
    const int nt = tiles1(lat);
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, nt); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = tile * kBlock + threadIdx.x;
        if (s >= lat.vol) break;
        const Nbr nb = neighbours(lat, s);
        C2<R> o[4], cen[4];
        dslash_site<R, DAG, NN2>(src, phi, lat, cf, nb, s, o, cen);
#pragma unroll
        for (int c = 0; c < 4; ++c) dst[c * lat.vol + s] = o[c];
    }
}

// Vectors of one conjugate-gradient solve in the Krylov precision R.
template <typename R>
struct CgVecs {
    C2<R>* r;       // residual
    C2<R>* p0;      // direction, buffer 0
    C2<R>* p1;      // direction, buffer 1
    C2<R>* t;       // M p
    C2<R>* x;       // solution accumulated in R (the caller's x in FP64 mode)
    C2<R>* z;       // preconditioned residual P r (the residual itself without preconditioner)
};

// Store this workgroup's partial (thread 0) after a block reduction.
__device__ __forceinline__ void store_partial(const CgCtl& c, int kind, const UPos& p, double v) {
    double a[1] = {v};
    block_reduce<1>(a);
    if (threadIdx.x == 0) part_slot(c, kind, p)[p.blk] = a[0];
}

// CG step A (iteration k):  p_k = r_k + beta_{k-1} p_{k-1};  t = M p_k;  partial |t|^2 =
// <p_k, M^dagger M p_k>.  p is double-buffered because neighbouring sites read the old
// direction.  The solution is updated every second iteration: when the previous step A left its
// step pending (alpha_old), x += alpha_{k-2} p_{k-2} + alpha_{k-1} p_{k-1}, p_{k-2} read from the
// buffer about to receive p_k; otherwise x is not touched and alpha_{k-1} becomes alpha_old.
// Per iteration that is 1.5 vector reads and 0.5 writes for x instead of one of each.
template <typename R, class Geo, bool NN2>
__global__ __launch_bounds__(kBlock) void k_cg_a(CgCtl ctl, Geo geo, CgVecs<R> v,
                                                 const R* __restrict__ phi_base, Coef<R> cf) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const R* phi = phi_base + pos.phioff;
    cg_finalize(ctl, pos, pos.bpr);
    const CgState& S = cg_shared();
    if (S.mode != CG_ACTIVE) {
        cg_publish(ctl, pos);
        return;
    }
    const R alpha = R(S.alpha), alpha_old = R(S.alpha_old), beta = R(S.beta);
    const bool fold = S.alpha_old != 0.0;
    const double defer = S.alpha;
    const int pb = S.pbuf;
    const size_t off = pos.voff;
    const C2<R>* pin = (pb ? v.p1 : v.p0) + off;
    C2<R>* pout = (pb ? v.p0 : v.p1) + off;
    C2<R>* x = v.x + off;
    C2<R>* t = v.t + off;
    SrcXpay<R> src{v.z + off, pin, beta, lat.vol};
    double part = 0.0;
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, tiles1(lat)); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = tile * kBlock + threadIdx.x;
        if (s < lat.vol) {
            if (fold) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int i = c * lat.vol + s;
                    x[i] = axpy<R>(alpha, pin[i], axpy<R>(alpha_old, pout[i], x[i]));
                }
            }
            const Nbr nb = neighbours(lat, s);
            C2<R> o[4], pn[4];
            dslash_site<R, false, NN2>(src, phi, lat, cf, nb, s, o, pn);
            R acc = R(0);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int i = c * lat.vol + s;
                pout[i] = pn[c];
                t[i] = o[c];
                acc += norm2<R>(o[c]);
            }
            part += double(acc);
        }
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

// CG step B:  r -= alpha_k M^dagger t;  partial |r|^2.
template <typename R, class Geo, bool NN2>
__global__ __launch_bounds__(kBlock) void k_cg_b(CgCtl ctl, Geo geo, CgVecs<R> v,
                                                 const R* __restrict__ phi_base, Coef<R> cf) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const R* phi = phi_base + pos.phioff;
    cg_finalize(ctl, pos, pos.bpr);
    const CgState& S = cg_shared();
    if (S.mode != CG_ACTIVE) {
        cg_publish(ctl, pos);
        return;
    }
    const R alpha = R(S.alpha_cur);
    const size_t off = pos.voff;
    SrcPlain<R> src{v.t + off, lat.vol};
    C2<R>* r = v.r + off;
    double part = 0.0;
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, tiles1(lat)); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = tile * kBlock + threadIdx.x;
        if (s < lat.vol) {
            const Nbr nb = neighbours(lat, s);
            C2<R> o[4], cen[4];
            dslash_site<R, true, NN2>(src, phi, lat, cf, nb, s, o, cen);
            R acc = R(0);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int i = c * lat.vol + s;
                const C2<R> rn = axpy<R>(-alpha, o[c], r[i]);
                r[i] = rn;
                acc += norm2<R>(rn);
            }
            part += double(acc);
        }
    }
    store_partial(ctl, PEND_RR, pos, part);
    if (threadIdx.x == 0) cg_shared().pending = PEND_RR;
    cg_publish(ctl, pos);
}

// Reliable update, part 1 (elementwise): fold the pending steps into the FP64 solution,
// x64 += alpha_old p_prev + alpha p + x_lo (mixed) or x64 += alpha_old p_prev + alpha p (FP64,
// where v.x is x64), clear x_lo.
template <typename R, class Geo>
__global__ __launch_bounds__(kBlock) void k_ru_fold(CgCtl ctl, Geo geo, double2* __restrict__ x64,
                                                    CgVecs<R> v, int filter) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    cg_finalize(ctl, pos, pos.bpr);
    const CgState& S = cg_shared();
    if (!((1 << S.mode) & filter)) {
        cg_publish(ctl, pos);
        return;
    }
    const double alpha = S.alpha, alpha_old = S.alpha_old;
    const size_t off = pos.voff;
    const C2<R>* p = (S.pbuf ? v.p1 : v.p0) + off;
    const C2<R>* q = (S.pbuf ? v.p0 : v.p1) + off;   // the previous direction
    const bool separate = (void*)v.x != (void*)x64, both = alpha_old != 0.0;
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, tiles1(lat)); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = tile * kBlock + threadIdx.x;
        if (s >= lat.vol) break;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const size_t i = off + size_t(c) * lat.vol + s;
            const C2<R> pc = p[c * lat.vol + s];
            double2 xv = x64[i];
            if (both) {
                const C2<R> qc = q[c * lat.vol + s];
                xv.x += alpha_old * double(qc.x);
                xv.y += alpha_old * double(qc.y);
            }
            xv.x += alpha * double(pc.x);
            xv.y += alpha * double(pc.y);
            if (separate) {
                const C2<R> xl = v.x[i];
                xv.x += double(xl.x);
                xv.y += double(xl.y);
                v.x[i] = mk<R>(R(0), R(0));
            }
            x64[i] = xv;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) cg_shared().alpha = cg_shared().alpha_old = 0.0;
    cg_publish(ctl, pos);
}

// Reliable update, part 2: t64 = M x64 (FP64) for right-hand sides in `filter`.
template <class Geo, bool NN2>
__global__ __launch_bounds__(kBlock) void k_ru_apply(CgCtl ctl, Geo geo, const double2* __restrict__ x64,
                                                     double2* __restrict__ t64,
                                                     const double* __restrict__ phi_base,
                                                     Coef<double> cf, int filter) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const double* phi = phi_base + pos.phioff;
    cg_finalize(ctl, pos, pos.bpr);
    const int mode = cg_shared().mode;
    cg_publish(ctl, pos);
    if (!((1 << mode) & filter)) return;
    const size_t off = pos.voff;
    SrcPlain<double> src{x64 + off, lat.vol};
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, tiles1(lat)); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = tile * kBlock + threadIdx.x;
        if (s >= lat.vol) break;
        const Nbr nb = neighbours(lat, s);
        double2 o[4], cen[4];
        dslash_site<double, false, NN2>(src, phi, lat, cf, nb, s, o, cen);
#pragma unroll
        for (int c = 0; c < 4; ++c) t64[off + size_t(c) * lat.vol + s] = o[c];
    }
}

// Reliable update, part 3: r = b - M^dagger t64 in FP64, stored in the Krylov precision;
// partial |r|^2 in FP64 (reduced by the next kernel: DONE, STOPPED or back to ACTIVE).
template <typename R, class Geo, bool NN2>
__global__ __launch_bounds__(kBlock) void k_ru_resid(CgCtl ctl, Geo geo, const double2* __restrict__ b,
                                                     const double2* __restrict__ t64,
                                                     const double* __restrict__ phi_base,
                                                     Coef<double> cf, C2<R>* __restrict__ r,
                                                     int filter) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const double* phi = phi_base + pos.phioff;
    cg_finalize(ctl, pos, pos.bpr);
    if (!((1 << cg_shared().mode) & filter)) {
        cg_publish(ctl, pos);
        return;
    }
    const size_t off = pos.voff;
    SrcPlain<double> src{t64 + off, lat.vol};
    double part = 0.0;
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, tiles1(lat)); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = tile * kBlock + threadIdx.x;
        if (s < lat.vol) {
            const Nbr nb = neighbours(lat, s);
            double2 o[4], cen[4];
            dslash_site<double, true, NN2>(src, phi, lat, cf, nb, s, o, cen);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = off + size_t(c) * lat.vol + s;
                const double2 rv = sub<double>(b[i], o[c]);
                part += norm2<double>(rv);
                r[i] = mk<R>(R(rv.x), R(rv.y));
            }
        }
    }
    store_partial(ctl, PEND_RU, pos, part);
    if (threadIdx.x == 0) cg_shared().pending = PEND_RU;
    cg_publish(ctl, pos);
}

// CG start from x = 0: x64 = 0, r = b, both direction buffers and x_lo cleared, partial |b|^2.
template <typename R, class Geo>
__global__ __launch_bounds__(kBlock) void k_cg_init(CgCtl ctl, Geo geo, const double2* __restrict__ b,
                                                    double2* __restrict__ x64, CgVecs<R> v,
                                                    double tol2, double drop2, int maxit, int pc) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const size_t off = pos.voff;
    const bool separate = (void*)v.x != (void*)x64;
    double part = 0.0;
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, tiles1(lat)); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = tile * kBlock + threadIdx.x;
        if (s < lat.vol) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = off + size_t(c) * lat.vol + s;
                const double2 bv = b[i];
                part += norm2<double>(bv);
                x64[i] = make_double2(0.0, 0.0);
                v.r[i] = mk<R>(R(bv.x), R(bv.y));
                v.p0[i] = mk<R>(R(0), R(0));
                v.p1[i] = mk<R>(R(0), R(0));
                if (separate) v.x[i] = mk<R>(R(0), R(0));
            }
        }
    }
    store_partial(ctl, PEND_BB, pos, part);
    if (threadIdx.x == 0) {
        CgState& S = cg_shared();
        S = CgState{};
        S.tol2 = tol2;
        S.drop2 = drop2;
        S.maxit = maxit;
        S.pc = pc;
        S.mode = CG_ACTIVE;
        S.pending = PEND_BB;
    }
    cg_publish(ctl, pos);
}

// One workgroup per right-hand side: reduce whatever is pending (nparts per unit: 0 selects
// the unit's CG workgroup count) and publish the record.
template <class Geo>
__global__ __launch_bounds__(kBlock) void k_cg_finalize(CgCtl ctl, Geo geo, int nparts) {
    const UPos pos = geo.unit(blockIdx.x, 0);
    cg_finalize(ctl, pos, nparts > 0 ? nparts : pos.bpr);
    cg_publish(ctl, pos);
}

// ------------------------------------------------------------------------------------
// FP32 forms with two sites per thread.  Sites s (even) and s + 1 share a row (L is even),
// so each component plane of a pair, and of its x+-1 and tau+-1 neighbours, is one aligned
// 16-byte load; only the two outer y neighbours are single 8-byte loads.  Half the load
// instructions of the one-site form, twice the bytes per instruction.
__device__ __forceinline__ float4 f4(float a, float b, float c, float d) { return make_float4(a, b, c, d); }
__device__ __forceinline__ float4 f4add(float4 a, float4 b) { return f4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
// a + s*b
__device__ __forceinline__ float4 f4axpy(float s, float4 b, float4 a) {
    return f4(a.x + s * b.x, a.y + s * b.y, a.z + s * b.z, a.w + s * b.w);
}
__device__ __forceinline__ float f4norm2(float4 a) { return a.x * a.x + a.y * a.y + a.z * a.z + a.w * a.w; }
__device__ __forceinline__ float4 ld4(const float2* p, size_t i) { return *reinterpret_cast<const float4*>(p + i); }
__device__ __forceinline__ void st4(float2* p, size_t i, float4 v) { *reinterpret_cast<float4*>(p + i) = v; }

struct SrcPlain2 {
    const float2* __restrict__ v;
    int vol;
    __device__ __forceinline__ float4 pair(int c, int i) const { return ld4(v, size_t(c) * vol + i); }
    __device__ __forceinline__ float2 one(int c, int i) const { return v[size_t(c) * vol + i]; }
};

struct SrcXpay2 {      // r + beta p
    const float2* __restrict__ r;
    const float2* __restrict__ p;
    float beta;
    int vol;
    __device__ __forceinline__ float4 pair(int c, int i) const {
        return f4axpy(beta, ld4(p, size_t(c) * vol + i), ld4(r, size_t(c) * vol + i));
    }
    __device__ __forceinline__ float2 one(int c, int i) const {
        return axpy<float>(beta, p[size_t(c) * vol + i], r[size_t(c) * vol + i]);
    }
};

// The stencil of Eq. (17) at sites s (even) and s + 1 (lanes .x .y and .z .w of each float4).
template <bool DAG, bool NN2, class Src>
__device__ __forceinline__ void dslash_pair(const Src& src, const float* __restrict__ phi,
                                            const Lat& lat, const Coef<float>& cf, const Nbr& nb,
                                            int s, float4 (&out)[4], float4 (&cen)[4]) {
    const int vol = lat.vol, L = lat.L;
    const int yl = nb.ym;                                   // y - 1 of site s
    const int yr = (nb.y + 2 == L) ? s + 2 - L : s + 2;     // y + 1 of site s + 1
    const int st = DAG ? nb.tm : nb.tp;
    const float ts = float(DAG ? nb.sbwd : nb.sfwd);
    // hops by two sites: rows x +- 2 at the same pair, and the pairs (y - 2, y - 1) and
    // (y + 2, y + 3), all aligned (y is even and so is L); the latter two also hold the y - 1
    // and y + 2 values of the nearest-neighbour terms
    Nbr2 n2{};
    if constexpr (NN2) n2 = neighbours2(lat, nb, s);
#pragma unroll
    for (int c = 0; c < 4; ++c) cen[c] = src.pair(c, s);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int a = c >> 1;
        const float4 xp = src.pair(c, nb.xp), xm = src.pair(c, nb.xm), tt = src.pair(c, st);
        float2 lo, hi;
        float4 ym2, yp2;
        if constexpr (NN2) {
            ym2 = src.pair(c, n2.ymm);
            yp2 = src.pair(c, n2.ypp);
            lo = make_float2(ym2.z, ym2.w);
            hi = make_float2(yp2.x, yp2.y);
        } else {
            lo = src.one(c, yl);
            hi = src.one(c, yr);
        }
        const float4 ce = cen[c];
        const float dg = cf.diag[a], h0 = cf.hop[a][0], h1 = cf.hop[a][1];
        float4 o;
        o.x = dg * ce.x + h0 * (xp.x + xm.x) + h1 * (lo.x + ce.z) + ts * tt.x;
        o.y = dg * ce.y + h0 * (xp.y + xm.y) + h1 * (lo.y + ce.w) + ts * tt.y;
        o.z = dg * ce.z + h0 * (xp.z + xm.z) + h1 * (ce.x + hi.x) + ts * tt.z;
        o.w = dg * ce.w + h0 * (xp.w + xm.w) + h1 * (ce.y + hi.y) + ts * tt.w;
        if constexpr (NN2) {
            const float4 xx = f4add(src.pair(c, n2.xpp), src.pair(c, n2.xmm));
            const float4 yy = f4add(ym2, yp2);
            const float u0 = cf.hop2[a][0], u1 = cf.hop2[a][1];
            o.x += u0 * xx.x + u1 * yy.x;
            o.y += u0 * xx.y + u1 * yy.y;
            o.z += u0 * xx.z + u1 * yy.z;
            o.w += u0 * xx.w + u1 * yy.w;
        }
        out[c] = o;
    }
    const float g0 = cf.cpl * float(nb.stag), g1 = -g0;     // (-1)^(x+y) flips between s, s+1
    const float2 P1 = *reinterpret_cast<const float2*>(phi + s);
    const float2 P2 = *reinterpret_cast<const float2*>(phi + vol + s);
    const float2 P3 = *reinterpret_cast<const float2*>(phi + 2 * vol + s);
    const float q1a = g0 * P1.x, q2a = g0 * P2.x, q3a = g0 * P3.x;
    const float q1b = g1 * P1.y, q2b = g1 * P2.y, q3b = g1 * P3.y;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const float4 u = cen[2 * (1 - a)], w = cen[2 * (1 - a) + 1];
        out[2 * a].x += q3a * u.x + q1a * w.x + q2a * w.y;
        out[2 * a].y += q3a * u.y + q1a * w.y - q2a * w.x;
        out[2 * a].z += q3b * u.z + q1b * w.z + q2b * w.w;
        out[2 * a].w += q3b * u.w + q1b * w.w - q2b * w.z;
        out[2 * a + 1].x += q1a * u.x - q2a * u.y - q3a * w.x;
        out[2 * a + 1].y += q1a * u.y + q2a * u.x - q3a * w.y;
        out[2 * a + 1].z += q1b * u.z - q2b * u.w - q3b * w.z;
        out[2 * a + 1].w += q1b * u.w + q2b * u.z - q3b * w.w;
    }
}

// out_k = M in_k (or M^dagger), FP32, one 512-site tile per workgroup.
template <bool DAG, class Geo, bool NN2>
__global__ __launch_bounds__(kBlock) void k_apply2(Geo geo, const float2* __restrict__ in,
                                                   float2* __restrict__ out,
                                                   const float* __restrict__ phi_base, Coef<float> cf) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const float* phi = phi_base + pos.phioff;
    const size_t off = pos.voff;
    SrcPlain2 src{in + off, lat.vol};
    const int nt = tiles2(lat);
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, nt); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = 2 * (tile * kBlock + threadIdx.x);
        if (s >= lat.vol) break;
        const Nbr nb = neighbours(lat, s);
        float4 o[4], cen[4];
        dslash_pair<DAG, NN2>(src, phi, lat, cf, nb, s, o, cen);
#pragma unroll
        for (int c = 0; c < 4; ++c) st4(out + off, size_t(c) * lat.vol + s, o[c]);
    }
}

// CG step A, FP32 pair form (same algebra as k_cg_a).  The nearest-neighbour form is scheduled
// for five waves per SIMD: its batch instantiation otherwise takes 130 VGPRs, and the one-lattice
// kernel runs about 2% faster so scheduled; the form with the two-site hops keeps its own.
template <class Geo, bool NN2>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NN2 ? 1 : 5)))
void k_cg_a2(CgCtl ctl, Geo geo, CgVecs<float> v, const float* __restrict__ phi_base, Coef<float> cf) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const float* phi = phi_base + pos.phioff;
    cg_finalize(ctl, pos, pos.bpr);
    const CgState& S = cg_shared();
    if (S.mode != CG_ACTIVE) {
        cg_publish(ctl, pos);
        return;
    }
    const float alpha = float(S.alpha), alpha_old = float(S.alpha_old), beta = float(S.beta);
    const bool fold = S.alpha_old != 0.0;
    const double defer = S.alpha;
    const int pb = S.pbuf;
    const size_t off = pos.voff;
    const float2* pin = (pb ? v.p1 : v.p0) + off;
    float2* pout = (pb ? v.p0 : v.p1) + off;
    float2* x = v.x + off;
    float2* t = v.t + off;
    SrcXpay2 src{v.z + off, pin, beta, lat.vol};
    double part = 0.0;
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, tiles2(lat)); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = 2 * (tile * kBlock + threadIdx.x);
        if (s < lat.vol) {
            if (fold) {   // before the stencil: its registers are free again when the stencil runs
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const size_t i = size_t(c) * lat.vol + s;
                    st4(x, i, f4axpy(alpha, ld4(pin, i), f4axpy(alpha_old, ld4(pout, i), ld4(x, i))));
                }
            }
            const Nbr nb = neighbours(lat, s);
            float4 o[4], pn[4];
            dslash_pair<false, NN2>(src, phi, lat, cf, nb, s, o, pn);
            float acc = 0.f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = size_t(c) * lat.vol + s;
                st4(pout, i, pn[c]);
                st4(t, i, o[c]);
                acc += f4norm2(o[c]);
            }
            part += double(acc);
        }
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

// CG step B, FP32 pair form (same algebra as k_cg_b).
template <class Geo, bool NN2>
__global__ __launch_bounds__(kBlock) void k_cg_b2(CgCtl ctl, Geo geo, CgVecs<float> v,
                                                  const float* __restrict__ phi_base, Coef<float> cf) {
    const UPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const float* phi = phi_base + pos.phioff;
    cg_finalize(ctl, pos, pos.bpr);
    const CgState& S = cg_shared();
    if (S.mode != CG_ACTIVE) {
        cg_publish(ctl, pos);
        return;
    }
    const float alpha = float(S.alpha_cur);
    const size_t off = pos.voff;
    SrcPlain2 src{v.t + off, lat.vol};
    float2* r = v.r + off;
    double part = 0.0;
    for (TileSpan sp = tile_span(pos.blk, pos.bpr, tiles2(lat)); sp.first < sp.end; sp.first += sp.step) {
        const int tile = sp.first;
        const int s = 2 * (tile * kBlock + threadIdx.x);
        if (s < lat.vol) {
            const Nbr nb = neighbours(lat, s);
            float4 o[4], cen[4];
            dslash_pair<true, NN2>(src, phi, lat, cf, nb, s, o, cen);
            float acc = 0.f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = size_t(c) * lat.vol + s;
                const float4 rn = f4axpy(-alpha, o[c], ld4(r, i));
                st4(r, i, rn);
                acc += f4norm2(rn);
            }
            part += double(acc);
        }
    }
    store_partial(ctl, PEND_RR, pos, part);
    if (threadIdx.x == 0) cg_shared().pending = PEND_RR;
    cg_publish(ctl, pos);
}

// ------------------------------------------------------------------------------------
// Gradient dS/dphi at one site (FP64).  Pseudofermion part: for each solution x_k,
// Y = M x_k at the site, then -2 dtau lambda (-1)^(x+y) Re[Y_bx^+ Pauli_l X_by + Y_by^+ Pauli_l X_bx]
// (bx, by: the two bands, each a spin doublet).  Boson part: the derivative of the lattice
// boson action, a 7-point Laplacian form plus mass and quartic terms.
// Output: F written to `force` (if non-null) and/or `nkick` half kicks pi -= h F applied
// one after another (the leapfrog's neighbouring half kicks kept separate).
__device__ __forceinline__ void pauli_contract(double2 u0, double2 u1, double2 v0, double2 v1,
                                               double& f1, double& f2, double& f3) {
    // Re/Im of conj(a) b
    const double re01 = u0.x * v1.x + u0.y * v1.y, im01 = u0.x * v1.y - u0.y * v1.x;
    const double re10 = u1.x * v0.x + u1.y * v0.y, im10 = u1.x * v0.y - u1.y * v0.x;
    const double re00 = u0.x * v0.x + u0.y * v0.y;
    const double re11 = u1.x * v1.x + u1.y * v1.y;
    f1 += re01 + re10;     // Pauli x
    f2 += im01 - im10;     // Pauli y: Re(-i conj(u0) v1 + i conj(u1) v0)
    f3 += re00 - re11;     // Pauli z
}

// Where a site-parallel (not CG) workgroup works: one 256-site tile of one lattice.
struct ChainDesc {
    Lat lat;
    long long voff;     // first complex element of the lattice's first right-hand side
    long long phioff;   // first element of its boson field
    BosonCoef bc;
    int npf;            // right-hand sides (consecutive vectors) of the lattice
    int pad;
};
struct CPos {
    Lat lat;
    size_t voff, phioff;
    BosonCoef bc;
    int npf, tile;
};
// One lattice: workgroup = tile.
struct CGeoOne {
    Lat lat;
    BosonCoef bc;
    int npf;
    __device__ __forceinline__ CPos at(int logical) const {
        CPos p;
        p.lat = lat;
        p.voff = 0;
        p.phioff = 0;
        p.bc = bc;
        p.npf = npf;
        p.tile = logical;
        return p;
    }
};
// A ragged batch: blocks[logical] = (lattice, tile).
struct CGeoBatch {
    const ChainDesc* chains;
    const int2* blocks;
    __device__ __forceinline__ CPos at(int logical) const {
        const int2 e = blocks[logical];
        const ChainDesc& c = chains[e.x];
        CPos p;
        p.lat = c.lat;
        p.voff = size_t(c.voff);
        p.phioff = size_t(c.phioff);
        p.bc = c.bc;
        p.npf = c.npf;
        p.tile = e.y;
        return p;
    }
};

template <class CGeo, bool NN2>
__global__ __launch_bounds__(kBlock) void k_force(CGeo geo, const double2* __restrict__ x_base,
                                                  const double* __restrict__ phi_base,
                                                  Coef<double> cf, int do_pf, int do_boson,
                                                  double* __restrict__ force_base,
                                                  double* __restrict__ pi_base, double h, int nkick) {
    const CPos pos = geo.at(xcd_remap(blockIdx.x, gridDim.x));
    const Lat& lat = pos.lat;
    const int s = pos.tile * kBlock + threadIdx.x;
    if (s >= lat.vol) return;
    const int vol = lat.vol;
    const double* phi = phi_base + pos.phioff;
    const BosonCoef& bc = pos.bc;
    const Nbr nb = neighbours(lat, s);
    double F[3] = {0.0, 0.0, 0.0};
    if (do_pf) {
        double f1 = 0.0, f2 = 0.0, f3 = 0.0;
        for (int k = 0; k < pos.npf; ++k) {
            SrcPlain<double> src{x_base + pos.voff + size_t(k) * 4 * vol, vol};
            double2 Y[4], X[4];
            dslash_site<double, false, NN2>(src, phi, lat, cf, nb, s, Y, X);
            pauli_contract(Y[0], Y[1], X[2], X[3], f1, f2, f3);
            pauli_contract(Y[2], Y[3], X[0], X[1], f1, f2, f3);
        }
        const double pre = -2.0 * cf.cpl * double(nb.stag);
        F[0] = pre * f1;
        F[1] = pre * f2;
        F[2] = pre * f3;
    }
    if (do_boson) {
        double p[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) p[l] = phi[l * vol + s];
        const double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const double* f = phi + l * vol;
            const double lt = 2.0 * p[l] - f[nb.tp] - f[nb.tm];
            const double ls = 4.0 * p[l] - f[nb.xp] - f[nb.xm] - f[nb.yp] - f[nb.ym];
            F[l] += bc.kt * lt + bc.ks * ls + bc.kr * p[l] + bc.ku * p2 * p[l];
        }
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (force_base != nullptr) force_base[pos.phioff + l * vol + s] = F[l];
        if (pi_base != nullptr) {
            double* pi = pi_base + pos.phioff;
            double pv = pi[l * vol + s];
            for (int j = 0; j < nkick; ++j) pv = pv - h * F[l];
            pi[l * vol + s] = pv;
        }
    }
}

// Kinetic energy 1/2 |pi|^2 and boson action S_B (Eq. 2 on the lattice): per-workgroup
// partials part[0][logical] = K, part[stride + logical] = S_B.
template <class CGeo>
__global__ __launch_bounds__(kBlock) void k_energy(CGeo geo, const double* __restrict__ pi_base,
                                                   const double* __restrict__ phi_base,
                                                   double* part, int stride) {
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    const CPos pos = geo.at(logical);
    const Lat& lat = pos.lat;
    const int s = pos.tile * kBlock + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (s < lat.vol) {
        const int vol = lat.vol;
        const double* phi = phi_base + pos.phioff;
        const double* pi = pi_base ? pi_base + pos.phioff : nullptr;
        const BosonCoef& bc = pos.bc;
        const Nbr nb = neighbours(lat, s);
        double kin = 0.0, st = 0.0, ss = 0.0, p2 = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const double* f = phi + l * vol;
            const double c = f[s];
            if (pi != nullptr) kin += pi[l * vol + s] * pi[l * vol + s];
            const double dt = f[nb.tp] - c, dx = f[nb.xp] - c, dy = f[nb.yp] - c;
            st += dt * dt;
            ss += dx * dx + dy * dy;
            p2 += c * c;
        }
        v[0] = 0.5 * kin;
        v[1] = 0.5 * bc.kt * st + 0.5 * bc.ks * ss + 0.5 * bc.kr * p2 + 0.25 * bc.ku * p2 * p2;
    }
    block_reduce<2>(v);
    if (threadIdx.x == 0) {
        part[logical] = v[0];
        part[stride + logical] = v[1];
    }
}

// sum_k Re <a_k, b_k> over the npf spinors of the workgroup's lattice (complex128):
// per-workgroup partials in part[logical].
template <class CGeo>
__global__ __launch_bounds__(kBlock) void k_dot_re(CGeo geo, const double2* __restrict__ a,
                                                   const double2* __restrict__ b, double* part) {
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    const CPos pos = geo.at(logical);
    const Lat& lat = pos.lat;
    const int s = pos.tile * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (s < lat.vol) {
        for (int k = 0; k < pos.npf; ++k) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t i = pos.voff + (size_t(k) * 4 + c) * lat.vol + s;
                const double2 u = a[i], w = b[i];
                v[0] += u.x * w.x + u.y * w.y;
            }
        }
    }
    block_reduce<1>(v);
    if (threadIdx.x == 0) part[logical] = v[0];
}

// One workgroup per lattice c: out[c * out_stride + q] = sum of part[q * stride + j] over the
// lattice's workgroups j in [first[c], first[c + 1]), q < nq, in index order.
__global__ __launch_bounds__(kBlock) void k_sum_chains(const double* __restrict__ part, int stride,
                                                       int nq, const int* __restrict__ first,
                                                       double* out, int out_stride) {
    const int c = blockIdx.x;
    const int j0 = first[c], j1 = first[c + 1];
    for (int q = 0; q < nq; ++q) {
        const double t = sum_partials(part + size_t(q) * stride + j0, j1 - j0);
        if (threadIdx.x == 0) out[size_t(c) * out_stride + q] = t;
    }
}

// One workgroup: out[q] = sum over n partials of row q (rows `stride` apart), q < nq.
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ part, int n,
                                                         int nq, int stride, double* out) {
    for (int q = 0; q < nq; ++q) {
        const double t = sum_partials(part + size_t(q) * stride, n);
        if (threadIdx.x == 0) out[q] = t;
    }
}

// phi += eps * pi (the leapfrog drift), elementwise over 3 * vol values.
__global__ __launch_bounds__(kBlock) void k_drift(double* __restrict__ phi,
                                                  const double* __restrict__ pi, double eps,
                                                  int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) phi[i] = phi[i] + eps * pi[i];
}

// phi32 = (float) phi64
__global__ __launch_bounds__(kBlock) void k_to_f32(const double* __restrict__ a,
                                                   float* __restrict__ b, int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = float(a[i]);
}

}  // namespace hmc
