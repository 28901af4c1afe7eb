// hmc.hip -- host side of libhmc: context and workspace management, the C ABI of
// include/hmc.h, the conjugate-gradient driver (FP64 and mixed precision with FP64
// reliable updates) and the HMC trajectory driver.
//
// Every step of the path runs in the kernels of kernels.h; the host only sequences
// launches on the caller's stream and reads back per-solve status words (CG
// convergence) and the energies of a trajectory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/hmc.h"
#include "../../include/hmc_testing.h"
#include "kernels.h"
#include "lattice.h"

using namespace hmc;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(HMC_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                           \
    } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

size_t align_up(size_t n, size_t a) { return (n + a - 1) / a * a; }

constexpr int kCheckEvery = 32;     // FP64 CG: iterations between host status reads
constexpr int kSlots = 32;          // device scalars (energies, actions)
constexpr int kDefaultBpr64 = 1024; // default CG workgroups per right-hand side, FP64
constexpr int kDefaultBpr32 = 512;  // ... mixed precision (FP32 pair kernels)
constexpr int kMaxBpr = 4096;       // largest accepted (sizes the partial-sum buffer)

// Slot indices in the device scalar area.
enum Slot : int {
    SL_K0 = 0, SL_SB0 = 1, SL_K1 = 2, SL_SB1 = 3, SL_SPF0 = 4, SL_SPF1 = 5, SL_TMP = 6,
    SL_TMP2 = 7,
};

}  // namespace

struct hmc_ctx {
    int device = 0;
    int L = 0, Lt = 0, vol = 0;
    double dtau = 0.0;
    hmc_params p{};
    int cap = 1;            // right-hand sides the workspace holds
    int nblk = 0;           // 256-site tiles per right-hand side (one site per thread)
    int nblk2 = 0;          // 512-site tiles per right-hand side (FP32 pair kernels)
    int bpr = 0;            // CG workgroups per right-hand side of the solve in flight
    int bpr64 = 0;          // ... chosen for FP64 solves
    int bpr32 = 0;          // ... chosen for mixed-precision solves
    int seq = 0;            // CG launch counter (selects the state record buffer)
    Lat lat{};
    Coef<double> cf64{};
    Coef<float> cf32{};
    BosonCoef bc{};

    // workspace (caller-owned)
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t need = 0;
    // carved pointers
    CgState* st = nullptr;       // 2 * cap records (double-buffered by launch parity)
    double* part = nullptr;      // CG partial sums: 4 kinds * cap * bpr
    double* gpart = nullptr;     // generic reductions: 2 * nblk
    double* slots = nullptr;
    double2 *r64 = nullptr, *p064 = nullptr, *p164 = nullptr, *t64 = nullptr;
    float2 *r32 = nullptr, *p032 = nullptr, *p132 = nullptr, *t32 = nullptr, *x32 = nullptr;
    double2 *chi = nullptr, *xsol = nullptr;
    double *pi = nullptr, *phi_save = nullptr;
    float* phi32 = nullptr;

    // pinned host status area
    CgState* h_st = nullptr;     // 2 * cap records (double buffer)
    double* h_slots = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};

    // sampled kernel timing (timing-enabled events, one triple per status slot)
    bool timing = false;
    hipEvent_t tev[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    hmc_kernel_times kt{};
};

// --------------------------------------------------------------------------------------
// helpers

static void set_coefs(hmc_ctx* c) {
    const double dt = c->dtau;
    const hmc_params& p = c->p;
    for (int a = 0; a < 2; ++a) {
        c->cf64.diag[a] = -1.0 - dt * p.mu[a];
        for (int d = 0; d < 2; ++d) c->cf64.hop[a][d] = -dt * p.t[a][d];
    }
    c->cf64.cpl = dt * p.lambda;
    for (int a = 0; a < 2; ++a) {
        c->cf32.diag[a] = float(c->cf64.diag[a]);
        for (int d = 0; d < 2; ++d) c->cf32.hop[a][d] = float(c->cf64.hop[a][d]);
    }
    c->cf32.cpl = float(c->cf64.cpl);
    c->bc.kt = 1.0 / (p.c * p.c * dt);
    c->bc.ks = dt;
    c->bc.kr = dt * p.r;
    c->bc.ku = dt * p.u;
}

static int check_params(const hmc_params* p) {
    if (p == nullptr) return fail(HMC_ERR_INVALID_ARG, "params is NULL");
    if (!(p->c > 0.0) || !std::isfinite(p->c)) return fail(HMC_ERR_INVALID_ARG, "boson velocity c must be > 0");
    if (!std::isfinite(p->lambda) || !std::isfinite(p->r) || !std::isfinite(p->u))
        return fail(HMC_ERR_INVALID_ARG, "non-finite coupling");
    for (int a = 0; a < 2; ++a) {
        if (!std::isfinite(p->mu[a])) return fail(HMC_ERR_INVALID_ARG, "non-finite mu");
        for (int d = 0; d < 2; ++d)
            if (!std::isfinite(p->t[a][d])) return fail(HMC_ERR_INVALID_ARG, "non-finite hopping");
    }
    if (p->n_pf < 0 || p->n_pf > HMC_MAX_RHS) return fail(HMC_ERR_INVALID_ARG, "n_pf out of range [0, %d]", HMC_MAX_RHS);
    if (p->max_rhs < 0 || p->max_rhs > HMC_MAX_RHS) return fail(HMC_ERR_INVALID_ARG, "max_rhs out of range");
    if (!(p->cg_tol > 0.0) || !(p->cg_tol < 1.0)) return fail(HMC_ERR_INVALID_ARG, "cg_tol must lie in (0, 1)");
    if (p->cg_maxit < 1) return fail(HMC_ERR_INVALID_ARG, "cg_maxit must be >= 1");
    if (p->precision != HMC_FP64 && p->precision != HMC_MIXED) return fail(HMC_ERR_INVALID_ARG, "unknown precision");
    if (p->precision == HMC_MIXED && p->reliable_every < 1)
        return fail(HMC_ERR_INVALID_ARG, "reliable_every must be >= 1 in mixed precision");
    if (p->n_leap < 0) return fail(HMC_ERR_INVALID_ARG, "n_leap must be >= 0");
    if (!std::isfinite(p->eps)) return fail(HMC_ERR_INVALID_ARG, "eps not finite");
    return HMC_OK;
}

static int geometry_ok(int L, int Lt) {
    if (L < 4 || L > kMaxL || (L & 1)) return 0;
    if (Lt < 2) return 0;
    const long long vol = (long long)Lt * L * L;
    if (vol >= (1LL << kMaxVolLog2)) return 0;
    return 1;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

static int need_ws(const hmc_ctx* c) {
    if (c->ws == nullptr) return fail(HMC_ERR_WORKSPACE, "workspace not set (hmc_set_workspace)");
    return HMC_OK;
}

static int grid_for(const hmc_ctx* c, int n) { return c->nblk * n; }

static int elem_grid(long long n) { return int((n + kBlock - 1) / kBlock); }

// --------------------------------------------------------------------------------------
// conjugate gradient driver

template <typename R> struct KrylovBufs;
template <> struct KrylovBufs<double> {
    static CgVecs<double> get(hmc_ctx* c, double2* x) { return {c->r64, c->p064, c->p164, c->t64, x}; }
    static const double* phi(hmc_ctx*, const double* phi64) { return phi64; }
    static Coef<double> cf(hmc_ctx* c) { return c->cf64; }
};
template <> struct KrylovBufs<float> {
    static CgVecs<float> get(hmc_ctx* c, double2*) { return {c->r32, c->p032, c->p132, c->t32, c->x32}; }
    static const float* phi(hmc_ctx* c, const double*) { return c->phi32; }
    static Coef<float> cf(hmc_ctx* c) { return c->cf32; }
};

static bool finished(int mode) { return mode == CG_DONE || mode == CG_STOPPED || mode == CG_FAILED; }

// Control block for the next CG launch; advances the state-record parity.
static CgCtl next_ctl(hmc_ctx* c, int expect, int ntiles) {
    CgCtl k;
    k.expect = expect;
    k.ntiles = ntiles;
    k.st_in = c->st + size_t(c->seq & 1) * c->cap;
    k.st_out = c->st + size_t((c->seq + 1) & 1) * c->cap;
    k.part = c->part;
    k.cap = c->cap;
    k.bpr = c->bpr;
    c->seq += 1;
    return k;
}

static const CgState* current_states(const hmc_ctx* c) { return c->st + size_t(c->seq & 1) * c->cap; }

// Enqueue the reliable-update / true-residual sequence for right-hand sides in `filter`,
// then reduce what is pending so the published records are complete.
template <typename R>
static int enqueue_ru(hmc_ctx* c, const double* phi64, const double2* b, double2* x, int n,
                      int filter, hipStream_t s) {
    CgVecs<R> v = KrylovBufs<R>::get(c, x);
    const int g = c->bpr * n;
    hipLaunchKernelGGL(k_ru_fold<R>, dim3(g), dim3(kBlock), 0, s, next_ctl(c, PEND_RR, c->nblk), x, v, c->lat, filter);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_ru_apply, dim3(g), dim3(kBlock), 0, s, next_ctl(c, PEND_NONE, c->nblk), x, c->t64, phi64,
                       c->lat, c->cf64, filter);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_ru_resid<R>, dim3(g), dim3(kBlock), 0, s, next_ctl(c, PEND_NONE, c->nblk), b, c->t64, phi64,
                       c->lat, c->cf64, v.r, filter);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_cg_finalize, dim3(n), dim3(kBlock), 0, s, next_ctl(c, PEND_RU, c->nblk));
    LAUNCHCHK();
    return HMC_OK;
}

template <typename R>
static int cg_run(hmc_ctx* c, const double* phi64, const double2* b, double2* x, int n,
                  hmc_cg_stats* stats, hipStream_t s) {
    const bool mixed = sizeof(R) == sizeof(float);
    CgVecs<R> v = KrylovBufs<R>::get(c, x);
    const R* phik = KrylovBufs<R>::phi(c, phi64);
    const Coef<R> cf = KrylovBufs<R>::cf(c);
    c->bpr = mixed ? c->bpr32 : c->bpr64;
    const int g = c->bpr * n;
    if (mixed) {
        hipLaunchKernelGGL(k_to_f32, dim3(elem_grid(3LL * c->vol)), dim3(kBlock), 0, s, phi64,
                           c->phi32, 3 * c->vol);
        LAUNCHCHK();
    }
    const double tol = c->p.cg_tol;
    c->seq = 0;
    hipLaunchKernelGGL(k_cg_init<R>, dim3(g), dim3(kBlock), 0, s, next_ctl(c, PEND_NONE, c->nblk), b, x, v, c->lat,
                       tol * tol, c->p.cg_maxit);
    LAUNCHCHK();

    const int chunk = mixed ? c->p.reliable_every : kCheckEvery;
    const int ru_filter = mixed ? (F_ACTIVE | F_CONV_ITER | F_MAXIT) : (F_CONV_ITER | F_MAXIT);
    const size_t st_bytes = sizeof(CgState) * size_t(n);
    int issued = 0;
    int k = 0;
    bool have_prev = false;
    const int kt_a = mixed ? 0 : 2;
    bool start_active_prev = true;   // were all right-hand sides iterating when chunk k-1 began
    // Chunks are issued one ahead of the status read, so the GPU never idles on the host;
    // once every right-hand side is finished the remaining launches return at once.
    for (;;) {
        for (int i = 0; i < chunk; ++i) {
            const bool sample = c->timing && i == chunk / 2;
            if (sample) HIPCHK(hipEventRecord(c->tev[k & 1][0], s));
            // the first step A of a solve reduces |b|^2; after a status chunk nothing is pending
            const int expect_a = i > 0 ? PEND_RR : (k == 0 ? PEND_BB : PEND_NONE);
            if constexpr (sizeof(R) == sizeof(float))
                hipLaunchKernelGGL(k_cg_a2, dim3(g), dim3(kBlock), 0, s, next_ctl(c, expect_a, c->nblk2), v,
                                   phik, c->lat, cf);
            else
                hipLaunchKernelGGL(k_cg_a<R>, dim3(g), dim3(kBlock), 0, s, next_ctl(c, expect_a, c->nblk), v,
                                   phik, c->lat, cf);
            LAUNCHCHK();
            if (sample) HIPCHK(hipEventRecord(c->tev[k & 1][1], s));
            if constexpr (sizeof(R) == sizeof(float))
                hipLaunchKernelGGL(k_cg_b2, dim3(g), dim3(kBlock), 0, s, next_ctl(c, PEND_TT, c->nblk2), v,
                                   phik, c->lat, cf);
            else
                hipLaunchKernelGGL(k_cg_b<R>, dim3(g), dim3(kBlock), 0, s, next_ctl(c, PEND_TT, c->nblk), v,
                                   phik, c->lat, cf);
            LAUNCHCHK();
            if (sample) HIPCHK(hipEventRecord(c->tev[k & 1][2], s));
        }
        issued += chunk;
        int rc = enqueue_ru<R>(c, phi64, b, x, n, ru_filter, s);
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(c->h_st + (k & 1) * c->cap, current_states(c), st_bytes,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(c->ev[k & 1], s));
        if (have_prev) {
            HIPCHK(hipEventSynchronize(c->ev[(k - 1) & 1]));
            const CgState* hs = c->h_st + ((k - 1) & 1) * c->cap;
            bool all = true, all_active = true;
            for (int j = 0; j < n; ++j) {
                all = all && finished(hs[j].mode);
                all_active = all_active && hs[j].mode == CG_ACTIVE;
            }
            // chunk k-1 began in the state chunk k-2 ended in; if every right-hand side was
            // iterating then and is still iterating at its end, its mid-chunk sample did full work
            if (c->timing && start_active_prev && all_active) {
                float ta = 0.f, tb = 0.f;
                HIPCHK(hipEventElapsedTime(&ta, c->tev[(k - 1) & 1][0], c->tev[(k - 1) & 1][1]));
                HIPCHK(hipEventElapsedTime(&tb, c->tev[(k - 1) & 1][1], c->tev[(k - 1) & 1][2]));
                c->kt.ms[kt_a] += ta;
                c->kt.ms[kt_a + 1] += tb;
                c->kt.count[kt_a] += 1;
                c->kt.count[kt_a + 1] += 1;
            }
            start_active_prev = all_active;
            if (all) break;
        }
        have_prev = true;
        ++k;
        // the device enforces cg_maxit; this bound only guards the host loop
        if (issued > c->p.cg_maxit + 4 * chunk) break;
    }
    HIPCHK(hipMemcpyAsync(c->h_st, current_states(c), st_bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int status = HMC_OK;
    for (int j = 0; j < n; ++j) {
        const CgState& h = c->h_st[j];
        if (h.mode == CG_FAILED) status = HMC_ERR_NONFINITE;
        else if (h.mode != CG_DONE && status == HMC_OK) status = HMC_ERR_NOT_CONVERGED;
    }
    if (stats != nullptr) {
        std::memset(stats, 0, sizeof(*stats));
        stats->n = n;
        stats->status = status;
        for (int j = 0; j < n; ++j) {
            const CgState& h = c->h_st[j];
            stats->iterations[j] = h.iters;
            stats->reliable_updates[j] = h.n_ru;
            stats->true_resid[j] = h.bb > 0.0 ? std::sqrt(h.rr_true / h.bb) : 0.0;
        }
    }
    if (status == HMC_ERR_NONFINITE) return fail(status, "CG met a non-finite value");
    if (status == HMC_ERR_NOT_CONVERGED)
        return fail(status, "CG did not reach tol %.3g within %d iterations", tol, c->p.cg_maxit);
    return HMC_OK;
}

static int cg_dispatch(hmc_ctx* c, const double* phi, const double2* b, double2* x, int n,
                       hmc_cg_stats* stats, hipStream_t s) {
    if (c->p.precision == HMC_MIXED) return cg_run<float>(c, phi, b, x, n, stats, s);
    return cg_run<double>(c, phi, b, x, n, stats, s);
}

static void merge_stats(hmc_traj_stats* t, const hmc_cg_stats& cs) {
    t->cg_solves += 1;
    for (int j = 0; j < cs.n; ++j) {
        t->cg_iterations += cs.iterations[j];
        if (cs.true_resid[j] > t->max_true_resid) t->max_true_resid = cs.true_resid[j];
    }
}

// Workspace layout: one walk that either only measures (base == nullptr) or also
// assigns the carved pointers.  Returns the bytes needed.
static size_t ws_layout(hmc_ctx* c, char* base) {
    const size_t V = size_t(c->vol);
    const size_t sp64 = 4 * V * sizeof(double2), sp32 = 4 * V * sizeof(float2);
    const size_t cap = size_t(c->cap);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + bytes, 256);
        return p;
    };
    char* st = take(sizeof(CgState) * 2 * cap);
    char* part = take(sizeof(double) * 4 * cap * size_t(kMaxBpr));
    char* gpart = take(sizeof(double) * 2 * size_t(c->nblk));
    char* slots = take(sizeof(double) * kSlots);
    char* v64 = take(4 * cap * sp64);
    char* v32 = take(5 * cap * sp32);
    char* tr = take(2 * cap * sp64);
    char* bos = take(2 * 3 * V * sizeof(double));
    char* f32 = take(3 * V * sizeof(float));
    if (base) {
        c->st = reinterpret_cast<CgState*>(st);
        c->part = reinterpret_cast<double*>(part);
        c->gpart = reinterpret_cast<double*>(gpart);
        c->slots = reinterpret_cast<double*>(slots);
        c->r64 = reinterpret_cast<double2*>(v64);
        c->p064 = reinterpret_cast<double2*>(v64 + cap * sp64);
        c->p164 = reinterpret_cast<double2*>(v64 + 2 * cap * sp64);
        c->t64 = reinterpret_cast<double2*>(v64 + 3 * cap * sp64);
        c->r32 = reinterpret_cast<float2*>(v32);
        c->p032 = reinterpret_cast<float2*>(v32 + cap * sp32);
        c->p132 = reinterpret_cast<float2*>(v32 + 2 * cap * sp32);
        c->t32 = reinterpret_cast<float2*>(v32 + 3 * cap * sp32);
        c->x32 = reinterpret_cast<float2*>(v32 + 4 * cap * sp32);
        c->chi = reinterpret_cast<double2*>(tr);
        c->xsol = reinterpret_cast<double2*>(tr + cap * sp64);
        c->pi = reinterpret_cast<double*>(bos);
        c->phi_save = reinterpret_cast<double*>(bos + 3 * V * sizeof(double));
        c->phi32 = reinterpret_cast<float*>(f32);
    }
    return off;
}

// CG launch shape: at most max_bpr workgroups per right-hand side; workgroup b takes
// tiles b, b + bpr, ... (so every consumer reduces at most kMaxBpr partials).
static int clamp_bpr(const hmc_ctx* c, int max_bpr) { return c->nblk2 < max_bpr ? c->nblk2 : max_bpr; }

static void set_cg_shape(hmc_ctx* c, int precision, int max_bpr) {
    if (precision != HMC_MIXED) c->bpr64 = clamp_bpr(c, max_bpr);
    if (precision != HMC_FP64) c->bpr32 = clamp_bpr(c, max_bpr);
}

// Process-wide memory of autotuned shapes, keyed by lattice, right-hand sides and device.
struct TuneKey {
    int L, Lt, n, dev;
    bool operator<(const TuneKey& o) const {
        return std::tie(L, Lt, n, dev) < std::tie(o.L, o.Lt, o.n, o.dev);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, std::pair<int, int>> g_tuned;   // -> (bpr64, bpr32)

// --------------------------------------------------------------------------------------
// C ABI

extern "C" {

const char* hmc_strerror(int code) {
    switch (code) {
        case HMC_OK: return "ok";
        case HMC_ERR_INVALID_ARG: return "invalid argument";
        case HMC_ERR_NOT_CONVERGED: return "conjugate gradient did not converge";
        case HMC_ERR_NONFINITE: return "non-finite value";
        case HMC_ERR_HIP: return "HIP runtime error";
        case HMC_ERR_WORKSPACE: return "workspace missing or too small";
        default: return "unknown error";
    }
}

const char* hmc_last_error(void) { return g_last_error.c_str(); }

int hmc_test_site(int L, int Lt, int s, int out[12]) {
    if (!geometry_ok(L, Lt) || out == nullptr) return -1;
    const Lat lat = make_lat(L, Lt);
    if (s < 0 || s >= lat.vol) return -1;
    const Nbr n = neighbours(lat, s);
    const int v[12] = {n.tau, n.x, n.y, n.xp, n.xm, n.yp, n.ym, n.tp, n.tm, n.sfwd, n.sbwd, n.stag};
    std::memcpy(out, v, sizeof(v));
    return 0;
}

int hmc_test_xcd_remap(int bid, int nb) {
    if (nb <= 0 || bid < 0 || bid >= nb) return -1;
    return xcd_remap(bid, nb);
}

int hmc_create(int L, int Lt, double dtau, const hmc_params* params, hmc_ctx** out) {
    g_last_error.clear();
    if (out == nullptr) return fail(HMC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!geometry_ok(L, Lt))
        return fail(HMC_ERR_INVALID_ARG,
                    "bad lattice L=%d L_tau=%d (need even 4 <= L <= %d, L_tau >= 2, volume < 2^%d)",
                    L, Lt, kMaxL, kMaxVolLog2);
    if (!(dtau > 0.0) || !std::isfinite(dtau)) return fail(HMC_ERR_INVALID_ARG, "dtau must be > 0");
    int rc = check_params(params);
    if (rc) return rc;
    hmc_ctx* c = new hmc_ctx();
    c->L = L;
    c->Lt = Lt;
    c->vol = Lt * L * L;
    c->dtau = dtau;
    c->p = *params;
    c->cap = params->max_rhs > 0 ? params->max_rhs : (params->n_pf > 0 ? params->n_pf : 1);
    c->lat = make_lat(L, Lt);
    c->nblk = (c->vol + kBlock - 1) / kBlock;
    c->nblk2 = (c->vol / 2 + kBlock - 1) / kBlock;
    set_coefs(c);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(HMC_ERR_HIP, "hipGetDevice failed");
    }
    set_cg_shape(c, HMC_FP64, kDefaultBpr64);
    set_cg_shape(c, HMC_MIXED, kDefaultBpr32);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(TuneKey{L, Lt, c->cap, c->device});
        if (it != g_tuned.end()) {
            c->bpr64 = it->second.first;
            c->bpr32 = it->second.second;
        }
    }
    c->need = ws_layout(c, nullptr);
    if (hipHostMalloc((void**)&c->h_st, sizeof(CgState) * 2 * size_t(c->cap), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_slots, sizeof(double) * kSlots, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) != hipSuccess) {
        hmc_destroy(c);
        return fail(HMC_ERR_HIP, "pinned status buffer or event creation failed");
    }
    *out = c;
    return HMC_OK;
}

int hmc_set_kernel_timing(hmc_ctx* c, int enable) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    if (enable && c->tev[0][0] == nullptr) {
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) HIPCHK(hipEventCreate(&c->tev[i][j]));
    }
    c->timing = enable != 0;
    std::memset(&c->kt, 0, sizeof(c->kt));
    return HMC_OK;
}

int hmc_set_cg_workgroups(hmc_ctx* c, int precision, int max_per_rhs) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    if (precision != HMC_FP64 && precision != HMC_MIXED && precision != -1)
        return fail(HMC_ERR_INVALID_ARG, "precision must be HMC_FP64, HMC_MIXED or -1");
    if (max_per_rhs < 1 || max_per_rhs > kMaxBpr)
        return fail(HMC_ERR_INVALID_ARG, "workgroups per right-hand side must lie in [1, %d]", kMaxBpr);
    set_cg_shape(c, precision, max_per_rhs);
    return HMC_OK;
}

int hmc_get_cg_workgroups(const hmc_ctx* c, int precision) {
    if (c == nullptr) return -1;
    return precision == HMC_MIXED ? c->bpr32 : c->bpr64;
}

static int check_solve_args(hmc_ctx* c, const void* phi, const void* b, const void* x, int n);

int hmc_autotune(hmc_ctx* c, const double* phi, const void* b, int n, hmc_tune_result* out,
                 void* stream) {
    int rc = check_solve_args(c, phi, b, c ? c->xsol : nullptr, n);
    if (rc) return rc;
    if (out == nullptr) return fail(HMC_ERR_INVALID_ARG, "out is NULL");
    hipStream_t s = (hipStream_t)stream;
    static const int cand[] = {128, 256, 384, 512, 768, 1024, 1536, 2048, 4096};
    const hmc_params saved = c->p;
    const int iters = 100;
    std::memset(out, 0, sizeof(*out));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int result = HMC_OK;
    for (int pi = 0; pi < 2 && result == HMC_OK; ++pi) {
        const int prec = pi == 0 ? HMC_FP64 : HMC_MIXED;
        c->p.precision = prec;
        c->p.cg_tol = 1e-30;           // never converges: every candidate runs `iters` iterations
        c->p.cg_maxit = iters;
        if (prec == HMC_MIXED && c->p.reliable_every < 1) c->p.reliable_every = 50;
        double best = 1e300;
        int best_bpr = 0, last = -1;
        for (int cb : cand) {
            const int bpr = clamp_bpr(c, cb);
            if (bpr == last) continue;
            last = bpr;
            set_cg_shape(c, prec, bpr);
            float ms = 0.f;
            for (int rep = 0; rep < 2; ++rep) {    // first run warms caches and code
                if (hipEventRecord(e0, s) != hipSuccess) { result = HMC_ERR_HIP; break; }
                const int r = cg_dispatch(c, phi, static_cast<const double2*>(b), c->xsol, n, nullptr, s);
                if (r != HMC_OK && r != HMC_ERR_NOT_CONVERGED) { result = r; break; }
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { result = HMC_ERR_HIP; break; }
            }
            if (result != HMC_OK) break;
            out->candidates += 1;
            const double us = 1e3 * ms / iters;
            if (us < best) { best = us; best_bpr = bpr; }
        }
        if (result == HMC_OK) {
            set_cg_shape(c, prec, best_bpr);
            out->cg_workgroups[pi] = best_bpr;
            out->us_per_iter[pi] = best;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->p = saved;
    if (result != HMC_OK) {
        set_cg_shape(c, HMC_FP64, kDefaultBpr64);
        set_cg_shape(c, HMC_MIXED, kDefaultBpr32);
        return result == HMC_ERR_HIP ? fail(result, "autotune: HIP call failed") : result;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[TuneKey{c->L, c->Lt, c->cap, c->device}] = {c->bpr64, c->bpr32};
    return HMC_OK;
}

int hmc_get_kernel_times(const hmc_ctx* c, hmc_kernel_times* out) {
    if (c == nullptr || out == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    *out = c->kt;
    return HMC_OK;
}

int hmc_destroy(hmc_ctx* c) {
    if (c == nullptr) return HMC_OK;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            if (c->tev[i][j]) (void)hipEventDestroy(c->tev[i][j]);
    if (c->h_st) (void)hipHostFree(c->h_st);
    if (c->h_slots) (void)hipHostFree(c->h_slots);
    for (int i = 0; i < 2; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    delete c;
    return HMC_OK;
}

int hmc_set_params(hmc_ctx* c, const hmc_params* params) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    int rc = check_params(params);
    if (rc) return rc;
    const int want = params->max_rhs > 0 ? params->max_rhs : params->n_pf;
    if (want > c->cap) return fail(HMC_ERR_INVALID_ARG, "n_pf/max_rhs %d exceeds workspace capacity %d", want, c->cap);
    c->p = *params;
    set_coefs(c);
    return HMC_OK;
}

size_t hmc_workspace_bytes(const hmc_ctx* c) { return c ? c->need : 0; }

int hmc_set_workspace(hmc_ctx* c, void* ptr, size_t bytes) {
    if (c == nullptr || ptr == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL ctx or workspace");
    if ((reinterpret_cast<uintptr_t>(ptr) & 255u) != 0) return fail(HMC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (bytes < c->need) return fail(HMC_ERR_WORKSPACE, "workspace of %zu bytes < %zu needed", bytes, c->need);
    char* base = static_cast<char*>(ptr);
    (void)ws_layout(c, base);
    c->ws = base;
    c->ws_bytes = bytes;
    return HMC_OK;
}

}  // extern "C"

// ---- operator applies -----------------------------------------------------------------

template <typename R, bool DAG>
static int apply_impl(hmc_ctx* c, const R* phi, const void* in, void* out, int n, void* stream) {
    if (c == nullptr || phi == nullptr || in == nullptr || out == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if (n < 1) return fail(HMC_ERR_INVALID_ARG, "n must be >= 1");
    if (!aligned16(phi) || !aligned16(in) || !aligned16(out)) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    if (in == out) return fail(HMC_ERR_INVALID_ARG, "in and out must not overlap");
    if ((long long)c->nblk * n >= (1LL << 31)) return fail(HMC_ERR_INVALID_ARG, "too many vectors");
    if constexpr (sizeof(R) == sizeof(double)) {
        hipLaunchKernelGGL((k_apply<double, DAG>), dim3(grid_for(c, n)), dim3(kBlock), 0,
                           (hipStream_t)stream, static_cast<const double2*>(in),
                           static_cast<double2*>(out), phi, c->lat, c->cf64, c->nblk);
    } else {
        hipLaunchKernelGGL(k_apply2<DAG>, dim3(c->nblk2 * n), dim3(kBlock), 0, (hipStream_t)stream,
                           static_cast<const float2*>(in), static_cast<float2*>(out), phi, c->lat,
                           c->cf32, c->nblk2);
    }
    LAUNCHCHK();
    return HMC_OK;
}

template <typename R>
static int apply_normal_impl(hmc_ctx* c, const R* phi, const void* in, void* out, int n, void* stream) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    int rc = need_ws(c);
    if (rc) return rc;
    if (n < 1 || n > c->cap) return fail(HMC_ERR_INVALID_ARG, "n must lie in [1, %d]", c->cap);
    void* tmp;
    if constexpr (sizeof(R) == sizeof(double)) tmp = c->t64; else tmp = c->t32;
    if (tmp == in || tmp == out) return fail(HMC_ERR_INVALID_ARG, "in/out alias the workspace");
    rc = apply_impl<R, false>(c, phi, in, tmp, n, stream);
    if (rc) return rc;
    return apply_impl<R, true>(c, phi, tmp, out, n, stream);
}

extern "C" {

int hmc_apply_M(hmc_ctx* c, const double* phi, const void* in, void* out, int n, void* stream) {
    return apply_impl<double, false>(c, phi, in, out, n, stream);
}
int hmc_apply_Mdag(hmc_ctx* c, const double* phi, const void* in, void* out, int n, void* stream) {
    return apply_impl<double, true>(c, phi, in, out, n, stream);
}
int hmc_apply_MdagM(hmc_ctx* c, const double* phi, const void* in, void* out, int n, void* stream) {
    return apply_normal_impl<double>(c, phi, in, out, n, stream);
}
int hmc_apply_M_f32(hmc_ctx* c, const float* phi, const void* in, void* out, int n, void* stream) {
    return apply_impl<float, false>(c, phi, in, out, n, stream);
}
int hmc_apply_Mdag_f32(hmc_ctx* c, const float* phi, const void* in, void* out, int n, void* stream) {
    return apply_impl<float, true>(c, phi, in, out, n, stream);
}
int hmc_apply_MdagM_f32(hmc_ctx* c, const float* phi, const void* in, void* out, int n, void* stream) {
    return apply_normal_impl<float>(c, phi, in, out, n, stream);
}

int hmc_heatbath(hmc_ctx* c, const double* phi, const void* eta, void* chi, int n_pf, void* stream) {
    return apply_impl<double, true>(c, phi, eta, chi, n_pf, stream);
}

// ---- solver, actions, gradient --------------------------------------------------------

static int check_solve_args(hmc_ctx* c, const void* phi, const void* b, const void* x, int n) {
    if (c == nullptr || phi == nullptr || b == nullptr || x == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    int rc = need_ws(c);
    if (rc) return rc;
    if (n < 1 || n > c->cap) return fail(HMC_ERR_INVALID_ARG, "n = %d outside [1, %d]", n, c->cap);
    if (!aligned16(phi) || !aligned16(b) || !aligned16(x)) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    if (b == x) return fail(HMC_ERR_INVALID_ARG, "b and x must not alias");
    return HMC_OK;
}

int hmc_cg_solve(hmc_ctx* c, const double* phi, const void* b, void* x, int n,
                 hmc_cg_stats* stats, void* stream) {
    int rc = check_solve_args(c, phi, b, x, n);
    if (rc) return rc;
    return cg_dispatch(c, phi, static_cast<const double2*>(b), static_cast<double2*>(x), n, stats,
                       (hipStream_t)stream);
}

static int launch_force(hmc_ctx* c, const double* phi, const double2* x, int npf, int flags,
                        double* force, double* pi, double h, int nkick, hipStream_t s) {
    hipLaunchKernelGGL(k_force, dim3(c->nblk), dim3(kBlock), 0, s, x, npf, phi, c->lat, c->cf64,
                       c->bc, (flags & HMC_FORCE_PF) ? 1 : 0, (flags & HMC_FORCE_BOSON) ? 1 : 0,
                       force, pi, h, nkick);
    LAUNCHCHK();
    return HMC_OK;
}

static int dot_re(hmc_ctx* c, const double2* a, const double2* b, int n, double* slot, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_re, dim3(c->nblk), dim3(kBlock), 0, s, a, b, n, c->lat, c->gpart);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, c->gpart, c->nblk, 1, 0, slot);
    LAUNCHCHK();
    return HMC_OK;
}

// K = |pi|^2 / 2 (pi may be NULL) and S_B into slot[0], slot[1].
static int energy(hmc_ctx* c, const double* pi, const double* phi, double* slot, hipStream_t s) {
    hipLaunchKernelGGL(k_energy, dim3(c->nblk), dim3(kBlock), 0, s, pi, phi, c->lat, c->bc,
                       c->gpart, c->nblk);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, c->gpart, c->nblk, 2, c->nblk, slot);
    LAUNCHCHK();
    return HMC_OK;
}

static int read_slots(hmc_ctx* c, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(c->h_slots, c->slots, sizeof(double) * kSlots, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HMC_OK;
}

int hmc_force_from_solution(hmc_ctx* c, const double* phi, const void* x, int n_pf,
                            double* force, int flags, void* stream) {
    if (c == nullptr || phi == nullptr || force == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if ((flags & HMC_FORCE_PF) && (x == nullptr || n_pf < 1)) return fail(HMC_ERR_INVALID_ARG, "pseudofermion force needs x and n_pf >= 1");
    if (n_pf < 0 || n_pf > HMC_MAX_RHS) return fail(HMC_ERR_INVALID_ARG, "n_pf out of range");
    if (!aligned16(phi) || !aligned16(force) || (x && !aligned16(x))) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    return launch_force(c, phi, static_cast<const double2*>(x), n_pf, flags, force, nullptr, 0.0, 0,
                        (hipStream_t)stream);
}

int hmc_pf_action(hmc_ctx* c, const double* phi, const void* chi, int n_pf, void* x, double* S,
                  hmc_cg_stats* stats, void* stream) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    double2* xs = x ? static_cast<double2*>(x) : c->xsol;
    int rc = check_solve_args(c, phi, chi, xs, n_pf);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = cg_dispatch(c, phi, static_cast<const double2*>(chi), xs, n_pf, stats, s);
    if (rc && rc != HMC_ERR_NOT_CONVERGED) return rc;
    int rc2 = dot_re(c, static_cast<const double2*>(chi), xs, n_pf, c->slots + SL_TMP, s);
    if (rc2) return rc2;
    rc2 = read_slots(c, s);
    if (rc2) return rc2;
    if (S) *S = c->h_slots[SL_TMP];
    return rc;
}

int hmc_force(hmc_ctx* c, const double* phi, const void* chi, int n_pf, double* force,
              double* S_pf, int flags, hmc_cg_stats* stats, void* stream) {
    if (c == nullptr || force == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int rc = HMC_OK;
    if (flags & HMC_FORCE_PF) {
        rc = check_solve_args(c, phi, chi, c->xsol, n_pf);
        if (rc) return rc;
        rc = cg_dispatch(c, phi, static_cast<const double2*>(chi), c->xsol, n_pf, stats, s);
        if (rc && rc != HMC_ERR_NOT_CONVERGED) return rc;
    } else if (phi == nullptr) {
        return fail(HMC_ERR_INVALID_ARG, "phi is NULL");
    }
    int rc2 = launch_force(c, phi, c->xsol, (flags & HMC_FORCE_PF) ? n_pf : 0, flags, force,
                           nullptr, 0.0, 0, s);
    if (rc2) return rc2;
    if ((flags & HMC_FORCE_PF) && S_pf) {
        rc2 = dot_re(c, static_cast<const double2*>(chi), c->xsol, n_pf, c->slots + SL_TMP, s);
        if (rc2) return rc2;
        rc2 = read_slots(c, s);
        if (rc2) return rc2;
        *S_pf = c->h_slots[SL_TMP];
    } else if (S_pf) {
        *S_pf = 0.0;
    }
    return rc;
}

int hmc_boson_action(hmc_ctx* c, const double* phi, double* S, void* stream) {
    if (c == nullptr || phi == nullptr || S == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    int rc = need_ws(c);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = energy(c, nullptr, phi, c->slots + SL_TMP, s);
    if (rc) return rc;
    rc = read_slots(c, s);
    if (rc) return rc;
    *S = c->h_slots[SL_TMP + 1];
    return HMC_OK;
}

// ---- trajectory ----------------------------------------------------------------------

// Leapfrog (kick-drift-kick) on (phi, pi) with pseudofermions chi fixed: n_leap steps of eps,
// one CG solve per step plus the one at the start, the two half kicks of neighbouring steps
// applied separately inside the gradient kernel.  Leaves sum_k Re<chi_k, x_k> of the last
// solve in slot SL_SPF1 and, if first_action, that of the first solve in SL_SPF0.
static int md_integrate(hmc_ctx* c, double* phi, double* pi, const double2* chi, int n_pf,
                        bool first_action, hmc_traj_stats* stats, hipStream_t s) {
    const double eps = c->p.eps, h = 0.5 * eps;
    const int nl = c->p.n_leap;
    const int flags = HMC_FORCE_BOSON | (n_pf > 0 ? HMC_FORCE_PF : 0);
    auto solve = [&]() -> int {
        if (n_pf == 0) return HMC_OK;
        hmc_cg_stats cs;
        int r = cg_dispatch(c, phi, chi, c->xsol, n_pf, &cs, s);
        if (r == HMC_OK || r == HMC_ERR_NOT_CONVERGED || r == HMC_ERR_NONFINITE) merge_stats(stats, cs);
        return r;
    };
    int rc = solve();
    if (rc) return rc;
    if (first_action && n_pf > 0) {
        rc = dot_re(c, chi, c->xsol, n_pf, c->slots + SL_SPF0, s);
        if (rc) return rc;
    }
    // first half kick with the force at the start
    rc = launch_force(c, phi, c->xsol, n_pf, flags, nullptr, pi, h, nl > 0 ? 1 : 0, s);
    if (rc) return rc;
    for (int step = 0; step < nl; ++step) {
        hipLaunchKernelGGL(k_drift, dim3(elem_grid(3LL * c->vol)), dim3(kBlock), 0, s, phi, pi, eps,
                           3 * c->vol);
        LAUNCHCHK();
        rc = solve();
        if (rc) return rc;
        // closing half kick of this step, then the opening half kick of the next one
        rc = launch_force(c, phi, c->xsol, n_pf, flags, nullptr, pi, h, step + 1 < nl ? 2 : 1, s);
        if (rc) return rc;
    }
    if (n_pf > 0) {
        rc = dot_re(c, chi, c->xsol, n_pf, c->slots + SL_SPF1, s);
        if (rc) return rc;
    }
    return HMC_OK;
}

static void fill_energies(hmc_ctx* c, int n_pf, hmc_traj_stats* stats) {
    const double* hs = c->h_slots;
    stats->K0 = hs[SL_K0];
    stats->S_b0 = hs[SL_SB0];
    stats->S_pf0 = n_pf > 0 ? hs[SL_SPF0] : 0.0;
    stats->K1 = hs[SL_K1];
    stats->S_b1 = hs[SL_SB1];
    stats->S_pf1 = n_pf > 0 ? hs[SL_SPF1] : 0.0;
    stats->H0 = stats->K0 + stats->S_b0 + stats->S_pf0;
    stats->H1 = stats->K1 + stats->S_b1 + stats->S_pf1;
    stats->dH = stats->H1 - stats->H0;
}

int hmc_trajectory(hmc_ctx* c, double* phi, const double* pi0, const void* eta, int n_pf,
                   double u, hmc_traj_stats* stats, void* stream) {
    if (c == nullptr || phi == nullptr || pi0 == nullptr || stats == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    int rc = need_ws(c);
    if (rc) return rc;
    if (n_pf < 0 || n_pf > c->cap) return fail(HMC_ERR_INVALID_ARG, "n_pf %d outside [0, %d]", n_pf, c->cap);
    if (n_pf > 0 && eta == nullptr) return fail(HMC_ERR_INVALID_ARG, "eta is NULL");
    if (!aligned16(phi) || !aligned16(pi0) || (eta && !aligned16(eta))) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    std::memset(stats, 0, sizeof(*stats));
    const size_t phib = 3 * size_t(c->vol) * sizeof(double);

    // start: keep phi0, copy pi0, heat-bath chi = M^dagger eta, energies at phi0
    HIPCHK(hipMemcpyAsync(c->phi_save, phi, phib, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(c->pi, pi0, phib, hipMemcpyDeviceToDevice, s));
    if (n_pf > 0) {
        rc = apply_impl<double, true>(c, phi, eta, c->chi, n_pf, s);
        if (rc) return rc;
        rc = dot_re(c, static_cast<const double2*>(eta), static_cast<const double2*>(eta), n_pf,
                    c->slots + SL_SPF0, s);
        if (rc) return rc;
    }
    rc = energy(c, c->pi, phi, c->slots + SL_K0, s);
    if (rc) return rc;

    auto restore = [&](int code) -> int {
        (void)hipMemcpyAsync(phi, c->phi_save, phib, hipMemcpyDeviceToDevice, s);
        (void)hipStreamSynchronize(s);
        stats->accepted = 0;
        stats->status = code;
        return code;
    };
    rc = md_integrate(c, phi, c->pi, c->chi, n_pf, false, stats, s);
    if (rc) return restore(rc);
    rc = energy(c, c->pi, phi, c->slots + SL_K1, s);
    if (rc) return restore(rc);
    rc = read_slots(c, s);
    if (rc) return restore(rc);
    fill_energies(c, n_pf, stats);
    if (!std::isfinite(stats->dH)) return restore(fail(HMC_ERR_NONFINITE, "dH is not finite"));
    stats->accepted = (u < std::exp(-stats->dH)) ? 1 : 0;
    stats->status = HMC_OK;
    if (!stats->accepted) {
        HIPCHK(hipMemcpyAsync(phi, c->phi_save, phib, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    return HMC_OK;
}

int hmc_leapfrog(hmc_ctx* c, double* phi, double* pi, const void* chi, int n_pf,
                 hmc_traj_stats* stats, void* stream) {
    if (c == nullptr || phi == nullptr || pi == nullptr || stats == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    int rc = need_ws(c);
    if (rc) return rc;
    if (n_pf < 0 || n_pf > c->cap) return fail(HMC_ERR_INVALID_ARG, "n_pf %d outside [0, %d]", n_pf, c->cap);
    if (n_pf > 0 && chi == nullptr) return fail(HMC_ERR_INVALID_ARG, "chi is NULL");
    if (!aligned16(phi) || !aligned16(pi) || (chi && !aligned16(chi))) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    std::memset(stats, 0, sizeof(*stats));
    rc = energy(c, pi, phi, c->slots + SL_K0, s);
    if (rc) return rc;
    rc = md_integrate(c, phi, pi, static_cast<const double2*>(chi), n_pf, true, stats, s);
    if (rc) { stats->status = rc; return rc; }
    rc = energy(c, pi, phi, c->slots + SL_K1, s);
    if (rc) return rc;
    rc = read_slots(c, s);
    if (rc) return rc;
    fill_energies(c, n_pf, stats);
    stats->accepted = 1;
    stats->status = HMC_OK;
    return HMC_OK;
}

}  // extern "C"
