// hmc.hip -- host side of libhmc: context and workspace management, the C ABI of
// include/hmc.h, the conjugate-gradient engine (FP64 and mixed precision with FP64 reliable
// updates, eager or replayed from HIP graphs) and the HMC trajectory drivers for one lattice
// and for a ragged batch of independent lattices.
//
// Every step of the path runs in the kernels of kernels.h; the host only sequences
// launches on the caller's stream and reads back per-solve status records (CG
// convergence) and the energies of a trajectory.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include <sys/stat.h>
#include <unistd.h>

#include "../../include/hmc.h"
#include "../../include/hmc_testing.h"
#include "fft.h"
#include "kernels.h"
#include "precond.h"
#include "metric.h"
#include "lattice.h"
#include "probe.h"
#include "march.h"

// Hash of the sources the library was built from (set by the build; keys the tuning cache).
#ifndef HMC_SOURCE_HASH
#define HMC_SOURCE_HASH "unknown"
#endif

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
constexpr int kChainSlots = 8;      // per-lattice scalars in batch mode
constexpr int kDefaultBpr64 = 1024; // default CG workgroups per right-hand side, FP64
constexpr int kDefaultBpr32 = 512;  // ... mixed precision (FP32 pair kernels)
constexpr int kMaxBpr = 4096;       // largest accepted (sizes the partial-sum buffer)
// Mixed precision: an FP64 reliable update is due once the FP32 iterated |r| has fallen by
// 1e-4 since the last true residual.  Beyond that the FP32 recurrence no longer tracks the
// true residual, and the direction kept across the update would be stale.
constexpr double kRuDrop2 = 1e-8;

// Slot indices in the device scalar area (and in each lattice's block in batch mode).
enum Slot : int {
    SL_K0 = 0, SL_SB0 = 1, SL_K1 = 2, SL_SB1 = 3, SL_SPF0 = 4, SL_SPF1 = 5, SL_TMP = 6,
    SL_TMP2 = 7,
};

int tiles1_host(int vol) { return (vol + kBlock - 1) / kBlock; }
int tiles2_host(int vol) { return (vol / 2 + kBlock - 1) / kBlock; }

}  // namespace

// Device scratch for the entry point that must not allocate (hmc_apply_MdagM_noalloc): the
// intermediate M in of its two passes.  Each GPU holds its own copy for the life of the
// process.  In host code the name stands for a host-side symbol, not a device address: the
// address comes from hipGetSymbolAddress, taken once per device when a context is created on
// it (scratch_for_device) and kept in the context.
constexpr size_t kStaticScratchBytes = size_t(HMC_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_addr;   // device -> device address of `scratch`

// Batch-mode description: nchains independent lattices, nrhs right-hand sides each.
struct BatchInfo {
    int nchains = 0, nrhs = 0;
    std::vector<Lat> lats;
    std::vector<double> r;
    std::vector<long long> phi_off;   // nchains + 1 prefix offsets (elements) of the boson fields
    std::vector<long long> sp_off;    // nchains + 1 prefix offsets (complex) of the spinor blocks
    std::vector<int> cfirst;          // nchains + 1 prefix of 256-site tiles (site kernels)
    std::vector<long long> pcoff;     // nchains + 1 prefix offsets (doubles) of preconditioner tables
    int nslices = 0;                  // sum over units of 4 L_tau (preconditioner slice workgroups)
    int ngroups[2] = {0, 0};          // sum over units of the tau-pass workgroups [FP64, FP32]
    // device tables in the workspace; index 0: FP64 launch shape, 1: mixed precision
    UnitDesc* units[2] = {nullptr, nullptr};
    int2* blocks[2] = {nullptr, nullptr};
    int nblocks[2] = {0, 0};
    // step A and the reliable update's FP64 stencils as marches (0 workgroups: the tile
    // kernels): block tables (unit, workgroup), workgroups, threads and LDS of a launch
    int2* mblocks[2] = {nullptr, nullptr};
    int2* rblocks[2] = {nullptr, nullptr};
    int mgrid[2] = {0, 0}, rgrid[2] = {0, 0};
    int mthreads[2] = {0, 0}, rthreads[2] = {0, 0};
    size_t mlds[2] = {0, 0}, rlds[2] = {0, 0};
    std::vector<UnitDesc> hunits[2];  // host copies of the unit tables
    int2* pxy_blocks = nullptr;       // preconditioner slice passes: (unit, slice)
    int2* pt_blocks[2] = {nullptr, nullptr};   // tau pass: (unit, column group) [FP64, FP32]
    ChainDesc* chains = nullptr;
    int2* cblocks = nullptr;
    int* cfirst_dev = nullptr;
    double* cslots = nullptr;         // nchains * kChainSlots
    double* h_cslots = nullptr;       // pinned copy
};

// Graph-replay cache of the two status chunks of a solve (see cg_run).
struct CgGraphs {
    hipGraphExec_t exec[2] = {nullptr, nullptr};   // [0] first chunk, [1] later chunks
    std::tuple<int, const void*, const void*, const void*, const void*, int, int, int, int, long, int>
        key{};
};

struct hmc_ctx {
    int device = 0;
    int L = 0, Lt = 0, vol = 0;
    double dtau = 0.0;
    hmc_params p{};
    int cap = 1;            // right-hand sides the workspace holds (one lattice)
    int nblk = 0;           // 256-site tiles per right-hand side (one site per thread)
    int nblk2 = 0;          // 512-site tiles per right-hand side (FP32 pair kernels)
    int bpr64 = 0;          // CG workgroups per right-hand side, FP64 solves
    int bpr32 = 0;          // ... mixed-precision solves
    int seq = 0;            // CG launch counter (selects the state record buffer)
    long generation = 0;    // bumped when coefficients, workspace or launch shapes change
    Lat lat{};
    Coef<double> cf64{};
    Coef<float> cf32{};
    BosonCoef bc{};

    // sizes of the workspace carve
    long long vec_sites = 0;   // sites of one full set of right-hand sides
    long long phi_sites = 0;   // sites of the boson field(s)
    int nunits = 1;            // CG state records
    int pslots = 0;            // CG partial-sum slots per kind (sum over units of the largest
                               // workgroup count any kernel runs on the unit)
    int pstride = 0;           // one lattice: partial slots per unit
    bool pc_ok[2] = {false, false};   // the Fourier preconditioner supports these lattices on
                                      // this GPU [FP64, FP32]
    size_t lds_xy[2] = {0, 0}; // dynamic LDS of the preconditioner passes [FP64, FP32]
    size_t lds_t[2] = {0, 0};
    int pc_q[2] = {0, 0};      // chunks per column of the tau pass [FP64, FP32]
    bool pc_full[2] = {false, false};   // every lattice's columns are pc_q full chunks
    long long blob_doubles = 0;    // preconditioner tables of all lattices
    bool pc_r7 = false;            // some lattice extent needs radix-7 FFT stages
    // Fourier-diagonal HMC metric (one lattice): the caller's sigma table (null: identity,
    // plain drift and kinetic energy), whether this lattice supports the metric passes, their
    // tau-pass LDS and per-workgroup partial sums
    const double* sigma = nullptr;
    bool metric_ok = false;
    size_t lds_mt_t = 0;
    double* mpart = nullptr;           // 3 x max(tau-pass groups, 256) partial sums
    double* piw = nullptr;             // momenta of a warm-up iteration (one lattice)
    int ngblk = 0;             // 256-site tiles of the site-parallel kernels

    bool is_batch = false;
    BatchInfo bi;

    // workspace (caller-owned)
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t need = 0;
    // carved pointers
    CgState* st = nullptr;       // 2 * nunits records (double-buffered by launch parity)
    double* part = nullptr;      // CG partial sums: kPendKinds * pslots
    double* gpart = nullptr;     // site-kernel partial sums: 2 * ngblk
    double* slots = nullptr;
    double2 *r64 = nullptr, *p064 = nullptr, *p164 = nullptr, *t64 = nullptr, *z64 = nullptr;
    float2 *r32 = nullptr, *p032 = nullptr, *p132 = nullptr, *t32 = nullptr, *x32 = nullptr, *z32 = nullptr;
    double* blob = nullptr;      // preconditioner tables
    double2 *chi = nullptr, *xsol = nullptr;
    double *pi = nullptr, *phi_save = nullptr;
    float* phi32 = nullptr;

    // pinned host status area
    CgState* h_st = nullptr;     // 2 * nunits records (double buffer)
    double* h_slots = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};

    // sampled kernel timing: start/stop events of steps A and B and of the three
    // preconditioner passes, taken by the dispatch of the kernel itself (no marker packets
    // between kernels), one set per status slot
    bool timing = false;
    static constexpr int kEv = 12;
    hipEvent_t tev[2][kEv] = {};
    hmc_kernel_times kt{};

    // fused M^dagger M (march.h): rows per band and slices per segment [FP64, FP32]; 0 = the
    // default for the lattice
    int mdm_rows[2] = {0, 0};
    int mdm_seg[2] = {0, 0};
    // CG step A as a march (march.h) [FP64, FP32]: rows per band (0: the tile kernels) and slices
    // per segment (0: the default)
    int cgm_rows[2] = {0, 0};
    int cgm_seg[2] = {0, 0};
    int cgb_march[2] = {1, 1};   // step B marches too (with step A's cut) [FP64, FP32]
    // partial sums the last launched kernel left per unit when its workgroup count is not the
    // CG launch shape's (a march); the next launch's control block takes it over
    int next_nparts = 0;

    // device address of the static scratch on this context's GPU (null if it could not be
    // resolved; only hmc_apply_MdagM_noalloc uses it)
    void* scratch = nullptr;

    // one graph per leapfrog step: the drift, the solve's start and a fixed number of status
    // chunks (sized from the previous solve), cached by shape
    bool step_graphs = false;
    int sg_last_iters = 0;     // most iterations of a unit in the last solve
    struct StepGraph {
        std::tuple<int, int, const void*, const void*, const void*, const void*, int, long, int, int, double, int> key;
        hipGraphExec_t exec = nullptr;
        int seq_after = 0;
    };
    std::vector<StepGraph> sgs;

    // graph replay of CG chunks
    bool graphs = false;
    hipStream_t cap_stream = nullptr;
    CgGraphs cgg[2];             // [0] FP64, [1] mixed
};

// The batch handle is the same engine configured for ragged lattices.
struct hmc_batch {
    hmc_ctx c;
};

static std::string device_tag(int dev);

// Cache key of a context: one lattice "one L Lt n", a batch "batch <hash of the chain list>",
// " nn2" with the two-site hops, then the device and the kernel-source hash.
static std::string tune_key(const hmc_ctx* c) {
    std::string k;
    if (c->is_batch) {
        uint64_t h = 1469598103934665603ULL;   // FNV-1a over the chain geometry
        auto mix = [&](long long v) {
            for (int i = 0; i < 8; ++i) {
                h ^= uint64_t((v >> (8 * i)) & 0xff);
                h *= 1099511628211ULL;
            }
        };
        mix(c->bi.nchains);
        mix(c->bi.nrhs);
        for (const Lat& l : c->bi.lats) {
            mix(l.L);
            mix(l.Lt);
        }
        char buf[64];
        std::snprintf(buf, sizeof(buf), "batch %016llx", (unsigned long long)h);
        k = buf;
    } else {
        k = "one " + std::to_string(c->L) + " " + std::to_string(c->Lt) + " " + std::to_string(c->cap);
    }
    if (c->cf64.nn2) k += " nn2";   // the two-site hops run other instantiations
    return k + " " + device_tag(c->device) + " " + HMC_SOURCE_HASH;
}

// --------------------------------------------------------------------------------------
// helpers

static BosonCoef boson_coef_of(double dt, double cv, double r, double u) {
    BosonCoef b;
    b.kt = 1.0 / (cv * cv * dt);
    b.ks = dt;
    b.kr = dt * r;
    b.ku = dt * u;
    return b;
}

// exp(-2 pi i j / n) in FP64
static double2 twiddle_host(int j, int n) {
    const double a = -2.0 * M_PI * double(j) / double(n);
    return make_double2(std::cos(a), std::sin(a));
}

// The preconditioner's per-lattice tables (layout pc_blob_layout).
static std::vector<double> pc_table_blob(const FftPlan& pl, const FftPlan& pt) {
    const int L = pl.n, Lt = pt.n;
    const PcBlob b = pc_blob_layout(L, Lt);
    std::vector<double> v(static_cast<size_t>(b.size));
    for (int j = 0; j < L; ++j) {
        const double2 w = twiddle_host(j, L);
        v[size_t(b.twl + 2 * j)] = w.x;
        v[size_t(b.twl + 2 * j + 1)] = w.y;
        v[size_t(b.cosx + j)] = std::cos(2.0 * M_PI * double(fft_freq(pl, j)) / double(L));
    }
    for (int j = 0; j < Lt; ++j) {
        const double2 w = twiddle_host(j, Lt);
        v[size_t(b.twT + 2 * j)] = w.x;
        v[size_t(b.twT + 2 * j + 1)] = w.y;
    }
    return v;
}

static Coef<double> coef64_of(double dt, const hmc_params& p) {
    Coef<double> cf;
    for (int a = 0; a < 2; ++a) {
        cf.diag[a] = -1.0 - dt * p.mu[a];
        for (int d = 0; d < 2; ++d) cf.hop[a][d] = -dt * p.t[a][d];
    }
    cf.cpl = dt * p.lambda;
    cf.nn2 = 0;
    for (int a = 0; a < 2; ++a)
        for (int d = 0; d < 2; ++d) {
            cf.hop2[a][d] = -dt * p.tn[a][d];
            if (p.tn[a][d] != 0.0) cf.nn2 = 1;
        }
    return cf;
}

static void set_coefs(hmc_ctx* c) {
    const double dt = c->dtau;
    const hmc_params& p = c->p;
    c->cf64 = coef64_of(dt, p);
    for (int a = 0; a < 2; ++a) {
        c->cf32.diag[a] = float(c->cf64.diag[a]);
        for (int d = 0; d < 2; ++d) {
            c->cf32.hop[a][d] = float(c->cf64.hop[a][d]);
            c->cf32.hop2[a][d] = float(c->cf64.hop2[a][d]);
        }
    }
    c->cf32.cpl = float(c->cf64.cpl);
    c->cf32.nn2 = c->cf64.nn2;
    c->bc = boson_coef_of(dt, p.c, p.r, p.u);
    c->generation += 1;
}

static int check_params(const hmc_params* p) {
    if (p == nullptr) return fail(HMC_ERR_INVALID_ARG, "params is NULL");
    if (!(p->c > 0.0) || !std::isfinite(p->c)) return fail(HMC_ERR_INVALID_ARG, "boson velocity c must be > 0");
    if (!std::isfinite(p->lambda) || !std::isfinite(p->r) || !std::isfinite(p->u))
        return fail(HMC_ERR_INVALID_ARG, "non-finite coupling");
    for (int a = 0; a < 2; ++a) {
        if (!std::isfinite(p->mu[a])) return fail(HMC_ERR_INVALID_ARG, "non-finite mu");
        for (int d = 0; d < 2; ++d)
            if (!std::isfinite(p->t[a][d]) || !std::isfinite(p->tn[a][d]))
                return fail(HMC_ERR_INVALID_ARG, "non-finite hopping");
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
    if (p->precond != HMC_PRECOND_NONE && p->precond != HMC_PRECOND_FOURIER)
        return fail(HMC_ERR_INVALID_ARG, "unknown preconditioner");
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
    if (c->ws == nullptr) return fail(HMC_ERR_WORKSPACE, "workspace not set");
    return HMC_OK;
}

static int elem_grid(long long n) { return int((n + kBlock - 1) / kBlock); }

// Workspace layout: one walk that either only measures (base == nullptr) or also
// assigns the carved pointers.  Returns the bytes needed.
static size_t ws_layout(hmc_ctx* c, char* base) {
    const size_t VS = size_t(c->vec_sites), PS = size_t(c->phi_sites);
    const size_t sp64 = 4 * VS * sizeof(double2), sp32 = 4 * VS * sizeof(float2);
    const size_t nu = size_t(c->nunits);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + bytes, 256);
        return p;
    };
    char* st = take(sizeof(CgState) * 2 * nu);
    char* part = take(sizeof(double) * kPendKinds * size_t(c->pslots));
    char* gpart = take(sizeof(double) * 2 * size_t(c->ngblk));
    char* slots = take(sizeof(double) * kSlots);
    char* v64 = take(5 * sp64);
    char* v32 = take(6 * sp32);
    char* blob = take(sizeof(double) * size_t(c->blob_doubles));
    char* tr = take(2 * sp64);
    char* bos = take(2 * 3 * PS * sizeof(double));
    char* f32 = take(3 * PS * sizeof(float));
    char* mp = c->is_batch ? nullptr : take(sizeof(double) * 3 * size_t(std::max(pc_groups(c->lat.LL, pc_ncol<double>()), 256)));
    char* pw = c->is_batch ? nullptr : take(3 * PS * sizeof(double));
    char *un0 = nullptr, *un1 = nullptr, *bl0 = nullptr, *bl1 = nullptr, *ch = nullptr,
         *cb = nullptr, *cf = nullptr, *cs = nullptr, *pxy = nullptr, *pt0 = nullptr, *pt1 = nullptr,
         *mb0 = nullptr, *mb1 = nullptr, *rb0 = nullptr, *rb1 = nullptr;
    if (c->is_batch) {
        const size_t nch = size_t(c->bi.nchains);
        un0 = take(sizeof(UnitDesc) * nu);
        un1 = take(sizeof(UnitDesc) * nu);
        bl0 = take(sizeof(int2) * size_t(c->pslots));
        bl1 = take(sizeof(int2) * size_t(c->pslots));
        ch = take(sizeof(ChainDesc) * nch);
        cb = take(sizeof(int2) * size_t(c->ngblk));
        cf = take(sizeof(int) * (nch + 1));
        cs = take(sizeof(double) * kChainSlots * nch);
        pxy = take(sizeof(int2) * size_t(c->bi.nslices));
        pt0 = take(sizeof(int2) * size_t(c->bi.ngroups[0]));
        pt1 = take(sizeof(int2) * size_t(c->bi.ngroups[1]));
        mb0 = take(sizeof(int2) * size_t(c->pslots));
        mb1 = take(sizeof(int2) * size_t(c->pslots));
        rb0 = take(sizeof(int2) * size_t(c->pslots));
        rb1 = take(sizeof(int2) * size_t(c->pslots));
    }
    if (base) {
        c->st = reinterpret_cast<CgState*>(st);
        c->part = reinterpret_cast<double*>(part);
        c->gpart = reinterpret_cast<double*>(gpart);
        c->slots = reinterpret_cast<double*>(slots);
        c->r64 = reinterpret_cast<double2*>(v64);
        c->p064 = reinterpret_cast<double2*>(v64 + sp64);
        c->p164 = reinterpret_cast<double2*>(v64 + 2 * sp64);
        c->t64 = reinterpret_cast<double2*>(v64 + 3 * sp64);
        c->z64 = reinterpret_cast<double2*>(v64 + 4 * sp64);
        c->z32 = reinterpret_cast<float2*>(v32 + 5 * sp32);
        c->blob = reinterpret_cast<double*>(blob);
        c->r32 = reinterpret_cast<float2*>(v32);
        c->p032 = reinterpret_cast<float2*>(v32 + sp32);
        c->p132 = reinterpret_cast<float2*>(v32 + 2 * sp32);
        c->t32 = reinterpret_cast<float2*>(v32 + 3 * sp32);
        c->x32 = reinterpret_cast<float2*>(v32 + 4 * sp32);
        c->chi = reinterpret_cast<double2*>(tr);
        c->xsol = reinterpret_cast<double2*>(tr + sp64);
        c->pi = reinterpret_cast<double*>(bos);
        c->phi_save = reinterpret_cast<double*>(bos + 3 * PS * sizeof(double));
        c->phi32 = reinterpret_cast<float*>(f32);
        c->mpart = reinterpret_cast<double*>(mp);
        c->piw = reinterpret_cast<double*>(pw);
        if (c->is_batch) {
            c->bi.units[0] = reinterpret_cast<UnitDesc*>(un0);
            c->bi.units[1] = reinterpret_cast<UnitDesc*>(un1);
            c->bi.blocks[0] = reinterpret_cast<int2*>(bl0);
            c->bi.blocks[1] = reinterpret_cast<int2*>(bl1);
            c->bi.chains = reinterpret_cast<ChainDesc*>(ch);
            c->bi.cblocks = reinterpret_cast<int2*>(cb);
            c->bi.cfirst_dev = reinterpret_cast<int*>(cf);
            c->bi.cslots = reinterpret_cast<double*>(cs);
            c->bi.pxy_blocks = reinterpret_cast<int2*>(pxy);
            c->bi.pt_blocks[0] = reinterpret_cast<int2*>(pt0);
            c->bi.pt_blocks[1] = reinterpret_cast<int2*>(pt1);
            c->bi.mblocks[0] = reinterpret_cast<int2*>(mb0);
            c->bi.mblocks[1] = reinterpret_cast<int2*>(mb1);
            c->bi.rblocks[0] = reinterpret_cast<int2*>(rb0);
            c->bi.rblocks[1] = reinterpret_cast<int2*>(rb1);
        }
    }
    return off;
}

// CG launch shape: at most max_bpr workgroups per right-hand side (unit); workgroup b of a
// unit takes tiles b, b + bpr, ... (so every consumer reduces at most kMaxBpr partials).
static int clamp_bpr(int ntiles2, int max_bpr) { return ntiles2 < max_bpr ? ntiles2 : max_bpr; }

// Partial slots a unit needs per kind: the most workgroups any kernel runs on it (the CG steps,
// at most kMaxBpr; the preconditioner's tau pass, 4 column groups per FP64 group width).
static int unit_slots(const Lat& l) {
    return std::max(clamp_bpr(tiles2_host(l.vol), kMaxBpr), 4 * pc_groups(l.LL, kPcCols));
}

// A unit's march cut: rows per band at most `rows` (and at most what one thread per element, or
// pair of elements in FP32, of a 512-thread workgroup and 64 KB of LDS allow), `seg` slices per
// segment (default 8), more slices per segment if the unit's partial slots require it.  Zero
// workgroups when rows = 0 or no cut fits.
static MarchPlan batch_march_plan(const Lat& l, int rows, int seg, bool f32, int slots, int& parts, int& threads,
                                  size_t& lds) {
    parts = 0;
    threads = 0;
    lds = 0;
    if (rows <= 0) return MarchPlan{};
    const int per_row = f32 ? l.L / 2 : l.L;
    const int R = std::min({rows, l.L, kMarchCgThreads / per_row - 2});
    if (R < 1) return MarchPlan{};
    const size_t need = f32 ? march_cg_lds<float>(R, l.L) : march_cg_lds<double>(R, l.L);
    if (need > (size_t(64) << 10)) return MarchPlan{};
    MarchPlan mp = make_march_plan(l.L, l.Lt, R, seg > 0 ? seg : 8);
    while (mp.nband * mp.nseg > slots && mp.seglen < l.Lt) mp = make_march_plan(l.L, l.Lt, R, mp.seglen * 2);
    if (mp.nband * mp.nseg > slots) return MarchPlan{};
    parts = mp.nband * mp.nseg;
    threads = ((R + 2) * per_row + 63) / 64 * 64;
    lds = need;
    return mp;
}

// Batch: (re)write the unit and block tables of one precision's launch shape, with the march
// cuts of step A (this precision) and of the reliable update (FP64).
static int upload_batch_shape(hmc_ctx* c, int pi, int max_bpr) {
    BatchInfo& b = c->bi;
    std::vector<UnitDesc> units(size_t(c->nunits));
    std::vector<int2> blocks, mblocks, rblocks;
    bool m_ok = c->cgm_rows[pi] > 0, r_ok = m_ok && c->cgm_rows[0] > 0;
    b.mthreads[pi] = b.rthreads[pi] = 0;
    b.mlds[pi] = b.rlds[pi] = 0;
    int part = 0;
    for (int ch = 0; ch < b.nchains; ++ch) {
        const Lat& lat = b.lats[size_t(ch)];
        for (int k = 0; k < b.nrhs; ++k) {
            const int u = ch * b.nrhs + k;
            UnitDesc& d = units[size_t(u)];
            d.lat = lat;
            d.voff = b.sp_off[size_t(ch)] + 4LL * k * lat.vol;
            d.phioff = b.phi_off[size_t(ch)];
            d.bpr = clamp_bpr(tiles2_host(lat.vol), max_bpr);
            d.part = part;
            part += unit_slots(lat);
            d.chain = ch;
            d.pcoff = int(b.pcoff[size_t(ch)]);
            for (int w = 0; w < d.bpr; ++w) blocks.push_back(make_int2(u, w));
            int th = 0;
            size_t lds = 0;
            d.mp = batch_march_plan(lat, c->cgm_rows[pi], c->cgm_seg[pi], pi == 1, unit_slots(lat), d.mparts, th, lds);
            m_ok = m_ok && d.mparts > 0;
            b.mthreads[pi] = std::max(b.mthreads[pi], th);
            b.mlds[pi] = std::max(b.mlds[pi], lds);
            for (int w = 0; w < d.mparts; ++w) mblocks.push_back(make_int2(u, w));
            d.rmp = batch_march_plan(lat, c->cgm_rows[0], c->cgm_seg[0], false, unit_slots(lat), d.rparts, th, lds);
            r_ok = r_ok && d.rparts > 0;
            b.rthreads[pi] = std::max(b.rthreads[pi], th);
            b.rlds[pi] = std::max(b.rlds[pi], lds);
            for (int w = 0; w < d.rparts; ++w) rblocks.push_back(make_int2(u, w));
        }
    }
    b.nblocks[pi] = int(blocks.size());
    // a launch marches every unit or none
    b.mgrid[pi] = m_ok ? int(mblocks.size()) : 0;
    b.rgrid[pi] = r_ok ? int(rblocks.size()) : 0;
    b.hunits[pi] = units;
    if (c->ws != nullptr) {
        // launches already queued may still read the old tables
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(b.units[pi], units.data(), sizeof(UnitDesc) * units.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b.blocks[pi], blocks.data(), sizeof(int2) * blocks.size(), hipMemcpyHostToDevice));
        if (b.mgrid[pi] > 0)
            HIPCHK(hipMemcpy(b.mblocks[pi], mblocks.data(), sizeof(int2) * mblocks.size(), hipMemcpyHostToDevice));
        if (b.rgrid[pi] > 0)
            HIPCHK(hipMemcpy(b.rblocks[pi], rblocks.data(), sizeof(int2) * rblocks.size(), hipMemcpyHostToDevice));
    }
    return HMC_OK;
}

static int set_cg_shape(hmc_ctx* c, int precision, int max_bpr) {
    if (precision != HMC_MIXED) c->bpr64 = c->is_batch ? max_bpr : clamp_bpr(c->nblk2, max_bpr);
    if (precision != HMC_FP64) c->bpr32 = c->is_batch ? max_bpr : clamp_bpr(c->nblk2, max_bpr);
    c->generation += 1;
    if (c->is_batch) {
        if (precision != HMC_MIXED) {
            int rc = upload_batch_shape(c, 0, c->bpr64);
            if (rc) return rc;
        }
        if (precision != HMC_FP64) {
            int rc = upload_batch_shape(c, 1, c->bpr32);
            if (rc) return rc;
        }
    }
    return HMC_OK;
}

// Autotuned launch shapes: CG workgroups per right-hand side and the step-A march, per
// precision.  Kept process-wide per (lattice, right-hand sides, device) and on disk.
struct TuneChoice {
    int bpr[2] = {0, 0};    // [FP64, FP32]
    int mrows[2] = {0, 0};
    int mseg[2] = {0, 0};
    int mb[2] = {1, 1};     // step B marches too
};
struct TuneKey {
    int L, Lt, n, dev, nn2;
    bool operator<(const TuneKey& o) const {
        return std::tie(L, Lt, n, dev, nn2) < std::tie(o.L, o.Lt, o.n, o.dev, o.nn2);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneChoice> g_tuned;

// The on-disk cache: one line per key, "<key> bpr64 bpr32 rows64 slices64 rows32 slices32 stepb64
// stepb32".
static std::string tune_cache_path() {
    const char* e = std::getenv("HMC_TUNE_CACHE");
    if (e != nullptr) return (*e == 0 || std::strcmp(e, "off") == 0) ? std::string() : std::string(e);
    const char* x = std::getenv("XDG_CACHE_HOME");
    if (x != nullptr && *x) return std::string(x) + "/hmc/tune.txt";
    const char* h = std::getenv("HOME");
    if (h != nullptr && *h) return std::string(h) + "/.cache/hmc/tune.txt";
    return std::string();
}

// Device identity in a cache key: architecture and compute-unit count.
static std::string device_tag(int dev) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string t = std::string(pr.gcnArchName) + "/" + std::to_string(pr.multiProcessorCount);
    for (char& ch : t)
        if (ch == ' ' || ch == '\t') ch = '_';
    return t;
}

static bool tune_cache_lookup(const std::string& key, TuneChoice& out) {
    const std::string path = tune_cache_path();
    if (path.empty()) return false;
    FILE* f = std::fopen(path.c_str(), "r");
    if (f == nullptr) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        const size_t kl = key.size();
        if (std::strncmp(line, key.c_str(), kl) != 0 || line[kl] != ' ') continue;
        TuneChoice c;
        if (std::sscanf(line + kl, "%d %d %d %d %d %d %d %d", &c.bpr[0], &c.bpr[1], &c.mrows[0], &c.mseg[0],
                        &c.mrows[1], &c.mseg[1], &c.mb[0], &c.mb[1]) == 8 &&
            c.bpr[0] >= 1 && c.bpr[1] >= 1) {
            out = c;
            found = true;   // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

static void make_parent_dirs(const std::string& path) {
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
}

// Replace (or add) the key's line; written to a temporary file and renamed into place.
static void tune_cache_store(const std::string& key, const TuneChoice& c) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    make_parent_dirs(path);
    std::vector<std::string> keep;
    if (FILE* f = std::fopen(path.c_str(), "r")) {
        char line[1024];
        while (std::fgets(line, sizeof(line), f)) {
            const size_t kl = key.size();
            if (std::strncmp(line, key.c_str(), kl) == 0 && line[kl] == ' ') continue;
            keep.emplace_back(line);
        }
        std::fclose(f);
    }
    const std::string tmp = path + ".tmp" + std::to_string(long(getpid()));
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (f == nullptr) return;
    for (const std::string& l : keep) std::fputs(l.c_str(), f);
    std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", key.c_str(), c.bpr[0], c.bpr[1], c.mrows[0], c.mseg[0],
                 c.mrows[1], c.mseg[1], c.mb[0], c.mb[1]);
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) (void)std::remove(tmp.c_str());
}


// --------------------------------------------------------------------------------------
// geometry of a launch

static GeoOne geo_one(const hmc_ctx* c, int bpr) { return GeoOne{c->lat, bpr, bpr, c->pstride}; }
static GeoBatch geo_batch(const hmc_ctx* c, int pi) { return GeoBatch{c->bi.units[pi], c->bi.blocks[pi]}; }
static CGeoOne cgeo_one(const hmc_ctx* c, int npf) { return CGeoOne{c->lat, c->bc, npf}; }
static CGeoBatch cgeo_batch(const hmc_ctx* c) { return CGeoBatch{c->bi.chains, c->bi.cblocks}; }

// Everything a solve launches: the CG steps and, with the preconditioner, its slice passes and
// its tau pass, each with its geometry and grid.
template <class Geo>
struct Launch {
    Geo cg, pxy, pt;
    int ncg = 0, npxy = 0, npt = 0;
    size_t lds_xy = 0, lds_t = 0;
    int pt_threads = 0;   // tau-pass workgroup size (64 columns x chunks per column)
    bool pt_full = false; // every chunk of the tau pass is full (the instantiation without
                          // per-step predicates)
    bool nn2 = false;     // the operator hops by two sites (the instantiations with those terms)
    bool pc = false;
    bool r7 = false;      // some lattice extent has a factor 7 (radix-7 FFT stages)
    // CG step A as a march (one lattice, nearest-neighbour operator): plan, threads, LDS and
    // workgroups per unit (0: the tile kernels k_cg_a / k_cg_a2)
    MarchPlan cgm{};
    int cgm_threads = 0, cgm_per_unit = 0;
    size_t cgm_lds = 0;
    bool cgbm = false;    // step B marches with step A's cut
    // the FP64 stencils of the reliable update as marches (with the FP64 march shape, whenever
    // step A marches): plan, threads, LDS and workgroups per unit (0: the tile kernels)
    MarchPlan rum{};
    int rum_threads = 0, rum_per_unit = 0;
    size_t rum_lds = 0;
    // a batch's marches: every unit with its own cut (0 workgroups: the tile kernels)
    MGeoBatch bm{}, br{};
    int bm_grid = 0, bm_threads = 0, br_grid = 0, br_threads = 0;
    size_t bm_lds = 0, br_lds = 0;
};

template <typename R>
static Launch<GeoOne> launch_one(const hmc_ctx* c, int n) {
    const int pi = sizeof(R) == sizeof(float) ? 1 : 0;
    const int bpr = pi ? c->bpr32 : c->bpr64;
    Launch<GeoOne> l;
    l.cg = geo_one(c, bpr);
    l.ncg = bpr * n;
    l.pc = c->p.precond == HMC_PRECOND_FOURIER && c->pc_ok[pi];
    const int nxy = 4 * c->Lt, nt = 4 * pc_groups(c->lat.LL, kPcCols);
    l.pxy = GeoOne{c->lat, bpr, nxy, c->pstride};
    l.pt = GeoOne{c->lat, bpr, nt, c->pstride};
    l.npxy = nxy * n;
    l.npt = nt * n;
    l.lds_xy = c->lds_xy[pi];
    l.lds_t = c->lds_t[pi];
    l.pt_threads = kPcCols * c->pc_q[pi];
    l.pt_full = c->pc_full[pi];
    l.nn2 = c->cf64.nn2 != 0;
    l.r7 = c->pc_r7;
    l.cgbm = c->cgb_march[pi] != 0;
    // step A as a march: rows per band so that the band and its two neighbour rows have one
    // thread each (at most kMarchCgThreads); slices per segment for about one workgroup per
    // compute unit over all right-hand sides (at least 2)
    // (the production model's two-site hops need two rows beside the band on either side)
    if (c->cgm_rows[pi] > 0) {
        const int per_row = pi ? c->L / 2 : c->L, H = l.nn2 ? 2 : 1;
        const int rows = std::max(1, std::min(c->cgm_rows[pi], kMarchCgThreads / per_row - 2 * H));
        const size_t lds = march_cg_lds<R>(rows + 2 * H - 2, c->L);
        if (rows >= 1 && (rows + 2 * H) * per_row <= kMarchCgThreads && lds <= (size_t(64) << 10)) {
            const int nband = (c->L + std::min(rows, c->L) - 1) / std::min(rows, c->L);
            int seg = c->cgm_seg[pi];
            if (seg <= 0) seg = std::max(2, (c->Lt * nband * n + 255) / 256);
            l.cgm = make_march_plan(c->L, c->Lt, rows, seg);
            l.cgm_per_unit = l.cgm.nband * l.cgm.nseg;
            if (l.cgm_per_unit > c->pstride) l.cgm_per_unit = 0;   // partial slots: keep the tile kernels
            l.cgm_threads = ((std::min(rows, c->L) + 2 * H) * per_row + 63) / 64 * 64;
            l.cgm_lds = lds;
        }
    }
    // the reliable update's FP64 marches: one thread per element of the band and its two
    // neighbour rows, as the FP64 step-A march
    if (l.cgm_per_unit > 0 && c->cgm_rows[0] > 0 && !l.nn2) {
        const int rows = std::max(1, std::min(c->cgm_rows[0], kMarchCgThreads / c->L - 2));
        const size_t lds = march_cg_lds<double>(rows, c->L);
        if ((rows + 2) * c->L <= kMarchCgThreads && lds <= (size_t(64) << 10)) {
            const int nband = (c->L + std::min(rows, c->L) - 1) / std::min(rows, c->L);
            int seg = c->cgm_seg[0];
            if (seg <= 0) seg = std::max(2, (c->Lt * nband * n + 255) / 256);
            l.rum = make_march_plan(c->L, c->Lt, rows, seg);
            l.rum_per_unit = l.rum.nband * l.rum.nseg;
            if (l.rum_per_unit > c->pstride) l.rum_per_unit = 0;
            l.rum_threads = ((std::min(rows, c->L) + 2) * c->L + 63) / 64 * 64;
            l.rum_lds = lds;
        }
    }
    return l;
}

template <typename R>
static Launch<GeoBatch> launch_batch(const hmc_ctx* c) {
    const int pi = sizeof(R) == sizeof(float) ? 1 : 0;
    Launch<GeoBatch> l;
    l.cg = geo_batch(c, pi);
    l.ncg = c->bi.nblocks[pi];
    l.pc = c->p.precond == HMC_PRECOND_FOURIER && c->pc_ok[pi];
    l.pxy = GeoBatch{c->bi.units[pi], c->bi.pxy_blocks};
    l.pt = GeoBatch{c->bi.units[pi], c->bi.pt_blocks[pi]};
    l.npxy = c->bi.nslices;
    l.npt = c->bi.ngroups[pi];
    l.lds_xy = c->lds_xy[pi];
    l.lds_t = c->lds_t[pi];
    l.pt_threads = kPcCols * c->pc_q[pi];
    l.pt_full = c->pc_full[pi];
    l.nn2 = c->cf64.nn2 != 0;
    l.r7 = c->pc_r7;
    l.cgbm = c->cgb_march[pi] != 0;
    if (!l.nn2 && c->bi.mgrid[pi] > 0) {
        l.bm = MGeoBatch{c->bi.units[pi], c->bi.mblocks[pi], 0};
        l.bm_grid = c->bi.mgrid[pi];
        l.bm_threads = c->bi.mthreads[pi];
        l.bm_lds = c->bi.mlds[pi];
        if (c->bi.rgrid[pi] > 0) {
            l.br = MGeoBatch{c->bi.units[pi], c->bi.rblocks[pi], 1};
            l.br_grid = c->bi.rgrid[pi];
            l.br_threads = c->bi.rthreads[pi];
            l.br_lds = c->bi.rlds[pi];
        }
    }
    return l;
}

// --------------------------------------------------------------------------------------
// conjugate-gradient engine

template <typename R> struct KrylovBufs;
template <> struct KrylovBufs<double> {
    static CgVecs<double> get(hmc_ctx* c, double2* x, bool pc) {
        return {c->r64, c->p064, c->p164, c->t64, x, pc ? c->z64 : c->r64};
    }
    static const double* phi(hmc_ctx*, const double* phi64) { return phi64; }
    static Coef<double> cf(hmc_ctx* c) { return c->cf64; }
};
template <> struct KrylovBufs<float> {
    static CgVecs<float> get(hmc_ctx* c, double2*, bool pc) {
        return {c->r32, c->p032, c->p132, c->t32, c->x32, pc ? c->z32 : c->r32};
    }
    static const float* phi(hmc_ctx* c, const double*) { return c->phi32; }
    static Coef<float> cf(hmc_ctx* c) { return c->cf32; }
};

static bool finished(int mode) { return mode == CG_DONE || mode == CG_STOPPED || mode == CG_FAILED; }

// Control block for the next CG launch; advances the state-record parity.
static CgCtl next_ctl(hmc_ctx* c, int expect) {
    CgCtl k;
    k.st_in = c->st + size_t(c->seq & 1) * c->nunits;
    k.st_out = c->st + size_t((c->seq + 1) & 1) * c->nunits;
    k.part = c->part;
    k.nslots = c->pslots;
    k.expect = expect;
    k.nparts = c->next_nparts;
    c->next_nparts = 0;
    c->seq += 1;
    return k;
}

static const CgState* current_states(const hmc_ctx* c) { return c->st + size_t(c->seq & 1) * c->nunits; }

// Launch the instantiation of a stencil kernel with or without the hops by two sites.
#define HMC_LAUNCH_NN2(nn2, KT, KF, ...)           \
    do {                                          \
        if (nn2) hipLaunchKernelGGL(KT, __VA_ARGS__); \
        else hipLaunchKernelGGL(KF, __VA_ARGS__);     \
    } while (0)
#define HMC_EXT_LAUNCH_NN2(nn2, KT, KF, ...)           \
    do {                                              \
        if (nn2) hipExtLaunchKernelGGL(KT, __VA_ARGS__); \
        else hipExtLaunchKernelGGL(KF, __VA_ARGS__);     \
    } while (0)

// Launch kernel k; with events e, start/stop timestamps of pass q come from its own dispatch.
template <typename... P, typename... A>
static void launch_timed(void (*k)(P...), int grid, int block, size_t lds, hipStream_t s, hipEvent_t* e, int q,
                         A&&... a) {
    if (e) hipExtLaunchKernelGGL(k, dim3(grid), dim3(block), lds, s, e[2 * q], e[2 * q + 1], 0, static_cast<P>(a)...);
    else hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, s, static_cast<P>(a)...);
}

// The three preconditioner passes, z = P r, for the units whose residual just changed; the
// first consumes the pending kind `expect1` (a new |r|^2, the first |b|^2 or a true residual).
template <typename R, class Geo, int MAXR>
static int enqueue_pc_r(hmc_ctx* c, const Launch<Geo>& lc, const CgVecs<R>& v, int expect1, hipStream_t s,
                        hipEvent_t* e) {
    // e: null, or the start/stop events of the three passes (timed by their own dispatches)
    launch_timed(k_pc_xy<R, false, Geo, MAXR>, lc.npxy, kPcBlock, lc.lds_xy, s, e, 0,
                 next_ctl(c, expect1), lc.pxy, v.r, v.z, c->blob);
    LAUNCHCHK();
    if (lc.pt_full)
        launch_timed(k_pc_t<R, Geo, true>, lc.npt, lc.pt_threads, lc.lds_t, s, e, 1,
                     next_ctl(c, PEND_NONE), lc.pt, v.z, c->blob, c->cf64);
    else
        launch_timed(k_pc_t<R, Geo, false>, lc.npt, lc.pt_threads, lc.lds_t, s, e, 1,
                     next_ctl(c, PEND_NONE), lc.pt, v.z, c->blob, c->cf64);
    LAUNCHCHK();
    launch_timed(k_pc_xy<R, true, Geo, MAXR>, lc.npxy, kPcBlock, lc.lds_xy, s, e, 2,
                 next_ctl(c, PEND_RZ), lc.pxy, v.z, v.z, c->blob);
    LAUNCHCHK();
    return HMC_OK;
}

template <typename R, class Geo>
static int enqueue_pc(hmc_ctx* c, const Launch<Geo>& lc, const CgVecs<R>& v, int expect1, hipStream_t s,
                      hipEvent_t* e = nullptr) {
    return lc.r7 ? enqueue_pc_r<R, Geo, 7>(c, lc, v, expect1, s, e) : enqueue_pc_r<R, Geo, 5>(c, lc, v, expect1, s, e);
}

// Launches of one status chunk (kept even, so that every chunk starts at the same record
// parity): without preconditioner 2 per iteration + 4; with it 5 per iteration + 6, plus a
// finalize if odd.
static int chunk_launches(int chunk, bool pc) {
    if (!pc) return 2 * chunk + 4;
    const int n = 5 * chunk + 6;
    return n + (n & 1);
}

// Step A (step_b false) or step B as a march: one lattice (every vector cut alike) or a batch
// (each unit its own cut); ev: start/stop events for a timed launch.
template <typename R, class Geo>
static void launch_step_march(hmc_ctx* c, const Launch<Geo>& lc, bool step_b, const CgCtl& ka, const CgVecs<R>& v,
                              const R* phik, const Coef<R>& cf, int grid, int threads, size_t lds, const hipEvent_t* ev,
                              hipStream_t s) {
    auto go = [&](auto mg, auto nn2) {
        using MG = decltype(mg);
        constexpr bool N2 = decltype(nn2)::value;
        auto launch = [&](auto kern) {
            if (ev) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, s, ev[0], ev[1], 0, ka, mg, v, phik, cf);
            else hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, s, ka, mg, v, phik, cf);
        };
        if constexpr (sizeof(R) == sizeof(float)) {
            if (step_b) launch(k_cg_b2_march<MG, N2>);
            else launch(k_cg_a2_march<MG, N2>);
        } else {
            if (step_b) launch(k_cg_b_march<MG, N2>);
            else launch(k_cg_a_march<MG, N2>);
        }
    };
    // batches march the nearest-neighbour operator only
    if constexpr (std::is_same<Geo, GeoOne>::value) {
        const MGeoOne mg{lc.cg.lat, lc.cgm, lc.cg.bpr, c->pstride};
        if (lc.nn2) go(mg, std::true_type{});
        else go(mg, std::false_type{});
    } else {
        go(lc.bm, std::false_type{});
    }
}

// One status chunk: `chunk` iterations (steps A and B, and the preconditioner passes), then
// the reliable-update / true-residual sequence for units in `filter`, then what makes the
// published records complete.  first: the first chunk of an unpreconditioned solve (its
// step A then reduces |b|^2).
template <typename R, class Geo>
static int enqueue_chunk(hmc_ctx* c, const Launch<Geo>& lc, int n, const double* phi64, const double2* b,
                         double2* x, int chunk, int filter, bool first, bool sample, int kslot, hipStream_t s) {
    CgVecs<R> v = KrylovBufs<R>::get(c, x, lc.pc);
    const R* phik = KrylovBufs<R>::phi(c, phi64);
    const Coef<R> cf = KrylovBufs<R>::cf(c);
    const Geo geo = lc.cg;
    const int grid = lc.ncg;
    for (int i = 0; i < chunk; ++i) {
        const int expect_a = lc.pc ? PEND_NONE : (i > 0 ? PEND_RR : (first ? PEND_BB : PEND_NONE));
        const CgCtl ka = next_ctl(c, expect_a);
        // step A as a march (one lattice, or every unit of a batch with its own cut); step B, a
        // march with the same cut or its tile kernel, reduces the march's partials
        int mgrid = 0, mthreads = 0, mparts = 0;
        size_t mlds = 0;
        if constexpr (std::is_same<Geo, GeoOne>::value) {
            if (lc.cgm_per_unit > 0) {
                mgrid = lc.cgm_per_unit * n;
                mthreads = lc.cgm_threads;
                mlds = lc.cgm_lds;
                mparts = lc.cgm_per_unit;
            }
        } else if (lc.bm_grid > 0) {
            mgrid = lc.bm_grid;
            mthreads = lc.bm_threads;
            mlds = lc.bm_lds;
            mparts = kPartsMarch;
        }
        if (mgrid > 0) {
            c->next_nparts = mparts;
            const CgCtl kb = next_ctl(c, PEND_TT);
            const hipEvent_t* e = (sample && i == chunk / 2) ? c->tev[kslot] : nullptr;
            // the next iteration's step A too (the solution update alternates between them)
            const hipEvent_t* ea = e ? e : (sample && i == chunk / 2 + 1) ? c->tev[kslot] + 10 : nullptr;
            launch_step_march<R, Geo>(c, lc, false, ka, v, phik, cf, mgrid, mthreads, mlds, ea, s);
            LAUNCHCHK();
            if (lc.cgbm) {
                // step B with the same cut; the next kernel reduces its partials
                launch_step_march<R, Geo>(c, lc, true, kb, v, phik, cf, mgrid, mthreads, mlds, e ? e + 2 : nullptr, s);
                LAUNCHCHK();
                c->next_nparts = mparts;
            } else {
                // the tile kernel, which reads t while the MALL still holds it
                if constexpr (sizeof(R) == sizeof(float)) {
                    if (e) HMC_EXT_LAUNCH_NN2(lc.nn2, (k_cg_b2<Geo, true>), (k_cg_b2<Geo, false>), dim3(grid),
                                              dim3(kBlock), 0, s, e[2], e[3], 0, kb, geo, v, phik, cf);
                    else HMC_LAUNCH_NN2(lc.nn2, (k_cg_b2<Geo, true>), (k_cg_b2<Geo, false>), dim3(grid), dim3(kBlock), 0,
                                        s, kb, geo, v, phik, cf);
                } else {
                    if (e) HMC_EXT_LAUNCH_NN2(lc.nn2, (k_cg_b<R, Geo, true>), (k_cg_b<R, Geo, false>), dim3(grid),
                                              dim3(kBlock), 0, s, e[2], e[3], 0, kb, geo, v, phik, cf);
                    else HMC_LAUNCH_NN2(lc.nn2, (k_cg_b<R, Geo, true>), (k_cg_b<R, Geo, false>), dim3(grid),
                                        dim3(kBlock), 0, s, kb, geo, v, phik, cf);
                }
                LAUNCHCHK();
            }
            if (lc.pc) {
                int rc = enqueue_pc<R, Geo>(c, lc, v, PEND_RR, s, e ? c->tev[kslot] + 4 : nullptr);
                if (rc) return rc;
            }
            continue;
        }
        const CgCtl kb = next_ctl(c, PEND_TT);
        if (sample && i == chunk / 2) {
            // timestamps from the dispatches themselves (not captured into graphs)
            hipEvent_t* e = c->tev[kslot];
            if constexpr (sizeof(R) == sizeof(float)) {
                HMC_EXT_LAUNCH_NN2(lc.nn2, (k_cg_a2<Geo, true>), (k_cg_a2<Geo, false>), dim3(grid), dim3(kBlock), 0, s,
                                   e[0], e[1], 0, ka, geo, v, phik, cf);
                LAUNCHCHK();
                HMC_EXT_LAUNCH_NN2(lc.nn2, (k_cg_b2<Geo, true>), (k_cg_b2<Geo, false>), dim3(grid), dim3(kBlock), 0, s,
                                   e[2], e[3], 0, kb, geo, v, phik, cf);
            } else {
                HMC_EXT_LAUNCH_NN2(lc.nn2, (k_cg_a<R, Geo, true>), (k_cg_a<R, Geo, false>), dim3(grid), dim3(kBlock), 0,
                                   s, e[0], e[1], 0, ka, geo, v, phik, cf);
                LAUNCHCHK();
                HMC_EXT_LAUNCH_NN2(lc.nn2, (k_cg_b<R, Geo, true>), (k_cg_b<R, Geo, false>), dim3(grid), dim3(kBlock), 0,
                                   s, e[2], e[3], 0, kb, geo, v, phik, cf);
            }
            LAUNCHCHK();
        } else if (sample && i == chunk / 2 + 1) {
            // the next iteration's step A (the solution update alternates between them)
            hipEvent_t* e = c->tev[kslot] + 10;
            if constexpr (sizeof(R) == sizeof(float)) {
                HMC_EXT_LAUNCH_NN2(lc.nn2, (k_cg_a2<Geo, true>), (k_cg_a2<Geo, false>), dim3(grid), dim3(kBlock), 0, s,
                                   e[0], e[1], 0, ka, geo, v, phik, cf);
                LAUNCHCHK();
                HMC_LAUNCH_NN2(lc.nn2, (k_cg_b2<Geo, true>), (k_cg_b2<Geo, false>), dim3(grid), dim3(kBlock), 0, s, kb,
                               geo, v, phik, cf);
            } else {
                HMC_EXT_LAUNCH_NN2(lc.nn2, (k_cg_a<R, Geo, true>), (k_cg_a<R, Geo, false>), dim3(grid), dim3(kBlock), 0,
                                   s, e[0], e[1], 0, ka, geo, v, phik, cf);
                LAUNCHCHK();
                HMC_LAUNCH_NN2(lc.nn2, (k_cg_b<R, Geo, true>), (k_cg_b<R, Geo, false>), dim3(grid), dim3(kBlock), 0, s,
                               kb, geo, v, phik, cf);
            }
            LAUNCHCHK();
        } else {
            if constexpr (sizeof(R) == sizeof(float)) {
                HMC_LAUNCH_NN2(lc.nn2, (k_cg_a2<Geo, true>), (k_cg_a2<Geo, false>), dim3(grid), dim3(kBlock), 0, s, ka,
                               geo, v, phik, cf);
                LAUNCHCHK();
                HMC_LAUNCH_NN2(lc.nn2, (k_cg_b2<Geo, true>), (k_cg_b2<Geo, false>), dim3(grid), dim3(kBlock), 0, s, kb,
                               geo, v, phik, cf);
            } else {
                HMC_LAUNCH_NN2(lc.nn2, (k_cg_a<R, Geo, true>), (k_cg_a<R, Geo, false>), dim3(grid), dim3(kBlock), 0, s,
                               ka, geo, v, phik, cf);
                LAUNCHCHK();
                HMC_LAUNCH_NN2(lc.nn2, (k_cg_b<R, Geo, true>), (k_cg_b<R, Geo, false>), dim3(grid), dim3(kBlock), 0, s,
                               kb, geo, v, phik, cf);
            }
            LAUNCHCHK();
        }
        if (lc.pc) {
            int rc = enqueue_pc<R, Geo>(c, lc, v, PEND_RR, s, sample && i == chunk / 2 ? c->tev[kslot] + 4 : nullptr);
            if (rc) return rc;
        }
    }
    hipLaunchKernelGGL((k_ru_fold<R, Geo>), dim3(grid), dim3(kBlock), 0, s, next_ctl(c, lc.pc ? PEND_NONE : PEND_RR),
                       geo, x, v, filter);
    LAUNCHCHK();
    // t64 = M x64 and r = b - M^dagger t64 as marches; the record after them reduces the
    // march's partials
    int rgrid = 0, rthreads = 0, rparts = 0;
    size_t rlds = 0;
    if constexpr (std::is_same<Geo, GeoOne>::value) {
        if (lc.rum_per_unit > 0) {
            rgrid = lc.rum_per_unit * n;
            rthreads = lc.rum_threads;
            rlds = lc.rum_lds;
            rparts = lc.rum_per_unit;
        }
    } else if (lc.br_grid > 0) {
        rgrid = lc.br_grid;
        rthreads = lc.br_threads;
        rlds = lc.br_lds;
        rparts = kPartsRu;
    }
    const bool ru_march = rgrid > 0;
    if (ru_march) {
        auto go = [&](auto mg) {
            using MG = decltype(mg);
            hipLaunchKernelGGL((k_ru_apply_march<MG>), dim3(rgrid), dim3(rthreads), rlds, s, next_ctl(c, PEND_NONE), mg,
                               x, c->t64, phi64, c->cf64, filter);
            hipLaunchKernelGGL((k_ru_resid_march<R, MG>), dim3(rgrid), dim3(rthreads), rlds, s, next_ctl(c, PEND_NONE),
                               mg, b, c->t64, phi64, c->cf64, v.r, filter);
        };
        if constexpr (std::is_same<Geo, GeoOne>::value) go(MGeoOne{geo.lat, lc.rum, geo.bpr, c->pstride});
        else go(lc.br);
        LAUNCHCHK();
        c->next_nparts = rparts;
    }
    if (!ru_march) {
        HMC_LAUNCH_NN2(lc.nn2, (k_ru_apply<Geo, true>), (k_ru_apply<Geo, false>), dim3(grid), dim3(kBlock), 0, s,
                       next_ctl(c, PEND_NONE), geo, x, c->t64, phi64, c->cf64, filter);
        LAUNCHCHK();
        HMC_LAUNCH_NN2(lc.nn2, (k_ru_resid<R, Geo, true>), (k_ru_resid<R, Geo, false>), dim3(grid), dim3(kBlock), 0,
                       s, next_ctl(c, PEND_NONE), geo, b, c->t64, phi64, c->cf64, v.r, filter);
        LAUNCHCHK();
    }
    if (lc.pc) {
        int rc = enqueue_pc<R, Geo>(c, lc, v, PEND_RU, s);
        if (rc) return rc;
        if ((5 * chunk + 6) & 1) {
            hipLaunchKernelGGL(k_cg_finalize<Geo>, dim3(n), dim3(kBlock), 0, s, next_ctl(c, PEND_NONE), geo, 0);
            LAUNCHCHK();
        }
    } else {
        hipLaunchKernelGGL(k_cg_finalize<Geo>, dim3(n), dim3(kBlock), 0, s, next_ctl(c, PEND_RU), geo, 0);
        LAUNCHCHK();
    }
    return HMC_OK;
}

// Capture the two kinds of status chunk of this solve shape into executable graphs, unless
// the cached ones match.  Capture happens on the context's own (idle) stream; the graphs
// are launched on the caller's stream.
template <typename R, class Geo>
static int prepare_graphs(hmc_ctx* c, const Launch<Geo>& lc, int n, const double* phi64, const double2* b,
                          double2* x, int chunk, int filter, int parity) {
    const int pi = sizeof(R) == sizeof(float) ? 1 : 0;
    CgGraphs& G = c->cgg[pi];
    const auto key = std::make_tuple(lc.ncg, (const void*)phi64, (const void*)b, (const void*)x,
                                     (const void*)c->st, n, chunk, filter, c->nunits, c->generation,
                                     lc.pc ? 1 : 0);
    if (G.exec[0] != nullptr && G.key == key) return HMC_OK;
    for (int g = 0; g < 2; ++g) {
        if (G.exec[g]) (void)hipGraphExecDestroy(G.exec[g]);
        G.exec[g] = nullptr;
    }
    if (c->cap_stream == nullptr) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const int saved = c->seq;
    for (int g = 0; g < 2; ++g) {
        hipGraph_t graph = nullptr;
        c->seq = parity;                              // every chunk starts at this parity
        c->next_nparts = 0;
        HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_chunk<R, Geo>(c, lc, n, phi64, b, x, chunk, filter, g == 0, false, 0, c->cap_stream);
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            c->seq = saved;
            return rc;
        }
        if (e != hipSuccess) {
            c->seq = saved;
            return fail(HMC_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
        }
        const hipError_t ei = hipGraphInstantiate(&G.exec[g], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            c->seq = saved;
            return fail(HMC_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(ei));
        }
    }
    c->seq = saved;
    G.key = key;
    return HMC_OK;
}

// Solve (M^dagger M) x_u = b_u for the n units of the launch.  Final records are left in
// c->h_st[0 .. n).  Returns HMC_OK, HMC_ERR_NOT_CONVERGED or HMC_ERR_NONFINITE.
// The start of a solve: FP32 copy of phi (mixed precision), the CG start (x = 0, r = b, |b|^2),
// and with the preconditioner z = P b.  Resets the launch counter.
template <typename R, class Geo>
static int cg_prologue(hmc_ctx* c, const Launch<Geo>& lc, const double* phi64, const double2* b, double2* x,
                       hipStream_t s) {
    const bool mixed = sizeof(R) == sizeof(float);
    CgVecs<R> v = KrylovBufs<R>::get(c, x, lc.pc);
    if (mixed) {
        hipLaunchKernelGGL(k_to_f32, dim3(elem_grid(3LL * c->phi_sites)), dim3(kBlock), 0, s, phi64,
                           c->phi32, int(3 * c->phi_sites));
        LAUNCHCHK();
    }
    const double tol = c->p.cg_tol;
    c->seq = 0;
    c->next_nparts = 0;
    hipLaunchKernelGGL((k_cg_init<R, Geo>), dim3(lc.ncg), dim3(kBlock), 0, s, next_ctl(c, PEND_NONE), lc.cg, b, x,
                       v, tol * tol, mixed ? kRuDrop2 : 0.0, c->p.cg_maxit, lc.pc ? 1 : 0);
    LAUNCHCHK();
    if (lc.pc) {
        int rc = enqueue_pc<R, Geo>(c, lc, v, PEND_BB, s);
        if (rc) return rc;
    }
    return HMC_OK;
}

// k0 > 0: the start and the first k0 status chunks are already on the stream (a step graph);
// the host reads the records once and goes on with further chunks only if some unit is not
// finished.
template <typename R, class Geo>
static int cg_run(hmc_ctx* c, const Launch<Geo>& lc, int n, const double* phi64, const double2* b,
                  double2* x, hipStream_t s, int k0 = 0) {
    const bool mixed = sizeof(R) == sizeof(float);
    const double tol = c->p.cg_tol;
    const int chunk = mixed ? c->p.reliable_every : kCheckEvery;
    const int ru_filter = mixed ? (F_ACTIVE | F_CONV_ITER | F_MAXIT) : (F_CONV_ITER | F_MAXIT);
    const bool use_graphs = c->graphs;
    // launches before the first chunk: the start (1), and with the preconditioner z = P b (3)
    const int parity = lc.pc ? 0 : 1;
    if (use_graphs) {
        int rc = prepare_graphs<R, Geo>(c, lc, n, phi64, b, x, chunk, ru_filter, parity);
        if (rc) return rc;
    }
    const size_t st_bytes = sizeof(CgState) * size_t(n);
    bool done_early = false;
    if (k0 == 0) {
        int rc = cg_prologue<R, Geo>(c, lc, phi64, b, x, s);
        if (rc) return rc;
    } else {
        HIPCHK(hipMemcpyAsync(c->h_st, current_states(c), st_bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        done_early = true;
        for (int j = 0; j < n; ++j) done_early = done_early && finished(c->h_st[j].mode);
    }

    const int nlaunch = chunk_launches(chunk, lc.pc);
    int issued = k0 * chunk;
    int k = k0;
    bool have_prev = false;
    const int kt_a = mixed ? 0 : 2;
    const bool sample = c->timing && !use_graphs;
    bool start_active_prev = true;   // were all units iterating when chunk k-1 began
    // Chunks are issued one ahead of the status read, so the GPU never idles on the host;
    // once every unit is finished the remaining launches return at once.
    for (; !done_early;) {
        if (use_graphs) {
            HIPCHK(hipGraphLaunch(c->cgg[mixed ? 1 : 0].exec[k == 0 ? 0 : 1], s));
            c->seq += nlaunch;
        } else {
            int rc = enqueue_chunk<R, Geo>(c, lc, n, phi64, b, x, chunk, ru_filter, k == 0, sample, k & 1, s);
            if (rc) return rc;
        }
        issued += chunk;
        HIPCHK(hipMemcpyAsync(c->h_st + size_t(k & 1) * c->nunits, current_states(c), st_bytes,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(c->ev[k & 1], s));
        if (have_prev) {
            HIPCHK(hipEventSynchronize(c->ev[(k - 1) & 1]));
            const CgState* hs = c->h_st + size_t((k - 1) & 1) * c->nunits;
            bool all = true, all_active = true;
            for (int j = 0; j < n; ++j) {
                all = all && finished(hs[j].mode);
                all_active = all_active && hs[j].mode == CG_ACTIVE;
            }
            // chunk k-1 began in the state chunk k-2 ended in; if every unit was iterating
            // then and is still iterating at its end, its mid-chunk sample did full work
            if (sample && start_active_prev && all_active) {
                const hipEvent_t* ev = c->tev[(k - 1) & 1];
                for (int q = 0; q < (lc.pc ? 5 : 2); ++q) {
                    float t = 0.f;
                    HIPCHK(hipEventElapsedTime(&t, ev[2 * q], ev[2 * q + 1]));
                    const int slot = q < 2 ? kt_a + q : (mixed ? 4 : 7) + q - 2;
                    c->kt.ms[slot] += t;
                    c->kt.count[slot] += 1;
                }
                if (chunk / 2 + 1 < chunk) {
                    float t = 0.f;
                    HIPCHK(hipEventElapsedTime(&t, ev[10], ev[11]));
                    c->kt.ms[mixed ? 10 : 11] += t;
                    c->kt.count[mixed ? 10 : 11] += 1;
                }
            }
            start_active_prev = all_active;
            if (all) break;
        }
        have_prev = true;
        ++k;
        // the device enforces cg_maxit; this bound only guards the host loop
        if (issued > c->p.cg_maxit + 4 * chunk) break;
    }
    if (!done_early) {
        HIPCHK(hipMemcpyAsync(c->h_st, current_states(c), st_bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    int status = HMC_OK;
    c->sg_last_iters = 0;
    for (int j = 0; j < n; ++j) c->sg_last_iters = std::max(c->sg_last_iters, c->h_st[j].iters);
    for (int j = 0; j < n; ++j) {
        const CgState& h = c->h_st[j];
        if (h.mode == CG_FAILED) status = HMC_ERR_NONFINITE;
        else if (h.mode != CG_DONE && status == HMC_OK) status = HMC_ERR_NOT_CONVERGED;
    }
    if (status == HMC_ERR_NONFINITE) return fail(status, "CG met a non-finite value");
    if (status == HMC_ERR_NOT_CONVERGED)
        return fail(status, "CG did not reach tol %.3g within %d iterations", tol, c->p.cg_maxit);
    return HMC_OK;
}

// A leapfrog step's drift (drift_pi non-null: phi += eps pi) and solve, or a trajectory's first
// solve, replayed from one graph: the drift, the solve's start and K status chunks, K from the
// last solve's iterations with a margin of a tenth and one chunk, rounded up to an even count
// (finished units make the spare chunks' kernels return after reading their record).  The host then reads the records once and
// finishes the solve with further chunks if K did not suffice.  Graphs are cached by shape.
template <typename R, class Geo>
static int solve_step_graph(hmc_ctx* c, const Launch<Geo>& lc, int n, double* phi, const double* drift_pi,
                            double eps, const double2* b, double2* x, hipStream_t s) {
    const bool mixed = sizeof(R) == sizeof(float);
    const int chunk = mixed ? c->p.reliable_every : kCheckEvery;
    const int ru_filter = mixed ? (F_ACTIVE | F_CONV_ITER | F_MAXIT) : (F_CONV_ITER | F_MAXIT);
    int K = (int(1.1 * c->sg_last_iters) + 2 * chunk - 1) / chunk;
    K = std::min((K + 1) / 2 * 2, c->p.cg_maxit / chunk + 2);
    const auto key = std::make_tuple(K, drift_pi ? 1 : 0, (const void*)phi, (const void*)drift_pi, (const void*)b,
                                     (const void*)x, n, c->generation, lc.pc ? 1 : 0, mixed ? 1 : 0, eps,
                                     c->nunits);
    hmc_ctx::StepGraph* g = nullptr;
    for (auto& e : c->sgs)
        if (e.key == key) g = &e;
    if (g == nullptr) {
        if (c->sgs.size() >= 8) {
            (void)hipGraphExecDestroy(c->sgs.front().exec);
            c->sgs.erase(c->sgs.begin());
        }
        if (c->cap_stream == nullptr) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = HMC_OK;
        if (drift_pi) {
            hipLaunchKernelGGL(k_drift, dim3(elem_grid(3LL * c->phi_sites)), dim3(kBlock), 0, c->cap_stream, phi,
                               drift_pi, eps, int(3 * c->phi_sites));
            if (hipGetLastError() != hipSuccess) rc = HMC_ERR_HIP;
        }
        if (rc == HMC_OK) rc = cg_prologue<R, Geo>(c, lc, phi, b, x, c->cap_stream);
        for (int k = 0; k < K && rc == HMC_OK; ++k)
            rc = enqueue_chunk<R, Geo>(c, lc, n, phi, b, x, chunk, ru_filter, k == 0, false, 0, c->cap_stream);
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(HMC_ERR_HIP, "step graph capture failed: %s", hipGetErrorString(e));
        hmc_ctx::StepGraph sg;
        sg.key = key;
        sg.seq_after = c->seq;
        const hipError_t ei = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(HMC_ERR_HIP, "step graph instantiate failed: %s", hipGetErrorString(ei));
        c->sgs.push_back(sg);
        g = &c->sgs.back();
    }
    HIPCHK(hipGraphLaunch(g->exec, s));
    c->seq = g->seq_after;
    c->next_nparts = 0;
    return cg_run<R, Geo>(c, lc, n, phi, b, x, s, K);
}

static double true_resid_of(const CgState& h) { return h.bb > 0.0 ? std::sqrt(h.rr_true / h.bb) : 0.0; }

static void fill_cg_stats(const hmc_ctx* c, int n, int status, hmc_cg_stats* stats) {
    if (stats == nullptr) return;
    std::memset(stats, 0, sizeof(*stats));
    stats->n = n;
    stats->status = status;
    for (int j = 0; j < n; ++j) {
        const CgState& h = c->h_st[j];
        stats->iterations[j] = h.iters;
        stats->reliable_updates[j] = h.n_ru;
        stats->true_resid[j] = true_resid_of(h);
    }
}

static int drift(hmc_ctx* c, double* phi, const double* pi, double eps, hipStream_t s);

// The drift phi += eps pi (pi non-null) and a solve: from a step graph when they are enabled,
// the metric is the identity and an earlier solve sized the graph; else launched one by one.
template <typename R, class Geo>
static int drift_solve(hmc_ctx* c, const Launch<Geo>& lc, int n, double* phi, const double* pi, double eps,
                       const double2* b, double2* x, hipStream_t s) {
    if (c->step_graphs && c->sigma == nullptr && c->sg_last_iters > 0)
        return solve_step_graph<R, Geo>(c, lc, n, phi, pi, eps, b, x, s);
    if (pi) {
        int rc = drift(c, phi, pi, eps, s);
        if (rc) return rc;
    }
    return cg_run<R, Geo>(c, lc, n, phi, b, x, s);
}

// One lattice, n right-hand sides; with pi, the drift phi += eps pi first (phi is written
// only then).
static int cg_dispatch(hmc_ctx* c, const double* phi, const double2* b, double2* x, int n, hmc_cg_stats* stats,
                       hipStream_t s, const double* pi = nullptr, double eps = 0.0) {
    int rc;
    double* pw = const_cast<double*>(phi);
    if (c->p.precision == HMC_MIXED)
        rc = drift_solve<float>(c, launch_one<float>(c, n), n, pw, pi, eps, b, x, s);
    else
        rc = drift_solve<double>(c, launch_one<double>(c, n), n, pw, pi, eps, b, x, s);
    if (rc == HMC_OK || rc == HMC_ERR_NOT_CONVERGED || rc == HMC_ERR_NONFINITE) fill_cg_stats(c, n, rc, stats);
    return rc;
}

// A batch: every (lattice, right-hand side) unit.
static int cg_dispatch_batch(hmc_ctx* c, const double* phi, const double2* b, double2* x, hipStream_t s,
                             const double* pi = nullptr, double eps = 0.0) {
    double* pw = const_cast<double*>(phi);
    if (c->p.precision == HMC_MIXED)
        return drift_solve<float>(c, launch_batch<float>(c), c->nunits, pw, pi, eps, b, x, s);
    return drift_solve<double>(c, launch_batch<double>(c), c->nunits, pw, pi, eps, b, x, s);
}

static void merge_stats(hmc_traj_stats* t, const hmc_cg_stats& cs) {
    t->cg_solves += 1;
    for (int j = 0; j < cs.n; ++j) {
        t->cg_iterations += cs.iterations[j];
        if (cs.true_resid[j] > t->max_true_resid) t->max_true_resid = cs.true_resid[j];
    }
}

// --------------------------------------------------------------------------------------
// site-parallel pieces shared by both modes

// Applies M (DAG false) or M^dagger to every unit; FP64 or FP32 pair kernels.
template <typename R, bool DAG>
static int launch_apply(hmc_ctx* c, const R* phi, const void* in, void* out, int n, hipStream_t s) {
    const bool nn2 = c->cf64.nn2 != 0;
    if constexpr (sizeof(R) == sizeof(double)) {
        if (c->is_batch)
            HMC_LAUNCH_NN2(nn2, (k_apply<double, DAG, GeoBatch, true>), (k_apply<double, DAG, GeoBatch, false>),
                           dim3(c->bi.nblocks[0]), dim3(kBlock), 0, s, geo_batch(c, 0),
                           static_cast<const double2*>(in), static_cast<double2*>(out), phi, c->cf64);
        else
            HMC_LAUNCH_NN2(nn2, (k_apply<double, DAG, GeoOne, true>), (k_apply<double, DAG, GeoOne, false>),
                           dim3(c->nblk * n), dim3(kBlock), 0, s, geo_one(c, c->nblk),
                           static_cast<const double2*>(in), static_cast<double2*>(out), phi, c->cf64);
    } else {
        if (c->is_batch)
            HMC_LAUNCH_NN2(nn2, (k_apply2<DAG, GeoBatch, true>), (k_apply2<DAG, GeoBatch, false>),
                           dim3(c->bi.nblocks[1]), dim3(kBlock), 0, s, geo_batch(c, 1),
                           static_cast<const float2*>(in), static_cast<float2*>(out), phi, c->cf32);
        else
            HMC_LAUNCH_NN2(nn2, (k_apply2<DAG, GeoOne, true>), (k_apply2<DAG, GeoOne, false>),
                           dim3(c->nblk2 * n), dim3(kBlock), 0, s, geo_one(c, c->nblk2),
                           static_cast<const float2*>(in), static_cast<float2*>(out), phi, c->cf32);
    }
    LAUNCHCHK();
    return HMC_OK;
}

static int launch_force(hmc_ctx* c, const double* phi, const double2* x, int npf, int flags,
                        double* force, double* pi, double h, int nkick, hipStream_t s) {
    const int do_pf = (flags & HMC_FORCE_PF) ? 1 : 0, do_b = (flags & HMC_FORCE_BOSON) ? 1 : 0;
    if (c->is_batch)
        HMC_LAUNCH_NN2(c->cf64.nn2, (k_force<CGeoBatch, true>), (k_force<CGeoBatch, false>), dim3(c->ngblk),
                       dim3(kBlock), 0, s, cgeo_batch(c), x, phi, c->cf64, do_pf, do_b, force, pi, h, nkick);
    else
        HMC_LAUNCH_NN2(c->cf64.nn2, (k_force<CGeoOne, true>), (k_force<CGeoOne, false>), dim3(c->nblk),
                       dim3(kBlock), 0, s, cgeo_one(c, npf), x, phi, c->cf64, do_pf, do_b, force, pi, h, nkick);
    LAUNCHCHK();
    return HMC_OK;
}

// sum_k Re<a_k, b_k>: one lattice -> slots[slot_index]; batch -> per lattice, slot_index of
// its block of kChainSlots.
static int dot_re(hmc_ctx* c, const double2* a, const double2* b, int n, int slot_index, hipStream_t s) {
    if (c->is_batch) {
        hipLaunchKernelGGL(k_dot_re<CGeoBatch>, dim3(c->ngblk), dim3(kBlock), 0, s, cgeo_batch(c), a, b, c->gpart);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_sum_chains, dim3(c->bi.nchains), dim3(kBlock), 0, s, c->gpart, 0, 1,
                           c->bi.cfirst_dev, c->bi.cslots + slot_index, kChainSlots);
    } else {
        hipLaunchKernelGGL(k_dot_re<CGeoOne>, dim3(c->nblk), dim3(kBlock), 0, s, cgeo_one(c, n), a, b, c->gpart);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, c->gpart, c->nblk, 1, 0,
                           c->slots + slot_index);
    }
    LAUNCHCHK();
    return HMC_OK;
}

// K = |pi|^2 / 2 (pi may be NULL) and S_B into slots [slot_index, slot_index + 1].
static int energy(hmc_ctx* c, const double* pi, const double* phi, int slot_index, hipStream_t s) {
    if (c->is_batch) {
        hipLaunchKernelGGL(k_energy<CGeoBatch>, dim3(c->ngblk), dim3(kBlock), 0, s, cgeo_batch(c), pi, phi,
                           c->gpart, c->ngblk);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_sum_chains, dim3(c->bi.nchains), dim3(kBlock), 0, s, c->gpart, c->ngblk, 2,
                           c->bi.cfirst_dev, c->bi.cslots + slot_index, kChainSlots);
    } else {
        hipLaunchKernelGGL(k_energy<CGeoOne>, dim3(c->nblk), dim3(kBlock), 0, s, cgeo_one(c, 0), pi, phi,
                           c->gpart, c->nblk);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, c->gpart, c->nblk, 2, c->nblk,
                           c->slots + slot_index);
    }
    LAUNCHCHK();
    return HMC_OK;
}

static int read_slots(hmc_ctx* c, hipStream_t s) {
    if (c->is_batch)
        HIPCHK(hipMemcpyAsync(c->bi.h_cslots, c->bi.cslots, sizeof(double) * kChainSlots * c->bi.nchains,
                              hipMemcpyDeviceToHost, s));
    else
        HIPCHK(hipMemcpyAsync(c->h_slots, c->slots, sizeof(double) * kSlots, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HMC_OK;
}

// The metric passes on one lattice (FP64): forward slice FFT of `in` into the scratch field
// (the FP64 CG vector t, idle outside solves), the tau pass (the reduction `red`, scaled by
// rs, into slots[slot]; the accumulation into acc; the scaling `mul`), and with `mul` the
// inverse slice FFT into out (add: out += h y; else out = y).  in may equal out.
template <int MAXR>
static int metric_passes_r(hmc_ctx* c, const double* in, double* out, int add, double h, int mul, int red,
                           double rs, double* acc, int slot, hipStream_t s, int acc_add) {
    const MetricGeo g{c->lat.L, c->lat.Lt, c->lat.LL, c->lat.vol};
    double2* scr = c->t64;
    const int nslice = 3 * g.Lt, ngrp = 3 * pc_groups(g.LL, pc_ncol<double>());
    hipLaunchKernelGGL((k_mt_xy<false, MAXR>), dim3(nslice), dim3(kPcBlock), c->lds_xy[0], s, g, in, scr,
                       static_cast<double*>(nullptr), 0, 0.0, c->blob);
    LAUNCHCHK();
    hipLaunchKernelGGL((k_mt_t<MAXR>), dim3(ngrp), dim3(kPcBlock), c->lds_mt_t, s, g, scr, c->sigma, mul, red, rs,
                       acc, acc_add, red ? c->mpart : static_cast<double*>(nullptr), c->blob);
    LAUNCHCHK();
    if (red) {
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, c->mpart, ngrp, 1, 0, c->slots + slot);
        LAUNCHCHK();
    }
    if (mul) {
        hipLaunchKernelGGL((k_mt_xy<true, MAXR>), dim3(nslice), dim3(kPcBlock), c->lds_xy[0], s, g,
                           static_cast<const double*>(nullptr), scr, out, add, h, c->blob);
        LAUNCHCHK();
    }
    return HMC_OK;
}

static int metric_passes(hmc_ctx* c, const double* in, double* out, int add, double h, int mul, int red,
                         double rs, double* acc, int slot, hipStream_t s, int acc_add = 1) {
    return c->pc_r7 ? metric_passes_r<7>(c, in, out, add, h, mul, red, rs, acc, slot, s, acc_add)
                    : metric_passes_r<5>(c, in, out, add, h, mul, red, rs, acc, slot, s, acc_add);
}

// The leapfrog drift phi += eps dphi/dt: eps pi (identity metric) or eps Sigma pi.
static int drift(hmc_ctx* c, double* phi, const double* pi, double eps, hipStream_t s) {
    if (c->sigma != nullptr) return metric_passes(c, pi, phi, 1, eps, MUL_SIGMA, RED_NONE, 1.0, nullptr, 0, s);
    hipLaunchKernelGGL(k_drift, dim3(elem_grid(3LL * c->phi_sites)), dim3(kBlock), 0, s, phi, pi, eps,
                       int(3 * c->phi_sites));
    LAUNCHCHK();
    return HMC_OK;
}

// Kinetic energy (1/2 |pi|^2, or 1/2 pi^T Sigma pi with the metric) and S_B into slots
// [slot_index, slot_index + 1].
static int energies(hmc_ctx* c, const double* pi, const double* phi, int slot_index, hipStream_t s) {
    if (c->sigma == nullptr) return energy(c, pi, phi, slot_index, s);
    int rc = energy(c, nullptr, phi, slot_index, s);
    if (rc) return rc;
    return metric_passes(c, pi, nullptr, 0, 0.0, 0, RED_SIGMA, 0.5, nullptr, slot_index, s);
}

// Leapfrog (kick-drift-kick) on (phi, pi) with pseudofermions chi fixed: n_leap steps of eps,
// one CG solve per step plus the one at the start, the two half kicks of neighbouring steps
// applied separately inside the gradient kernel.  Leaves sum_k Re<chi_k, x_k> of the last
// solve in slot SL_SPF1 and, if first_action, that of the first solve in SL_SPF0.
static int md_integrate(hmc_ctx* c, double* phi, double* pi, const double2* chi, int n_pf,
                        bool first_action, hmc_traj_stats* stats, hipStream_t s) {
    const double eps = c->p.eps, h = 0.5 * eps;
    const int nl = c->p.n_leap;
    const int flags = HMC_FORCE_BOSON | (n_pf > 0 ? HMC_FORCE_PF : 0);
    // with dpi: the drift phi += eps dpi, then the solve
    auto solve = [&](const double* dpi) -> int {
        if (n_pf == 0) return dpi ? drift(c, phi, dpi, eps, s) : HMC_OK;
        if (c->is_batch) {
            const int r = cg_dispatch_batch(c, phi, chi, c->xsol, s, dpi, eps);
            if (r == HMC_OK || r == HMC_ERR_NOT_CONVERGED || r == HMC_ERR_NONFINITE) {
                stats->cg_solves += 1;
                for (int j = 0; j < c->nunits; ++j) {
                    stats->cg_iterations += c->h_st[j].iters;
                    const double tr = true_resid_of(c->h_st[j]);
                    if (tr > stats->max_true_resid) stats->max_true_resid = tr;
                }
            }
            return r;
        }
        hmc_cg_stats cs;
        const int r = cg_dispatch(c, phi, chi, c->xsol, n_pf, &cs, s, dpi, eps);
        if (r == HMC_OK || r == HMC_ERR_NOT_CONVERGED || r == HMC_ERR_NONFINITE) merge_stats(stats, cs);
        return r;
    };
    int rc = solve(nullptr);
    if (rc) return rc;
    if (first_action && n_pf > 0) {
        rc = dot_re(c, chi, c->xsol, n_pf, SL_SPF0, s);
        if (rc) return rc;
    }
    // first half kick with the force at the start
    rc = launch_force(c, phi, c->xsol, n_pf, flags, nullptr, pi, h, nl > 0 ? 1 : 0, s);
    if (rc) return rc;
    for (int step = 0; step < nl; ++step) {
        rc = solve(pi);
        if (rc) return rc;
        // closing half kick of this step, then the opening half kick of the next one
        rc = launch_force(c, phi, c->xsol, n_pf, flags, nullptr, pi, h, step + 1 < nl ? 2 : 1, s);
        if (rc) return rc;
    }
    if (n_pf > 0) {
        rc = dot_re(c, chi, c->xsol, n_pf, SL_SPF1, s);
        if (rc) return rc;
    }
    return HMC_OK;
}

static void fill_energies(const double* hs, int n_pf, hmc_traj_stats* stats) {
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

// Preconditioner support and sizes for the lattices of the context: FFT plans for L and L_tau,
// dynamic LDS of the three passes per precision against the device's per-workgroup limit,
// table offsets; batch: the workgroup counts of the slice and tau passes.
static void pc_setup(hmc_ctx* c) {
    int maxlds = 0;
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
        maxlds = 0;
    std::vector<Lat> lats;
    if (c->is_batch) lats = c->bi.lats;
    else lats.push_back(c->lat);
    bool plans = true;
    long long blob = 0;
    c->pc_r7 = false;
    c->bi.pcoff.assign(1, 0);
    c->bi.nslices = 0;
    c->bi.ngroups[0] = c->bi.ngroups[1] = 0;
    for (int pi = 0; pi < 2; ++pi) c->lds_xy[pi] = c->lds_t[pi] = 0, c->pc_q[pi] = 0, c->pc_full[pi] = false;
    for (const Lat& l : lats) {
        FftPlan pa, pb;
        const bool ok = make_fft_plan(l.L, pa) && make_fft_plan(l.Lt, pb);
        plans = plans && ok;
        if (ok) c->pc_r7 = c->pc_r7 || fft_max_radix(pa) == 7 || fft_max_radix(pb) == 7;
        blob += pc_blob_layout(l.L, l.Lt).size;
        c->bi.pcoff.push_back(blob);
        const int nrhs = c->is_batch ? c->bi.nrhs : 1;
        c->bi.nslices += 4 * l.Lt * nrhs;
        c->bi.ngroups[0] += 4 * pc_groups(l.LL, kPcCols) * nrhs;
        c->bi.ngroups[1] += 4 * pc_groups(l.LL, kPcCols) * nrhs;
        const size_t c64 = sizeof(double2), c32 = sizeof(float2);
        c->lds_xy[0] = std::max(c->lds_xy[0], size_t(l.LL + l.L) * c64);
        c->lds_xy[1] = std::max(c->lds_xy[1], size_t(l.LL + l.L) * c32);
        const int q64 = pc_chunks<double>(l.Lt), q32 = pc_chunks<float>(l.Lt);
        c->pc_q[0] = (q64 == 0 || c->pc_q[0] < 0) ? -1 : std::max(c->pc_q[0], q64);
        c->pc_q[1] = (q32 == 0 || c->pc_q[1] < 0) ? -1 : std::max(c->pc_q[1], q32);
    }
    c->blob_doubles = blob;
    c->pc_full[0] = c->pc_q[0] > 0;
    c->pc_full[1] = c->pc_q[1] > 0;
    for (const Lat& l : lats) {
        c->pc_full[0] = c->pc_full[0] && l.Lt == c->pc_q[0] * pc_chunk_max<double>();
        c->pc_full[1] = c->pc_full[1] && l.Lt == c->pc_q[1] * pc_chunk_max<float>();
    }
    c->lds_t[0] = c->pc_q[0] > 0 ? pc_tau_lds<double>(c->pc_q[0]) : 0;
    c->lds_t[1] = c->pc_q[1] > 0 ? pc_tau_lds<float>(c->pc_q[1]) : 0;
    for (int pi = 0; pi < 2; ++pi)
        c->pc_ok[pi] = plans && c->pc_q[pi] > 0 && c->lds_xy[pi] <= size_t(maxlds) &&
                       c->lds_t[pi] <= size_t(maxlds);
    if (!c->is_batch) {
        const Lat& l = c->lat;
        c->lds_mt_t = size_t(l.Lt) * (pc_ncol<double>() + 1) * sizeof(double2) + size_t(l.Lt + l.L) * sizeof(int);
        c->metric_ok = plans && c->lds_xy[0] <= size_t(maxlds) && c->lds_mt_t <= size_t(maxlds);
    }
}

static int check_precond(const hmc_ctx* c, const hmc_params* p) {
    if (p->precond == HMC_PRECOND_FOURIER && !c->pc_ok[p->precision == HMC_MIXED ? 1 : 0])
        return fail(HMC_ERR_INVALID_ARG,
                    "Fourier preconditioner unavailable for this lattice and precision (L and L_tau need "
                    "prime factors <= 7, and an L x L slice must fit the GPU's LDS)");
    return HMC_OK;
}

// Allow the preconditioner passes their dynamic LDS (above the default per-workgroup amount).
template <typename R, class Geo, int MAXR>
static void pc_lds_attributes_r(size_t xy, size_t t) {
    const hipFuncAttribute a = hipFuncAttributeMaxDynamicSharedMemorySize;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pc_xy<R, false, Geo, MAXR>), a, int(xy));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pc_xy<R, true, Geo, MAXR>), a, int(xy));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pc_t<R, Geo, false>), a, int(t));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pc_t<R, Geo, true>), a, int(t));
}

template <class Geo>
static void pc_lds_attributes(const hmc_ctx* c) {
    if (c->pc_ok[0]) {
        if (c->pc_r7) pc_lds_attributes_r<double, Geo, 7>(c->lds_xy[0], c->lds_t[0]);
        else pc_lds_attributes_r<double, Geo, 5>(c->lds_xy[0], c->lds_t[0]);
    }
    if (c->pc_ok[1]) {
        if (c->pc_r7) pc_lds_attributes_r<float, Geo, 7>(c->lds_xy[1], c->lds_t[1]);
        else pc_lds_attributes_r<float, Geo, 5>(c->lds_xy[1], c->lds_t[1]);
    }
    (void)hipGetLastError();
}

// Preconditioner tables of every lattice into the workspace; batch: the pass block tables.
static int upload_pc(hmc_ctx* c) {
    std::vector<Lat> lats;
    if (c->is_batch) lats = c->bi.lats;
    else lats.push_back(c->lat);
    std::vector<double> all;
    for (const Lat& l : lats) {
        FftPlan pa, pb;
        if (!make_fft_plan(l.L, pa) || !make_fft_plan(l.Lt, pb)) return HMC_OK;   // unsupported: no tables
        const std::vector<double> b = pc_table_blob(pa, pb);
        all.insert(all.end(), b.begin(), b.end());
    }
    if (!all.empty()) HIPCHK(hipMemcpy(c->blob, all.data(), sizeof(double) * all.size(), hipMemcpyHostToDevice));
    if (c->is_batch) {
        BatchInfo& b = c->bi;
        std::vector<int2> xy, t[2];
        for (int ch = 0; ch < b.nchains; ++ch) {
            const Lat& l = b.lats[size_t(ch)];
            for (int k = 0; k < b.nrhs; ++k) {
                const int u = ch * b.nrhs + k;
                for (int r = 0; r < 4 * l.Lt; ++r) xy.push_back(make_int2(u, r));
                for (int r = 0; r < 4 * pc_groups(l.LL, kPcCols); ++r) t[0].push_back(make_int2(u, r));
                for (int r = 0; r < 4 * pc_groups(l.LL, kPcCols); ++r) t[1].push_back(make_int2(u, r));
            }
        }
        HIPCHK(hipMemcpy(b.pxy_blocks, xy.data(), sizeof(int2) * xy.size(), hipMemcpyHostToDevice));
        for (int pi = 0; pi < 2; ++pi)
            HIPCHK(hipMemcpy(b.pt_blocks[pi], t[pi].data(), sizeof(int2) * t[pi].size(), hipMemcpyHostToDevice));
        pc_lds_attributes<GeoBatch>(c);
    } else {
        pc_lds_attributes<GeoOne>(c);
        if (c->metric_ok) {
            const hipFuncAttribute a = hipFuncAttributeMaxDynamicSharedMemorySize;
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mt_xy<false, 5>), a, int(c->lds_xy[0]));
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mt_xy<true, 5>), a, int(c->lds_xy[0]));
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mt_t<5>), a, int(c->lds_mt_t));
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mt_xy<false, 7>), a, int(c->lds_xy[0]));
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mt_xy<true, 7>), a, int(c->lds_xy[0]));
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mt_t<7>), a, int(c->lds_mt_t));
            (void)hipGetLastError();
        }
    }
    return HMC_OK;
}

// The device address of `scratch` on `device` (current), resolved once per device.  Returns
// null, with the failure left in hmc_last_error, if the runtime cannot resolve it.
static void* scratch_for_device(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) return it->second;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(HMC_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    g_scratch_addr[device] = p;
    return p;
}

static int create_common(hmc_ctx* c) {
    if (hipGetDevice(&c->device) != hipSuccess) return fail(HMC_ERR_HIP, "hipGetDevice failed");
    c->scratch = scratch_for_device(c->device);
    if (hipHostMalloc((void**)&c->h_st, sizeof(CgState) * 2 * size_t(c->nunits), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_slots, sizeof(double) * kSlots, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) != hipSuccess)
        return fail(HMC_ERR_HIP, "pinned status buffer or event creation failed");
    if (c->is_batch &&
        hipHostMalloc((void**)&c->bi.h_cslots, sizeof(double) * kChainSlots * size_t(c->bi.nchains),
                      hipHostMallocDefault) != hipSuccess)
        return fail(HMC_ERR_HIP, "pinned status buffer creation failed");
    return HMC_OK;
}

static void destroy_common(hmc_ctx* c) {
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < hmc_ctx::kEv; ++j)
            if (c->tev[i][j]) (void)hipEventDestroy(c->tev[i][j]);
    for (int p = 0; p < 2; ++p)
        for (int g = 0; g < 2; ++g)
            if (c->cgg[p].exec[g]) (void)hipGraphExecDestroy(c->cgg[p].exec[g]);
    for (auto& g : c->sgs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    c->sgs.clear();
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->h_st) (void)hipHostFree(c->h_st);
    if (c->h_slots) (void)hipHostFree(c->h_slots);
    if (c->bi.h_cslots) (void)hipHostFree(c->bi.h_cslots);
    for (int i = 0; i < 2; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
}

// Batch: per-lattice descriptors of the site-parallel kernels (geometry, offsets, boson
// coefficients with the lattice's own r) and the tile prefix of the per-lattice sums.
static int upload_chains(hmc_ctx* c) {
    BatchInfo& b = c->bi;
    HIPCHK(hipDeviceSynchronize());     // launches already queued may still read the tables
    std::vector<ChainDesc> chains(size_t(b.nchains));
    std::vector<int2> cblocks;
    for (int ch = 0; ch < b.nchains; ++ch) {
        ChainDesc& d = chains[size_t(ch)];
        d.lat = b.lats[size_t(ch)];
        d.voff = b.sp_off[size_t(ch)];
        d.phioff = b.phi_off[size_t(ch)];
        d.bc = boson_coef_of(c->dtau, c->p.c, b.r[size_t(ch)], c->p.u);
        d.npf = b.nrhs;
        d.pad = 0;
        for (int t = 0; t < tiles1_host(d.lat.vol); ++t) cblocks.push_back(make_int2(ch, t));
    }
    HIPCHK(hipMemcpy(b.chains, chains.data(), sizeof(ChainDesc) * chains.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b.cblocks, cblocks.data(), sizeof(int2) * cblocks.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b.cfirst_dev, b.cfirst.data(), sizeof(int) * b.cfirst.size(), hipMemcpyHostToDevice));
    return HMC_OK;
}

static int set_workspace_common(hmc_ctx* c, void* ptr, size_t bytes) {
    if (c == nullptr || ptr == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL handle or workspace");
    if ((reinterpret_cast<uintptr_t>(ptr) & 255u) != 0) return fail(HMC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (bytes < c->need) return fail(HMC_ERR_WORKSPACE, "workspace of %zu bytes < %zu needed", bytes, c->need);
    char* base = static_cast<char*>(ptr);
    (void)ws_layout(c, base);
    c->ws = base;
    c->ws_bytes = bytes;
    c->generation += 1;
    {
        int rc = upload_pc(c);
        if (rc) return rc;
    }
    if (c->is_batch) {
        int rc = upload_chains(c);
        if (rc) return rc;
        rc = set_cg_shape(c, HMC_FP64, c->bpr64);
        if (rc) return rc;
        rc = set_cg_shape(c, HMC_MIXED, c->bpr32);
        if (rc) return rc;
    }
    return HMC_OK;
}

// Launch shapes of a tuning choice (clamped as the setters clamp them).
static void apply_choice(hmc_ctx* c, const TuneChoice& ch) {
    c->bpr64 = c->is_batch ? ch.bpr[0] : clamp_bpr(c->nblk2, ch.bpr[0]);
    c->bpr32 = c->is_batch ? ch.bpr[1] : clamp_bpr(c->nblk2, ch.bpr[1]);
    for (int pi = 0; pi < 2; ++pi) {
        c->cgm_rows[pi] = ch.mrows[pi];
        c->cgm_seg[pi] = ch.mseg[pi];
        c->cgb_march[pi] = ch.mb[pi];
    }
    c->generation += 1;
}

static TuneChoice current_choice(const hmc_ctx* c) {
    TuneChoice ch;
    ch.bpr[0] = c->bpr64;
    ch.bpr[1] = c->bpr32;
    for (int pi = 0; pi < 2; ++pi) {
        ch.mrows[pi] = c->cgm_rows[pi];
        ch.mseg[pi] = c->cgm_seg[pi];
        ch.mb[pi] = c->cgb_march[pi];
    }
    return ch;
}

// Autotuner core: time `iters` CG iterations per candidate shape and keep the fastest.
static int autotune_common(hmc_ctx* c, const double* phi, const double2* b, int n, hmc_tune_result* out,
                           hipStream_t s) {
    static const int cand[HMC_TUNE_MAX] = {128, 256, 384, 512, 640, 768, 1024, 1280, 1536, 2048, 3072, 4096};
    const hmc_params saved = c->p;
    const int iters = 100;
    std::memset(out, 0, sizeof(*out));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int result = HMC_OK;
    int maxt = c->nblk2;
    if (c->is_batch)
        for (const Lat& l : c->bi.lats) maxt = std::max(maxt, tiles2_host(l.vol));
    for (int pi = 0; pi < 2 && result == HMC_OK; ++pi) {
        const int prec = pi == 0 ? HMC_FP64 : HMC_MIXED;
        c->p.precision = prec;
        c->p.cg_tol = 1e-30;           // never converges: every candidate runs `iters` iterations
        c->p.cg_maxit = iters;
        if (prec == HMC_MIXED && c->p.reliable_every < 1) c->p.reliable_every = 50;
        double best = 1e300;
        int best_bpr = 0, last = -1;
        // the workgroup count is tuned on the tile kernels, then the march shapes with it
        c->cgm_rows[pi] = 0;
        c->generation += 1;
        for (int cb : cand) {
            const int bpr = clamp_bpr(maxt, cb);
            if (bpr == last) continue;
            last = bpr;
            result = set_cg_shape(c, prec, bpr);
            if (result) break;
            float ms = 0.f;
            for (int rep = 0; rep < 2; ++rep) {    // first run warms caches, code and graphs
                if (hipEventRecord(e0, s) != hipSuccess) { result = HMC_ERR_HIP; break; }
                const int r = c->is_batch ? cg_dispatch_batch(c, phi, b, c->xsol, s)
                                          : cg_dispatch(c, phi, b, c->xsol, n, nullptr, s);
                if (r != HMC_OK && r != HMC_ERR_NOT_CONVERGED) { result = r; break; }
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { result = HMC_ERR_HIP; break; }
            }
            if (result != HMC_OK) break;
            out->candidates += 1;
            const double us = 1e3 * ms / iters;
            out->tried_workgroups[pi][out->tried[pi]] = bpr;
            out->tried_us[pi][out->tried[pi]] = us;
            out->tried[pi] += 1;
            if (us < best) { best = us; best_bpr = bpr; }
        }
        if (result == HMC_OK) {
            result = set_cg_shape(c, prec, best_bpr);
            out->cg_workgroups[pi] = best_bpr;
            out->us_per_iter[pi] = best;
        }
        // step A as a march (nearest neighbours): rows per band x slices per segment; in a
        // batch the rows are a cap, each lattice taking at most what its band allows
        if (result == HMC_OK && !(c->is_batch && c->cf64.nn2)) {
            static const int rows32[] = {4, 6, 8, 10}, rows64[] = {2, 3, 4};
            static const int segs32[] = {4, 6, 8}, segs64[] = {4, 6, 8, 12};
            static const int brows32[] = {4, 8, 12, 16}, bsegs[] = {4, 8};
            const int per_row = pi ? c->L / 2 : c->L;
            int best_r = 0, best_s = 0;
            const int* rows = c->is_batch ? (pi ? brows32 : rows64) : (pi ? rows32 : rows64);
            const int* segs = c->is_batch ? bsegs : (pi ? segs32 : segs64);
            const int nr = pi ? 4 : 3, ns = c->is_batch ? 2 : (pi ? 3 : 4);
            // in a batch the FP32 shape's reliable-update cut follows the FP64 rows
            auto apply_march = [&](int r, int sl) -> int {
                c->cgm_rows[pi] = r;
                c->cgm_seg[pi] = sl;
                c->generation += 1;
                if (!c->is_batch) return HMC_OK;
                int rc = upload_batch_shape(c, pi, pi ? c->bpr32 : c->bpr64);
                if (rc == HMC_OK && pi == 0) rc = upload_batch_shape(c, 1, c->bpr32);
                return rc;
            };
            for (int a = 0; a < nr && result == HMC_OK; ++a) {
                if (!c->is_batch && ((rows[a] + (c->cf64.nn2 ? 4 : 2)) * per_row > kMarchCgThreads || rows[a] > c->L))
                    continue;
                for (int q = 0; q < ns && result == HMC_OK; ++q) {
                    if (out->mtried[pi] >= HMC_TUNE_MARCH_MAX) break;
                    result = apply_march(rows[a], segs[q]);
                    if (result) break;
                    if (c->is_batch && c->bi.mgrid[pi] == 0) continue;     // no lattice of the batch marches
                    float ms = 0.f;
                    for (int rep = 0; rep < 2; ++rep) {
                        if (hipEventRecord(e0, s) != hipSuccess) { result = HMC_ERR_HIP; break; }
                        const int r = c->is_batch ? cg_dispatch_batch(c, phi, b, c->xsol, s)
                                                  : cg_dispatch(c, phi, b, c->xsol, n, nullptr, s);
                        if (r != HMC_OK && r != HMC_ERR_NOT_CONVERGED) { result = r; break; }
                        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { result = HMC_ERR_HIP; break; }
                    }
                    if (result != HMC_OK) break;
                    out->candidates += 1;
                    const double us = 1e3 * ms / iters;
                    const int j = out->mtried[pi]++;
                    out->mtried_rows[pi][j] = rows[a];
                    out->mtried_slices[pi][j] = segs[q];
                    out->mtried_us[pi][j] = us;
                    if (us < best) {
                        best = us;
                        best_r = rows[a];
                        best_s = segs[q];
                    }
                }
            }
            if (result == HMC_OK) result = apply_march(best_r, best_s);
            // step B as a march too, or the tile kernel, with the chosen cut
            if (result == HMC_OK && best_r > 0 && (!c->is_batch || c->bi.mgrid[pi] > 0)) {
                double tb[2] = {1e300, 1e300};
                for (int mb = 0; mb < 2 && result == HMC_OK; ++mb) {
                    c->cgb_march[pi] = mb;
                    c->generation += 1;
                    float ms = 0.f;
                    for (int rep = 0; rep < 2; ++rep) {
                        if (hipEventRecord(e0, s) != hipSuccess) { result = HMC_ERR_HIP; break; }
                        const int r = c->is_batch ? cg_dispatch_batch(c, phi, b, c->xsol, s)
                                                  : cg_dispatch(c, phi, b, c->xsol, n, nullptr, s);
                        if (r != HMC_OK && r != HMC_ERR_NOT_CONVERGED) { result = r; break; }
                        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { result = HMC_ERR_HIP; break; }
                    }
                    if (result != HMC_OK) break;
                    out->candidates += 1;
                    tb[mb] = 1e3 * ms / iters;
                    out->step_b_us[pi][mb] = tb[mb];
                }
                c->cgb_march[pi] = tb[1] < tb[0] ? 1 : 0;
                c->generation += 1;
                best = std::min(best, std::min(tb[0], tb[1]));
            }
            out->march_step_b[pi] = c->cgb_march[pi];
            out->march_rows[pi] = best_r;
            out->march_slices[pi] = best_s;
            out->us_per_iter[pi] = best;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->p = saved;
    if (result != HMC_OK) {
        c->cgm_rows[0] = 4;
        c->cgm_rows[1] = 8;
        c->cgm_seg[0] = c->cgm_seg[1] = 8;
        c->cgb_march[0] = 1;
        c->cgb_march[1] = 1;
        (void)set_cg_shape(c, HMC_FP64, kDefaultBpr64);
        (void)set_cg_shape(c, HMC_MIXED, kDefaultBpr32);
        return result == HMC_ERR_HIP ? fail(result, "autotune: HIP call failed") : result;
    }
    return HMC_OK;
}

// A cached choice as the tuner's result (nothing timed).
static void choice_result(const TuneChoice& ch, hmc_tune_result* out) {
    std::memset(out, 0, sizeof(*out));
    for (int pi = 0; pi < 2; ++pi) {
        out->cg_workgroups[pi] = ch.bpr[pi];
        out->march_rows[pi] = ch.mrows[pi];
        out->march_slices[pi] = ch.mseg[pi];
        out->march_step_b[pi] = ch.mb[pi];
    }
    out->from_cache = 1;
}

static bool reuse_cached() {
    const char* e = std::getenv("HMC_TUNE_REUSE");
    return e != nullptr && std::strcmp(e, "1") == 0;
}

static int check_solve_args(hmc_ctx* c, const void* phi, const void* b, const void* x, int n) {
    if (c == nullptr || phi == nullptr || b == nullptr || x == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    int rc = need_ws(c);
    if (rc) return rc;
    if (n < 1 || n > c->cap) return fail(HMC_ERR_INVALID_ARG, "n = %d outside [1, %d]", n, c->cap);
    if (!aligned16(phi) || !aligned16(b) || !aligned16(x)) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    if (b == x) return fail(HMC_ERR_INVALID_ARG, "b and x must not alias");
    return HMC_OK;
}

template <typename R, bool DAG>
static int apply_impl(hmc_ctx* c, const R* phi, const void* in, void* out, int n, void* stream) {
    if (c == nullptr || phi == nullptr || in == nullptr || out == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if (n < 1) return fail(HMC_ERR_INVALID_ARG, "n must be >= 1");
    if (!aligned16(phi) || !aligned16(in) || !aligned16(out)) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    if (in == out) return fail(HMC_ERR_INVALID_ARG, "in and out must not overlap");
    if ((long long)c->nblk * n >= (1LL << 31)) return fail(HMC_ERR_INVALID_ARG, "too many vectors");
    return launch_apply<R, DAG>(c, phi, in, out, n, (hipStream_t)stream);
}

// Launch shape of the fused M^dagger M for n vectors: rows per band, slices per segment (1: one
// workgroup per slice and band, k_mdm*_tile, whose chi rows fit 64 KB of LDS; more: the march,
// k_mdm*_march), threads (one per element of the rows a workgroup holds, at most 512).  The
// shape does not depend on n.
struct MdmShape {
    MarchPlan plan;
    int threads;
    size_t lds;
    bool tile;   // one slice per workgroup (k_mdm*_tile), else the march (k_mdm*_march)
};
template <typename R>
static MdmShape mdm_shape(const hmc_ctx* c, int n) {
    const int pi = sizeof(R) == sizeof(float) ? 1 : 0;
    const int L = c->L, Lt = c->Lt, per_row = pi ? L / 2 : L;
    // defaults: the fastest shapes at 80 x 80 x 200 (the march: 8 rows FP32, 4 rows FP64, 8 slices)
    int rows = c->mdm_rows[pi] > 0 ? c->mdm_rows[pi] : (pi ? 8 : 4);
    const int rows_lds = int((size_t(64) << 10) / (4 * size_t(L) * sizeof(C2<R>))) - 2;
    rows = std::max(1, std::min({rows, rows_lds, 4 * kMarchMaxThreads / per_row}));
    const int seg = c->mdm_seg[pi] > 0 ? c->mdm_seg[pi] : 8;
    (void)n;
    MdmShape m;
    m.tile = seg == 1;
    if (m.tile) {
        rows = std::max(1, std::min(rows, kMarchMaxThreads / per_row));
        m.plan = make_march_plan(L, Lt, rows, seg);
        // one element of the band per thread, and the rows beside it on the first 2 rows' worth
        m.threads = (std::max(m.plan.R * per_row, 2 * per_row) + 63) / 64 * 64;
        m.lds = march_lds<R>(m.plan.R, L);
    } else {
        // the march: one thread per element of the band and of the two rows on either side;
        // psi and chi of two slices each in LDS (at most 160 KB)
        const int rows_lds = int((size_t(160) << 10) / (4 * size_t(L) * sizeof(C2<R>)) - 12) / 4;
        rows = std::max(1, std::min({rows, kMdmMarchThreads / per_row - 4, rows_lds}));
        m.plan = make_march_plan(L, Lt, rows, seg);
        m.threads = ((std::min(rows, L) + 4) * per_row + 63) / 64 * 64;
        m.lds = mdm_march_lds<R>(m.plan.R, L);
    }
    return m;
}

// out = M^dagger M in, one pass (nearest-neighbour operator, one lattice).
template <typename R>
static int launch_mdm(hmc_ctx* c, const R* phi, const void* in, void* out, int n, hipStream_t s) {
    const MdmShape m = mdm_shape<R>(c, n);
    const long long grid = (long long)n * m.plan.nband * m.plan.nseg;
    if (grid >= (1LL << 31)) return fail(HMC_ERR_INVALID_ARG, "too many vectors");
    if (m.threads > (m.tile ? kMarchMaxThreads : kMdmMarchThreads) || m.lds > (size_t(160) << 10))
        return fail(HMC_ERR_INVALID_ARG, "one-pass M^dagger M: no launch shape fits this lattice");
    const bool narrow = m.threads <= kMarchMaxThreads, mid = m.threads <= kMdmMidThreads;
    if constexpr (sizeof(R) == sizeof(float)) {
        const float2* a = static_cast<const float2*>(in);
        float2* b = static_cast<float2*>(out);
        if (m.tile)
            hipLaunchKernelGGL(k_mdm2_tile, dim3(int(grid)), dim3(m.threads), m.lds, s, c->lat, m.plan, a, b, phi,
                               c->cf32);
        else if (narrow)
            hipLaunchKernelGGL(k_mdm2_march<kMarchMaxThreads>, dim3(int(grid)), dim3(m.threads), m.lds, s, c->lat,
                               m.plan, a, b, phi, c->cf32);
        else if (mid)
            hipLaunchKernelGGL(k_mdm2_march<kMdmMidThreads>, dim3(int(grid)), dim3(m.threads), m.lds, s, c->lat,
                               m.plan, a, b, phi, c->cf32);
        else
            hipLaunchKernelGGL(k_mdm2_march<kMdmMarchThreads>, dim3(int(grid)), dim3(m.threads), m.lds, s, c->lat,
                               m.plan, a, b, phi, c->cf32);
    } else {
        const double2* a = static_cast<const double2*>(in);
        double2* b = static_cast<double2*>(out);
        if (m.tile)
            hipLaunchKernelGGL(k_mdm_tile, dim3(int(grid)), dim3(m.threads), m.lds, s, c->lat, m.plan, a, b, phi,
                               c->cf64);
        else if (narrow)
            hipLaunchKernelGGL(k_mdm_march<kMarchMaxThreads>, dim3(int(grid)), dim3(m.threads), m.lds, s, c->lat,
                               m.plan, a, b, phi, c->cf64);
        else if (mid)
            hipLaunchKernelGGL(k_mdm_march<kMdmMidThreads>, dim3(int(grid)), dim3(m.threads), m.lds, s, c->lat,
                               m.plan, a, b, phi, c->cf64);
        else
            hipLaunchKernelGGL(k_mdm_march<kMdmMarchThreads>, dim3(int(grid)), dim3(m.threads), m.lds, s, c->lat,
                               m.plan, a, b, phi, c->cf64);
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
    if (!c->cf64.nn2) {
        // one pass: M^dagger (M in) with M in held on chip
        if (phi == nullptr || in == nullptr || out == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
        if (!aligned16(phi) || !aligned16(in) || !aligned16(out))
            return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
        if (in == out) return fail(HMC_ERR_INVALID_ARG, "in and out must not overlap");
        return launch_mdm<R>(c, phi, in, out, n, (hipStream_t)stream);
    }
    // the two-site hops: two passes through the workspace
    void* tmp;
    if constexpr (sizeof(R) == sizeof(double)) tmp = c->t64; else tmp = c->t32;
    if (tmp == in || tmp == out) return fail(HMC_ERR_INVALID_ARG, "in/out alias the workspace");
    rc = apply_impl<R, false>(c, phi, in, tmp, n, stream);
    if (rc) return rc;
    return apply_impl<R, true>(c, phi, tmp, out, n, stream);
}

static int check_batch(hmc_batch* hb, std::initializer_list<const void*> ptrs) {
    if (hb == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL batch");
    for (const void* p : ptrs) {
        if (p == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
        if (!aligned16(p)) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    }
    return need_ws(&hb->c);
}

// One application z = P r of the Fourier preconditioner on the GPU, through the same launches
// a preconditioned solve makes: the CG start (r = b, |b|^2), then the three passes; the last
// reduces the <r, z> partials of the second into the state records.
template <typename R>
static int apply_precond_impl(hmc_ctx* c, const double2* in, void* out, int n, double* rz, hipStream_t s) {
    Launch<GeoOne> lc = launch_one<R>(c, n);
    lc.pc = true;
    CgVecs<R> v = KrylovBufs<R>::get(c, c->xsol, true);
    const size_t bytes = size_t(n) * 4 * size_t(c->vol) * sizeof(C2<R>);
    HIPCHK(hipMemsetAsync(v.z, 0, bytes, s));   // P 0 = 0: a zero input leaves z untouched
    c->seq = 0;
    c->next_nparts = 0;
    hipLaunchKernelGGL((k_cg_init<R, GeoOne>), dim3(lc.ncg), dim3(kBlock), 0, s, next_ctl(c, PEND_NONE), lc.cg,
                       in, c->xsol, v, 0.0, 0.0, 1, 1);
    LAUNCHCHK();
    int rc = enqueue_pc<R, GeoOne>(c, lc, v, PEND_BB, s);   // the last pass consumes <r, z>
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(out, v.z, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(c->h_st, current_states(c), sizeof(CgState) * size_t(n), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int j = 0; j < n; ++j) {
        if (c->h_st[j].mode == CG_FAILED) return fail(HMC_ERR_NONFINITE, "preconditioner met a non-finite value");
        if (rz) rz[j] = c->h_st[j].mode == CG_DONE ? 0.0 : c->h_st[j].rz;
    }
    return HMC_OK;
}

// --------------------------------------------------------------------------------------
// C ABI: one lattice

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

int hmc_test_fft(int n, int inverse, const double* in, double* out) {
    FftPlan pl;
    if (in == nullptr || out == nullptr || !make_fft_plan(n, pl)) return -1;
    std::vector<double2> buf(static_cast<size_t>(n)), tw(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
        buf[size_t(i)] = make_double2(in[2 * i], in[2 * i + 1]);
        tw[size_t(i)] = twiddle_host(i, n);
    }
    if (inverse) fft_lines<double, true>(ExHost(), buf.data(), 1, n, 1, pl, tw.data());
    else fft_lines<double, false>(ExHost(), buf.data(), 1, n, 1, pl, tw.data());
    for (int i = 0; i < n; ++i) {
        out[2 * i] = buf[size_t(i)].x;
        out[2 * i + 1] = buf[size_t(i)].y;
    }
    return 0;
}

int hmc_test_fft_freq(int n, int pos) {
    FftPlan pl;
    if (!make_fft_plan(n, pl) || pos < 0 || pos >= n) return -1;
    return fft_freq(pl, pos);
}

int hmc_test_precond(int L, int Lt, double dtau, const hmc_params* params, const double* in, double* out,
                     double* rz) {
    FftPlan pl, pt;
    constexpr int MC = pc_chunk_max<double>();
    const int Q = pc_chunks<double>(Lt);
    if (params == nullptr || in == nullptr || out == nullptr || !geometry_ok(L, Lt) ||
        !make_fft_plan(L, pl) || !make_fft_plan(Lt, pt) || Q == 0)
        return -1;
    const Coef<double> cf = coef64_of(dtau, *params);
    const int LL = L * L, vol = Lt * LL;
    std::vector<double2> w(size_t(4) * vol);
    for (size_t i = 0; i < w.size(); ++i) w[i] = make_double2(in[2 * i], in[2 * i + 1]);
    const std::vector<double> blob = pc_table_blob(pl, pt);
    const PcBlob bl = pc_blob_layout(L, Lt);
    const double2* twl = reinterpret_cast<const double2*>(blob.data() + bl.twl);
    const ExHost ex;
    std::vector<double2> sbuf(static_cast<size_t>(LL));   // the kernels' LDS copy of a slice
    for (int sl = 0; sl < 4 * Lt; ++sl) {
        double2* slice = w.data() + size_t(sl) * LL;
        fft_slice_io<double, false>(ex, slice, sbuf.data(), slice, pl, twl);
    }
    // the tau pass as the kernel runs it: Q chunks per column, each reduced to an affine map,
    // the maps closed around the cycle, the chunks rerun from their entering values
    double acc = 0.0;
    for (int c = 0; c < 4; ++c) {
        for (int col = 0; col < LL; ++col) {
            const double b = pc_column_b(col, L, c >> 1, blob.data() + bl.cosx, cf);
            const RecCoef<double> k = rec_coef(b);
            constexpr int QM = pc_max_chunks<double>();
            double2 ch[QM][MC], sc[QM], sx[QM + 1];
            double sa[QM];
            ChunkSpan sp[QM];
            const bool rev = !k.before;   // chunks held in the order K^{-1} walks them
            auto at = [&](int q, int j) {
                return size_t(c) * vol + size_t(sp[q].t0 + (rev ? sp[q].n - 1 - j : j)) * LL + col;
            };
            for (int q = 0; q < Q; ++q) {
                sp[q] = pc_chunk_span<double>(q, Lt);
                for (int j = 0; j < MC; ++j) ch[q][j] = j < sp[q].n ? w[at(q, j)] : make_double2(0.0, 0.0);
            }
            auto wk = [&](int q) { return sp[q].n > 0 && sp[q].t0 + sp[q].n == Lt; };
            auto wkd = [&](int q) { return sp[q].n > 0 && sp[q].t0 == 0; };
            for (int q = 0; q < Q; ++q) {
                chunk_scale<double, MC>(ch[q], k.B);
                chunk_map<double, MC, true>(ch[q], sp[q].n, k, sa[q], sc[q]);
                wrap_map<double>(wk(q), k.before, sa[q], sc[q]);
            }
            chunk_close<double>(sa, sc, sx, Q, 1, k.before);
            for (int q = 0; q < Q; ++q) {
                chunk_apply<double, MC, true>(ch[q], sp[q].n, k, wrap_entry<double>(wk(q), k.before, sx[k.before ? q : q + 1]));
                acc += chunk_norm2<double, MC>(ch[q], sp[q].n) / LL;
            }
            for (int q = 0; q < Q; ++q) {
                chunk_scale<double, MC>(ch[q], k.B * (1.0 / LL));   // z with the 1 / L^2
                chunk_map<double, MC, false>(ch[q], sp[q].n, k, sa[q], sc[q]);
                wrap_map<double>(wkd(q), k.before, sa[q], sc[q]);
            }
            chunk_close<double>(sa, sc, sx, Q, 1, !k.before);
            for (int q = 0; q < Q; ++q) {
                chunk_apply<double, MC, false>(ch[q], sp[q].n, k, wrap_entry<double>(wkd(q), k.before, sx[k.before ? q + 1 : q]));
                for (int j = 0; j < sp[q].n; ++j) w[at(q, j)] = ch[q][j];
            }
        }
    }
    for (int sl = 0; sl < 4 * Lt; ++sl) {
        double2* slice = w.data() + size_t(sl) * LL;
        fft_slice_io<double, true>(ex, slice, sbuf.data(), slice, pl, twl);
    }
    for (size_t i = 0; i < w.size(); ++i) {
        out[2 * i] = w[i].x;
        out[2 * i + 1] = w[i].y;
    }
    if (rz) *rz = acc;
    return 0;
}

int hmc_test_apply_precond(hmc_ctx* c, int precision, const void* in, void* out, int n, double* rz, void* stream) {
    if (c == nullptr || in == nullptr || out == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    int rc = need_ws(c);
    if (rc) return rc;
    if (c->is_batch) return fail(HMC_ERR_INVALID_ARG, "one-lattice contexts only");
    if (precision != HMC_FP64 && precision != HMC_MIXED) return fail(HMC_ERR_INVALID_ARG, "unknown precision");
    if (n < 1 || n > c->cap) return fail(HMC_ERR_INVALID_ARG, "n = %d outside [1, %d]", n, c->cap);
    if (!aligned16(in) || !aligned16(out)) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    const int pi = precision == HMC_MIXED ? 1 : 0;
    if (!c->pc_ok[pi]) return fail(HMC_ERR_INVALID_ARG, "Fourier preconditioner unavailable for this lattice");
    const hipStream_t s = (hipStream_t)stream;
    return pi ? apply_precond_impl<float>(c, static_cast<const double2*>(in), out, n, rz, s)
              : apply_precond_impl<double>(c, static_cast<const double2*>(in), out, n, rz, s);
}

int hmc_stream_probe(int kind, const void* src, void* dst, size_t bytes, int grid, void* stream) {
    if (dst == nullptr || (kind != HMC_PROBE_WRITE && src == nullptr)) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if (bytes == 0 || bytes % 16 != 0) return fail(HMC_ERR_INVALID_ARG, "bytes must be a positive multiple of 16");
    if (!aligned16(dst) || (src != nullptr && !aligned16(src))) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    if (grid == 0) grid = 2048;
    if (grid < 1 || grid > 65536) return fail(HMC_ERR_INVALID_ARG, "grid outside [1, 65536]");
    const size_t n4 = bytes / 16;
    const float4* a = static_cast<const float4*>(src);
    float4* b = static_cast<float4*>(dst);
    const hipStream_t s = (hipStream_t)stream;
    switch (kind) {
        case HMC_PROBE_READ:
            hipLaunchKernelGGL((k_stream<1, 0>), dim3(grid), dim3(kBlock), 0, s, a, nullptr, n4, static_cast<double*>(dst));
            break;
        case HMC_PROBE_WRITE:
            hipLaunchKernelGGL((k_stream<0, 1>), dim3(grid), dim3(kBlock), 0, s, nullptr, b, n4, nullptr);
            break;
        case HMC_PROBE_COPY:
            hipLaunchKernelGGL((k_stream<1, 1>), dim3(grid), dim3(kBlock), 0, s, a, b, n4, nullptr);
            break;
        case HMC_PROBE_3R3W:
            hipLaunchKernelGGL((k_stream<3, 3>), dim3(grid), dim3(kBlock), 0, s, a, b, n4, nullptr);
            break;
        case HMC_PROBE_READ_NT:
            hipLaunchKernelGGL((k_stream<1, 0, true>), dim3(grid), dim3(kBlock), 0, s, a, nullptr, n4,
                               static_cast<double*>(dst));
            break;
        default:
            return fail(HMC_ERR_INVALID_ARG, "unknown probe kind %d", kind);
    }
    LAUNCHCHK();
    return HMC_OK;
}

int hmc_test_tile_span(int blk, int bpr, int nt, int out[3]) {
    if (out == nullptr || bpr < 1 || blk < 0 || blk >= bpr || nt < 0) return -1;
    const TileSpan t = tile_span(blk, bpr, nt);
    out[0] = t.first;
    out[1] = t.end;
    out[2] = t.step;
    return 0;
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
    c->nblk = tiles1_host(c->vol);
    c->nblk2 = tiles2_host(c->vol);
    c->vec_sites = (long long)c->cap * c->vol;
    c->phi_sites = c->vol;
    c->nunits = c->cap;
    c->pstride = unit_slots(c->lat);
    c->pslots = c->cap * c->pstride;
    c->ngblk = c->nblk;
    set_coefs(c);
    rc = create_common(c);
    if (rc == HMC_OK) {
        pc_setup(c);
        rc = check_precond(c, params);
    }
    if (rc) {
        destroy_common(c);
        delete c;
        return rc;
    }
    (void)set_cg_shape(c, HMC_FP64, kDefaultBpr64);
    (void)set_cg_shape(c, HMC_MIXED, kDefaultBpr32);
    // the one-pass M^dagger M march holds two slices of psi and two of chi in LDS (above 64 KB)
    for (const void* k : {reinterpret_cast<const void*>(&k_mdm2_march<kMarchMaxThreads>),
                          reinterpret_cast<const void*>(&k_mdm2_march<kMdmMidThreads>),
                          reinterpret_cast<const void*>(&k_mdm2_march<kMdmMarchThreads>),
                          reinterpret_cast<const void*>(&k_mdm_march<kMarchMaxThreads>),
                          reinterpret_cast<const void*>(&k_mdm_march<kMdmMidThreads>),
                          reinterpret_cast<const void*>(&k_mdm_march<kMdmMarchThreads>)})
        (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 << 10);
    (void)hipGetLastError();
    // step A marches by default (the tile kernels where a lattice's band does not fit)
    c->cgm_rows[0] = 4;
    c->cgm_rows[1] = 8;
    c->cgm_seg[0] = c->cgm_seg[1] = 8;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(TuneKey{L, Lt, c->cap, c->device, c->cf64.nn2 != 0});
        TuneChoice ch;
        bool have = it != g_tuned.end();
        if (have) ch = it->second;
        else have = tune_cache_lookup(tune_key(c), ch);
        if (have) apply_choice(c, ch);
    }
    c->need = ws_layout(c, nullptr);
    *out = c;
    return HMC_OK;
}

int hmc_set_kernel_timing(hmc_ctx* c, int enable) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    if (enable && c->tev[0][0] == nullptr) {
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < hmc_ctx::kEv; ++j) HIPCHK(hipEventCreate(&c->tev[i][j]));
    }
    c->timing = enable != 0;
    std::memset(&c->kt, 0, sizeof(c->kt));
    return HMC_OK;
}

int hmc_set_metric(hmc_ctx* c, const double* sigma) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    if (c->is_batch) return fail(HMC_ERR_INVALID_ARG, "the Fourier metric is for one-lattice contexts");
    if (sigma != nullptr) {
        if (!c->metric_ok)
            return fail(HMC_ERR_INVALID_ARG,
                        "Fourier metric unavailable for this lattice (L and L_tau need prime factors <= 7, "
                        "and an L x L FP64 slice must fit the GPU's LDS)");
        if (!aligned16(sigma)) return fail(HMC_ERR_INVALID_ARG, "sigma must be 16-byte aligned");
    }
    c->sigma = sigma;
    return HMC_OK;
}

// Common checks of the metric entry points (two field pointers, either may be required).
static int metric_check(hmc_ctx* c, const void* a, const void* b) {
    if (c == nullptr || a == nullptr || b == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if (c->is_batch) return fail(HMC_ERR_INVALID_ARG, "the Fourier metric is for one-lattice contexts");
    int rc = need_ws(c);
    if (rc) return rc;
    if (!c->metric_ok)
        return fail(HMC_ERR_INVALID_ARG,
                    "Fourier metric unavailable for this lattice (L and L_tau need prime factors <= 7, "
                    "and an L x L FP64 slice must fit the GPU's LDS)");
    if (!aligned16(a) || !aligned16(b)) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    return HMC_OK;
}

static int read_slot(hmc_ctx* c, int slot, double* out, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(c->h_slots + slot, c->slots + slot, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = c->h_slots[slot];
    return HMC_OK;
}

int hmc_metric_momenta(hmc_ctx* c, const double* xi, double* pi, void* stream) {
    int rc = metric_check(c, xi, pi);
    if (rc) return rc;
    return metric_passes(c, xi, pi, 0, 0.0, MUL_RSQRT, RED_NONE, 1.0, nullptr, 0, (hipStream_t)stream);
}

int hmc_metric_kinetic(hmc_ctx* c, const double* pi, double* K, void* stream) {
    int rc = metric_check(c, pi, K);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = metric_passes(c, pi, nullptr, 0, 0.0, 0, RED_SIGMA, 0.5, nullptr, SL_TMP, s);
    if (rc) return rc;
    return read_slot(c, SL_TMP, K, s);
}

int hmc_metric_norm2(hmc_ctx* c, const double* v, double* out, void* stream) {
    int rc = metric_check(c, v, out);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = metric_passes(c, v, nullptr, 0, 0.0, 0, RED_INV, 1.0, nullptr, SL_TMP, s);
    if (rc) return rc;
    return read_slot(c, SL_TMP, out, s);
}

int hmc_metric_accumulate(hmc_ctx* c, const double* phi, double* acc, void* stream) {
    int rc = metric_check(c, phi, acc);
    if (rc) return rc;
    return metric_passes(c, phi, nullptr, 0, 0.0, 0, RED_NONE, 1.0, acc, 0, (hipStream_t)stream);
}

int hmc_sdw_accumulate(hmc_ctx* c, const double* phi, double* chi, void* stream) {
    int rc = metric_check(c, phi, chi);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // per-component spectra into the idle FP64 CG residual, then summed into chi
    double* t = reinterpret_cast<double*>(c->r64);
    const double* sg = c->sigma;
    c->sigma = nullptr;
    rc = metric_passes(c, phi, nullptr, 0, 0.0, 0, RED_NONE, 1.0, t, 0, s, 0);
    c->sigma = sg;
    if (rc) return rc;
    hipLaunchKernelGGL(k_mt_sum3, dim3(elem_grid(c->vol)), dim3(kBlock), 0, s, static_cast<const double*>(t), chi,
                       c->dtau, int(c->vol));
    LAUNCHCHK();
    return HMC_OK;
}

int hmc_order_parameter(hmc_ctx* c, const double* phi, double* Phi, void* stream) {
    if (c == nullptr || phi == nullptr || Phi == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if (c->is_batch) return fail(HMC_ERR_INVALID_ARG, "the order parameter is for one-lattice contexts");
    int rc = need_ws(c);
    if (rc) return rc;
    if (!aligned16(phi)) return fail(HMC_ERR_INVALID_ARG, "phi must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const int nb = std::min(256, elem_grid(c->vol));
    hipLaunchKernelGGL(k_mt_csum, dim3(3 * nb), dim3(kBlock), 0, s, phi, c->mpart, int(c->vol), nb);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, static_cast<const double*>(c->mpart), nb, 3, nb,
                       c->slots + SL_TMP);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(c->h_slots + SL_TMP, c->slots + SL_TMP, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int l = 0; l < 3; ++l) Phi[l] = c->h_slots[SL_TMP + l];
    return HMC_OK;
}

double hmc_binder(const double* Phi, int S) {
    if (Phi == nullptr || S < 1) return std::nan("");
    double s2 = 0.0, s4 = 0.0;
    for (int i = 0; i < S; ++i) {
        const double n2 = Phi[3 * i] * Phi[3 * i] + Phi[3 * i + 1] * Phi[3 * i + 1] + Phi[3 * i + 2] * Phi[3 * i + 2];
        s2 += n2;
        s4 += n2 * n2;
    }
    const double m2 = s2 / S, m4 = s4 / S;
    return 1.0 - 3.0 * m4 / (5.0 * m2 * m2);
}

int hmc_set_graphs(hmc_ctx* c, int enable) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    c->graphs = enable != 0;
    return HMC_OK;
}

int hmc_set_step_graphs(hmc_ctx* c, int enable) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    c->step_graphs = enable != 0;
    return HMC_OK;
}

int hmc_set_cg_workgroups(hmc_ctx* c, int precision, int max_per_rhs) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    if (precision != HMC_FP64 && precision != HMC_MIXED && precision != -1)
        return fail(HMC_ERR_INVALID_ARG, "precision must be HMC_FP64, HMC_MIXED or -1");
    if (max_per_rhs < 1 || max_per_rhs > kMaxBpr)
        return fail(HMC_ERR_INVALID_ARG, "workgroups per right-hand side must lie in [1, %d]", kMaxBpr);
    return set_cg_shape(c, precision, max_per_rhs);
}

int hmc_set_mdm_shape(hmc_ctx* c, int precision, int rows, int slices) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    if (precision != HMC_FP64 && precision != HMC_MIXED && precision != -1)
        return fail(HMC_ERR_INVALID_ARG, "unknown precision");
    if (rows < 0 || rows > 256 || slices < 0 || slices > 1 << 20)
        return fail(HMC_ERR_INVALID_ARG, "rows must lie in [0, 256] and slices be >= 0");
    for (int pi = 0; pi < 2; ++pi)
        if (precision == -1 || precision == (pi ? HMC_MIXED : HMC_FP64)) {
            c->mdm_rows[pi] = rows;
            c->mdm_seg[pi] = slices;
        }
    return HMC_OK;
}

int hmc_set_cg_march(hmc_ctx* c, int precision, int rows, int slices) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    if (c->is_batch) return fail(HMC_ERR_INVALID_ARG, "one-lattice contexts only");
    if (precision != HMC_FP64 && precision != HMC_MIXED && precision != -1)
        return fail(HMC_ERR_INVALID_ARG, "unknown precision");
    if (rows < 0 || rows > 256 || slices < 0 || slices > 1 << 20)
        return fail(HMC_ERR_INVALID_ARG, "rows must lie in [0, 256] and slices be >= 0");
    for (int pi = 0; pi < 2; ++pi)
        if (precision == -1 || precision == (pi ? HMC_MIXED : HMC_FP64)) {
            c->cgm_rows[pi] = rows;
            c->cgm_seg[pi] = slices;
        }
    c->generation += 1;   // captured graphs hold the launch shape
    return HMC_OK;
}

int hmc_set_cg_march_step_b(hmc_ctx* c, int precision, int enable) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    if (precision != HMC_FP64 && precision != HMC_MIXED && precision != -1)
        return fail(HMC_ERR_INVALID_ARG, "unknown precision");
    for (int pi = 0; pi < 2; ++pi)
        if (precision == -1 || precision == (pi ? HMC_MIXED : HMC_FP64)) c->cgb_march[pi] = enable != 0;
    c->generation += 1;   // captured graphs hold the launch shape
    return HMC_OK;
}

int hmc_get_cg_march_step_b(const hmc_ctx* c, int precision) {
    if (c == nullptr || (precision != HMC_FP64 && precision != HMC_MIXED)) return -1;
    return c->cgb_march[precision == HMC_MIXED ? 1 : 0];
}

int hmc_get_cg_march(const hmc_ctx* c, int precision, int* rows, int* slices) {
    if (c == nullptr || rows == nullptr || slices == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if (precision != HMC_FP64 && precision != HMC_MIXED) return fail(HMC_ERR_INVALID_ARG, "unknown precision");
    const int pi = precision == HMC_MIXED ? 1 : 0;
    *rows = c->cgm_rows[pi];
    *slices = c->cgm_seg[pi];
    return HMC_OK;
}

int hmc_get_mdm_shape(const hmc_ctx* c, int precision, int n, int* rows, int* slices, int* workgroups) {
    if (c == nullptr || rows == nullptr || slices == nullptr || workgroups == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if (precision != HMC_FP64 && precision != HMC_MIXED) return fail(HMC_ERR_INVALID_ARG, "unknown precision");
    if (n < 1) return fail(HMC_ERR_INVALID_ARG, "n must be >= 1");
    const MdmShape m = precision == HMC_MIXED ? mdm_shape<float>(c, n) : mdm_shape<double>(c, n);
    *rows = m.plan.R;
    *slices = m.plan.seglen;
    *workgroups = n * m.plan.nband * m.plan.nseg;
    return HMC_OK;
}

int hmc_get_cg_workgroups(const hmc_ctx* c, int precision) {
    if (c == nullptr) return -1;
    return precision == HMC_MIXED ? c->bpr32 : c->bpr64;
}

int hmc_autotune(hmc_ctx* c, const double* phi, const void* b, int n, hmc_tune_result* out,
                 void* stream) {
    int rc = check_solve_args(c, phi, b, c ? c->xsol : nullptr, n);
    if (rc) return rc;
    if (out == nullptr) return fail(HMC_ERR_INVALID_ARG, "out is NULL");
    if (reuse_cached()) {
        TuneChoice ch;
        if (tune_cache_lookup(tune_key(c), ch)) {
            apply_choice(c, ch);
            choice_result(ch, out);
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned[TuneKey{c->L, c->Lt, c->cap, c->device, c->cf64.nn2 != 0}] = ch;
            return HMC_OK;
        }
    }
    rc = autotune_common(c, phi, static_cast<const double2*>(b), n, out, (hipStream_t)stream);
    if (rc) return rc;
    const TuneChoice ch = current_choice(c);
    tune_cache_store(tune_key(c), ch);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[TuneKey{c->L, c->Lt, c->cap, c->device, c->cf64.nn2 != 0}] = ch;
    return HMC_OK;
}

int hmc_get_kernel_times(const hmc_ctx* c, hmc_kernel_times* out) {
    if (c == nullptr || out == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    *out = c->kt;
    return HMC_OK;
}

int hmc_destroy(hmc_ctx* c) {
    if (c == nullptr) return HMC_OK;
    destroy_common(c);
    delete c;
    return HMC_OK;
}

int hmc_set_params(hmc_ctx* c, const hmc_params* params) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "ctx is NULL");
    int rc = check_params(params);
    if (rc) return rc;
    const int want = params->max_rhs > 0 ? params->max_rhs : params->n_pf;
    if (want > c->cap) return fail(HMC_ERR_INVALID_ARG, "n_pf/max_rhs %d exceeds workspace capacity %d", want, c->cap);
    rc = check_precond(c, params);
    if (rc) return rc;
    c->p = *params;
    set_coefs(c);
    return HMC_OK;
}

size_t hmc_workspace_bytes(const hmc_ctx* c) { return c ? c->need : 0; }

int hmc_set_workspace(hmc_ctx* c, void* ptr, size_t bytes) {
    if (c == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL ctx");
    return set_workspace_common(c, ptr, bytes);
}

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

int hmc_apply_MdagM_noalloc(hmc_ctx* c, const double* phi, const void* in, void* out, int n, void* stream) {
    if (c == nullptr || phi == nullptr || in == nullptr || out == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if (c->is_batch) return fail(HMC_ERR_INVALID_ARG, "one-lattice contexts only");
    if (n < 1) return fail(HMC_ERR_INVALID_ARG, "n must be >= 1");
    const size_t need = size_t(n) * 4 * size_t(c->vol) * sizeof(double2);
    if (need > kStaticScratchBytes)
        return fail(HMC_ERR_INVALID_ARG, "n = %d vectors of this lattice need %zu bytes of scratch, above the %zu "
                    "of the static buffer", n, need, kStaticScratchBytes);
    if (c->scratch == nullptr) return fail(HMC_ERR_HIP, "the static scratch has no device address on this GPU");
    if (in == c->scratch || out == c->scratch) return fail(HMC_ERR_INVALID_ARG, "in/out alias the static scratch");
    int rc = apply_impl<double, false>(c, phi, in, c->scratch, n, stream);
    if (rc) return rc;
    return apply_impl<double, true>(c, phi, c->scratch, out, n, stream);
}

int hmc_heatbath(hmc_ctx* c, const double* phi, const void* eta, void* chi, int n_pf, void* stream) {
    return apply_impl<double, true>(c, phi, eta, chi, n_pf, stream);
}

int hmc_cg_solve(hmc_ctx* c, const double* phi, const void* b, void* x, int n,
                 hmc_cg_stats* stats, void* stream) {
    int rc = check_solve_args(c, phi, b, x, n);
    if (rc) return rc;
    return cg_dispatch(c, phi, static_cast<const double2*>(b), static_cast<double2*>(x), n, stats,
                       (hipStream_t)stream);
}

int hmc_force_from_solution(hmc_ctx* c, const double* phi, const void* x, int n_pf,
                            double* force, int flags, void* stream) {
    if (c == nullptr || phi == nullptr || force == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if ((flags & HMC_FORCE_PF) && (x == nullptr || n_pf < 1)) return fail(HMC_ERR_INVALID_ARG, "pseudofermion force needs x and n_pf >= 1");
    if (n_pf < 0 || n_pf > HMC_MAX_RHS) return fail(HMC_ERR_INVALID_ARG, "n_pf out of range");
    if (!aligned16(phi) || !aligned16(force) || (x && !aligned16(x))) return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    return launch_force(c, phi, static_cast<const double2*>(x), (flags & HMC_FORCE_PF) ? n_pf : 0, flags,
                        force, nullptr, 0.0, 0, (hipStream_t)stream);
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
    int rc2 = dot_re(c, static_cast<const double2*>(chi), xs, n_pf, SL_TMP, s);
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
        rc2 = dot_re(c, static_cast<const double2*>(chi), c->xsol, n_pf, SL_TMP, s);
        if (rc2) return rc2;
        HIPCHK(hipMemcpyAsync(S_pf, c->slots + SL_TMP, sizeof(double), hipMemcpyDeviceToDevice, s));
    } else if (S_pf) {
        HIPCHK(hipMemsetAsync(S_pf, 0, sizeof(double), s));
    }
    return rc;
}

int hmc_boson_action(hmc_ctx* c, const double* phi, double* S, void* stream) {
    if (c == nullptr || phi == nullptr || S == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    int rc = need_ws(c);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = energy(c, nullptr, phi, SL_TMP, s);
    if (rc) return rc;
    rc = read_slots(c, s);
    if (rc) return rc;
    *S = c->h_slots[SL_TMP + 1];
    return HMC_OK;
}

// The proposal of one trajectory from (phi, pi0): phi0 kept in c->phi_save, pi0 copied to
// c->pi, heat-bath chi = M^dagger eta, energies at both ends and the molecular dynamics.
// Leaves the proposal in phi and fills stats (no decision).  On an error phi is restored.
static int traj_propose(hmc_ctx* c, double* phi, const double* pi0, const void* eta, int n_pf,
                        hmc_traj_stats* stats, hipStream_t s) {
    std::memset(stats, 0, sizeof(*stats));
    const size_t phib = 3 * size_t(c->vol) * sizeof(double);
    HIPCHK(hipMemcpyAsync(c->phi_save, phi, phib, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(c->pi, pi0, phib, hipMemcpyDeviceToDevice, s));
    int rc;
    if (n_pf > 0) {
        rc = launch_apply<double, true>(c, phi, eta, c->chi, n_pf, s);
        if (rc) return rc;
        rc = dot_re(c, static_cast<const double2*>(eta), static_cast<const double2*>(eta), n_pf, SL_SPF0, s);
        if (rc) return rc;
    }
    rc = energies(c, c->pi, phi, SL_K0, s);
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
    rc = energies(c, c->pi, phi, SL_K1, s);
    if (rc) return restore(rc);
    rc = read_slots(c, s);
    if (rc) return restore(rc);
    fill_energies(c->h_slots, n_pf, stats);
    if (!std::isfinite(stats->dH)) return restore(fail(HMC_ERR_NONFINITE, "dH is not finite"));
    stats->status = HMC_OK;
    return HMC_OK;
}

static int restore_phi(hmc_ctx* c, double* phi, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(phi, c->phi_save, 3 * size_t(c->vol) * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return HMC_OK;
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
    rc = traj_propose(c, phi, pi0, eta, n_pf, stats, s);
    if (rc) return rc;
    stats->accepted = (u < std::exp(-stats->dH)) ? 1 : 0;
    if (!stats->accepted) return restore_phi(c, phi, s);
    return HMC_OK;
}

// --------------------------------------------------------------------------------------
// Warm-up tuning (Eq. 31, Eq. 32): host arithmetic

static double accept_prob(double dH) { return dH <= 0.0 ? 1.0 : std::exp(-dH); }

int hmc_tuner_init(hmc_tuner* t, double eps, int window, double factor, int n_cap) {
    if (t == nullptr) return fail(HMC_ERR_INVALID_ARG, "tuner is NULL");
    if (!(eps > 0.0) || !std::isfinite(eps) || window < 1 || !(factor > 1.0) || !std::isfinite(factor) ||
        n_cap < 1 || n_cap > HMC_TUNER_MAX_LEN)
        return fail(HMC_ERR_INVALID_ARG, "tuner needs eps > 0, window >= 1, factor > 1, 1 <= n_cap <= %d",
                    HMC_TUNER_MAX_LEN);
    std::memset(t, 0, sizeof(*t));
    t->eps = eps;
    t->factor = factor;
    t->window = window;
    t->n_cap = n_cap;
    return HMC_OK;
}

static bool tuner_valid(const hmc_tuner* t) {
    return t != nullptr && t->eps > 0.0 && std::isfinite(t->eps) && t->window >= 1 && t->factor > 1.0 &&
           t->n_cap >= 1 && t->n_cap <= HMC_TUNER_MAX_LEN && t->count >= 0 && t->count < t->window;
}

int hmc_tuner_add_step(hmc_tuner* t, double dH_eps, double dH_half) {
    if (!tuner_valid(t)) return fail(HMC_ERR_INVALID_ARG, "invalid tuner");
    if (std::isnan(dH_eps) || std::isnan(dH_half)) return fail(HMC_ERR_INVALID_ARG, "dH is NaN");
    t->sum_alpha_eps += accept_prob(dH_eps);
    t->sum_alpha_half += accept_prob(dH_half);
    t->count += 1;
    if (t->count >= t->window) {
        const double ae = t->sum_alpha_eps / t->count, ah = t->sum_alpha_half / t->count;
        const bool holds = ae > 0.0 && ah * ah <= 2.0 * ae;
        t->eps = holds ? t->eps * t->factor : t->eps / t->factor;
        t->count = 0;
        t->sum_alpha_eps = t->sum_alpha_half = 0.0;
    }
    return HMC_OK;
}

int hmc_tuner_add_jump(hmc_tuner* t, int n, double sqdist, double dH) {
    if (!tuner_valid(t)) return fail(HMC_ERR_INVALID_ARG, "invalid tuner");
    if (n < 1 || n > t->n_cap) return fail(HMC_ERR_INVALID_ARG, "length %d outside [1, %d]", n, t->n_cap);
    if (!std::isfinite(sqdist) || std::isnan(dH)) return fail(HMC_ERR_INVALID_ARG, "non-finite jump sample");
    t->esjd_sum[n] += sqdist * accept_prob(dH);
    t->esjd_count[n] += 1;
    return HMC_OK;
}

int hmc_tuner_best_length(const hmc_tuner* t) {
    if (t == nullptr || t->n_cap < 1 || t->n_cap > HMC_TUNER_MAX_LEN) return 0;
    int best = 0;
    double bv = 0.0;
    for (int n = 1; n <= t->n_cap; ++n) {
        if (t->esjd_count[n] == 0) continue;
        const double v = t->esjd_sum[n] / double(t->esjd_count[n]);
        if (best == 0 || v > bv) {
            best = n;
            bv = v;
        }
    }
    return best;
}

int hmc_jitter(double u, int n_max) {
    if (n_max < 1 || !(u >= 0.0 && u < 1.0)) return 0;
    const double k = std::floor(u * double(n_max));
    return 1 + (k > double(n_max - 1) ? n_max - 1 : int(k));
}

int hmc_warmup_iteration(hmc_ctx* c, hmc_tuner* t, double* phi, const double* xi, const void* eta, int n_pf,
                         double u_accept, double u_length, hmc_warmup_stats* out, void* stream) {
    if (c == nullptr || t == nullptr || phi == nullptr || xi == nullptr || out == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    if (c->is_batch) return fail(HMC_ERR_INVALID_ARG, "warm-up iterations are for one-lattice contexts");
    if (!tuner_valid(t)) return fail(HMC_ERR_INVALID_ARG, "invalid tuner");
    int rc = need_ws(c);
    if (rc) return rc;
    if (n_pf < 0 || n_pf > c->cap) return fail(HMC_ERR_INVALID_ARG, "n_pf %d outside [0, %d]", n_pf, c->cap);
    if (n_pf > 0 && eta == nullptr) return fail(HMC_ERR_INVALID_ARG, "eta is NULL");
    if (!aligned16(phi) || !aligned16(xi) || (eta && !aligned16(eta)))
        return fail(HMC_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    const int n = hmc_jitter(u_length, t->n_cap);
    if (n == 0) return fail(HMC_ERR_INVALID_ARG, "u_length must lie in [0, 1)");
    hipStream_t s = (hipStream_t)stream;
    std::memset(out, 0, sizeof(*out));
    const size_t phib = 3 * size_t(c->vol) * sizeof(double);
    const double eps = t->eps;
    const double saved_eps = c->p.eps;
    const int saved_nl = c->p.n_leap;
    auto done = [&](int code) {
        c->p.eps = saved_eps;
        c->p.n_leap = saved_nl;
        return code;
    };
    // momenta under the metric, kept for all three proposals
    if (c->sigma != nullptr) rc = metric_passes(c, xi, c->piw, 0, 0.0, MUL_RSQRT, RED_NONE, 1.0, nullptr, 0, s);
    else rc = hipMemcpyAsync(c->piw, xi, phib, hipMemcpyDeviceToDevice, s) == hipSuccess
                  ? HMC_OK : fail(HMC_ERR_HIP, "copy failed");
    if (rc) return done(rc);
    hmc_traj_stats st[3];
    const double eps_of[3] = {eps, 0.5 * eps, eps};
    const int len_of[3] = {1, 1, n};
    for (int k = 0; k < 3; ++k) {
        c->p.eps = eps_of[k];
        c->p.n_leap = len_of[k];
        rc = traj_propose(c, phi, c->piw, eta, n_pf, &st[k], s);
        if (rc) return done(rc);
        out->cg_iterations += st[k].cg_iterations;
        out->max_true_resid = std::max(out->max_true_resid, st[k].max_true_resid);
        if (k < 2) {
            rc = restore_phi(c, phi, s);
            if (rc) return done(rc);
        }
    }
    // squared jump distance of the proposal: dphi = phi' - phi0 in the (idle) CG residual
    double* dphi = reinterpret_cast<double*>(c->r64);
    double sq = 0.0;
    rc = hipMemcpyAsync(dphi, phi, phib, hipMemcpyDeviceToDevice, s) == hipSuccess ? HMC_OK
                                                                                : fail(HMC_ERR_HIP, "copy failed");
    if (!rc) {
        hipLaunchKernelGGL(k_drift, dim3(elem_grid(3LL * c->phi_sites)), dim3(kBlock), 0, s, dphi,
                           static_cast<const double*>(c->phi_save), -1.0, int(3 * c->phi_sites));
        rc = hipGetLastError() == hipSuccess ? HMC_OK : fail(HMC_ERR_HIP, "kernel launch failed");
    }
    if (!rc) {
        if (c->sigma != nullptr) rc = metric_passes(c, dphi, nullptr, 0, 0.0, 0, RED_INV, 1.0, nullptr, SL_TMP, s);
        else rc = energy(c, dphi, phi, SL_TMP, s);      // slot SL_TMP: |dphi|^2 / 2
    }
    if (!rc) rc = read_slot(c, SL_TMP, &sq, s);
    if (rc) {
        (void)restore_phi(c, phi, s);
        return done(rc);
    }
    if (c->sigma == nullptr) sq *= 2.0;
    out->eps = eps;
    out->dH_eps = st[0].dH;
    out->dH_half = st[1].dH;
    out->dH = st[2].dH;
    out->n_leap = n;
    out->sqdist = sq;
    out->accepted = (u_accept < std::exp(-st[2].dH)) ? 1 : 0;
    if (!out->accepted) {
        rc = restore_phi(c, phi, s);
        if (rc) return done(rc);
    }
    (void)hmc_tuner_add_jump(t, n, sq, st[2].dH);
    (void)hmc_tuner_add_step(t, st[0].dH, st[1].dH);
    out->eps_next = t->eps;
    return done(HMC_OK);
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
    rc = energies(c, pi, phi, SL_K0, s);
    if (rc) return rc;
    rc = md_integrate(c, phi, pi, static_cast<const double2*>(chi), n_pf, true, stats, s);
    if (rc) { stats->status = rc; return rc; }
    rc = energies(c, pi, phi, SL_K1, s);
    if (rc) return rc;
    rc = read_slots(c, s);
    if (rc) return rc;
    fill_energies(c->h_slots, n_pf, stats);
    stats->accepted = 1;
    stats->status = HMC_OK;
    return HMC_OK;
}

// --------------------------------------------------------------------------------------
// C ABI: batch of independent lattices

int hmc_batch_create(int nchains, const int* L, const int* L_tau, const double* r, double dtau,
                     const hmc_params* params, hmc_batch** out) {
    g_last_error.clear();
    if (out == nullptr || L == nullptr || L_tau == nullptr || r == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (nchains < 1) return fail(HMC_ERR_INVALID_ARG, "nchains must be >= 1");
    if (!(dtau > 0.0) || !std::isfinite(dtau)) return fail(HMC_ERR_INVALID_ARG, "dtau must be > 0");
    int rc = check_params(params);
    if (rc) return rc;
    if (params->n_pf < 1) return fail(HMC_ERR_INVALID_ARG, "batch mode needs n_pf >= 1");
    long long tot_vol = 0;
    for (int i = 0; i < nchains; ++i) {
        if (!geometry_ok(L[i], L_tau[i]))
            return fail(HMC_ERR_INVALID_ARG, "chain %d: bad lattice L=%d L_tau=%d", i, L[i], L_tau[i]);
        if (!std::isfinite(r[i])) return fail(HMC_ERR_INVALID_ARG, "chain %d: r not finite", i);
        tot_vol += (long long)L_tau[i] * L[i] * L[i];
    }
    const long long tot_units = (long long)nchains * params->n_pf;
    if (tot_units > (1 << 14) || 4LL * params->n_pf * tot_vol >= (1LL << 31) || 3LL * tot_vol >= (1LL << 31))
        return fail(HMC_ERR_INVALID_ARG, "batch too large");
    hmc_batch* hb = new hmc_batch();
    hmc_ctx* c = &hb->c;
    c->is_batch = true;
    c->dtau = dtau;
    c->p = *params;
    c->cap = params->n_pf;
    BatchInfo& b = c->bi;
    b.nchains = nchains;
    b.nrhs = params->n_pf;
    b.phi_off.push_back(0);
    b.sp_off.push_back(0);
    b.cfirst.push_back(0);
    for (int i = 0; i < nchains; ++i) {
        const Lat lat = make_lat(L[i], L_tau[i]);
        b.lats.push_back(lat);
        b.r.push_back(r[i]);
        b.phi_off.push_back(b.phi_off.back() + 3LL * lat.vol);
        b.sp_off.push_back(b.sp_off.back() + 4LL * b.nrhs * lat.vol);
        b.cfirst.push_back(b.cfirst.back() + tiles1_host(lat.vol));
    }
    c->vec_sites = (long long)b.nrhs * tot_vol;
    c->phi_sites = tot_vol;
    c->nunits = int(tot_units);
    c->pslots = 0;
    for (const Lat& l : b.lats) c->pslots += b.nrhs * unit_slots(l);
    c->ngblk = b.cfirst.back();
    c->lat = b.lats[0];
    c->nblk = tiles1_host(c->lat.vol);
    c->nblk2 = tiles2_host(c->lat.vol);
    set_coefs(c);
    rc = create_common(c);
    if (rc == HMC_OK) {
        pc_setup(c);
        rc = check_precond(c, params);
    }
    if (rc) {
        destroy_common(c);
        delete hb;
        return rc;
    }
    c->bpr64 = kDefaultBpr64;
    c->bpr32 = kDefaultBpr32;
    // step A and the reliable update march by default (row caps per band; every lattice takes
    // the rows its band allows, or the tile kernels if some lattice fits no cut)
    c->cgm_rows[0] = 4;
    c->cgm_rows[1] = 8;
    c->cgm_seg[0] = c->cgm_seg[1] = 8;
    {
        TuneChoice ch;
        if (tune_cache_lookup(tune_key(c), ch)) apply_choice(c, ch);
    }
    (void)upload_batch_shape(c, 0, c->bpr64);    // counts only until the workspace is set
    (void)upload_batch_shape(c, 1, c->bpr32);
    c->need = ws_layout(c, nullptr);
    c->graphs = true;
    *out = hb;
    return HMC_OK;
}

int hmc_batch_destroy(hmc_batch* hb) {
    if (hb == nullptr) return HMC_OK;
    destroy_common(&hb->c);
    delete hb;
    return HMC_OK;
}

size_t hmc_batch_workspace_bytes(const hmc_batch* hb) { return hb ? hb->c.need : 0; }

int hmc_batch_set_workspace(hmc_batch* hb, void* ptr, size_t bytes) {
    if (hb == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL batch");
    return set_workspace_common(&hb->c, ptr, bytes);
}

int hmc_batch_layout(const hmc_batch* hb, long long* phi_offsets, long long* spinor_offsets) {
    if (hb == nullptr || phi_offsets == nullptr || spinor_offsets == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    const BatchInfo& b = hb->c.bi;
    for (int i = 0; i <= b.nchains; ++i) {
        phi_offsets[i] = b.phi_off[size_t(i)];
        spinor_offsets[i] = b.sp_off[size_t(i)];
    }
    return HMC_OK;
}

int hmc_batch_set_cg_workgroups(hmc_batch* hb, int precision, int max_per_unit) {
    if (hb == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL batch");
    return hmc_set_cg_workgroups(&hb->c, precision, max_per_unit);
}

int hmc_batch_get_cg_workgroups(const hmc_batch* hb, int precision) {
    return hb ? hmc_get_cg_workgroups(&hb->c, precision) : -1;
}

int hmc_batch_set_graphs(hmc_batch* hb, int enable) {
    if (hb == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL batch");
    hb->c.graphs = enable != 0;
    return HMC_OK;
}

int hmc_batch_set_cg_march(hmc_batch* hb, int precision, int rows, int slices) {
    if (hb == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL batch");
    hmc_ctx* c = &hb->c;
    if (precision != HMC_FP64 && precision != HMC_MIXED && precision != -1)
        return fail(HMC_ERR_INVALID_ARG, "unknown precision");
    if (rows < 0 || rows > 256 || slices < 0 || slices > 1 << 20)
        return fail(HMC_ERR_INVALID_ARG, "rows must lie in [0, 256] and slices be >= 0");
    for (int pi = 0; pi < 2; ++pi)
        if (precision == -1 || precision == (pi ? HMC_MIXED : HMC_FP64)) {
            c->cgm_rows[pi] = rows;
            c->cgm_seg[pi] = slices;
        }
    c->generation += 1;
    int rc = upload_batch_shape(c, 0, c->bpr64);
    if (rc == HMC_OK) rc = upload_batch_shape(c, 1, c->bpr32);
    return rc;
}

int hmc_batch_set_cg_march_step_b(hmc_batch* hb, int precision, int enable) {
    if (hb == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL batch");
    return hmc_set_cg_march_step_b(&hb->c, precision, enable);
}

int hmc_batch_get_cg_march(const hmc_batch* hb, int chain, int precision, int* rows, int* slices, int* ru_rows,
                           int* ru_slices, int* step_b) {
    if (hb == nullptr || rows == nullptr || slices == nullptr || ru_rows == nullptr || ru_slices == nullptr ||
        step_b == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL argument");
    const BatchInfo& b = hb->c.bi;
    if (chain < 0 || chain >= b.nchains) return fail(HMC_ERR_INVALID_ARG, "chain out of range");
    if (precision != HMC_FP64 && precision != HMC_MIXED) return fail(HMC_ERR_INVALID_ARG, "unknown precision");
    const int pi = precision == HMC_MIXED ? 1 : 0;
    const bool nn2 = hb->c.cf64.nn2 != 0;
    const UnitDesc& u = b.hunits[pi][size_t(chain) * size_t(b.nrhs)];
    const bool m = !nn2 && b.mgrid[pi] > 0, r = m && b.rgrid[pi] > 0;
    *rows = m ? u.mp.R : 0;
    *slices = m ? u.mp.seglen : 0;
    *ru_rows = r ? u.rmp.R : 0;
    *ru_slices = r ? u.rmp.seglen : 0;
    *step_b = m ? hb->c.cgb_march[pi] : 0;
    return HMC_OK;
}

int hmc_batch_set_step_graphs(hmc_batch* hb, int enable) {
    if (hb == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL batch");
    hb->c.step_graphs = enable != 0;
    return HMC_OK;
}

int hmc_batch_set_params(hmc_batch* hb, const hmc_params* params) {
    if (hb == nullptr) return fail(HMC_ERR_INVALID_ARG, "NULL batch");
    int rc = check_params(params);
    if (rc) return rc;
    if (params->n_pf != hb->c.bi.nrhs) return fail(HMC_ERR_INVALID_ARG, "n_pf is fixed at creation in batch mode");
    rc = check_precond(&hb->c, params);
    if (rc) return rc;
    hb->c.p = *params;
    set_coefs(&hb->c);
    if (hb->c.ws != nullptr) return upload_chains(&hb->c);
    return HMC_OK;
}

int hmc_batch_apply(hmc_batch* hb, int dagger, int precision, const void* phi, const void* in, void* out,
                    void* stream) {
    int rc = check_batch(hb, {phi, in, out});
    if (rc) return rc;
    if (in == out) return fail(HMC_ERR_INVALID_ARG, "in and out must not overlap");
    hmc_ctx* c = &hb->c;
    hipStream_t s = (hipStream_t)stream;
    if (precision == HMC_MIXED)
        return dagger ? launch_apply<float, true>(c, static_cast<const float*>(phi), in, out, 1, s)
                      : launch_apply<float, false>(c, static_cast<const float*>(phi), in, out, 1, s);
    if (precision != HMC_FP64) return fail(HMC_ERR_INVALID_ARG, "precision must be HMC_FP64 or HMC_MIXED");
    return dagger ? launch_apply<double, true>(c, static_cast<const double*>(phi), in, out, 1, s)
                  : launch_apply<double, false>(c, static_cast<const double*>(phi), in, out, 1, s);
}

int hmc_batch_cg_solve(hmc_batch* hb, const double* phi, const void* b, void* x, int* iterations,
                       double* true_resid, void* stream) {
    int rc = check_batch(hb, {phi, b, x});
    if (rc) return rc;
    if (b == x) return fail(HMC_ERR_INVALID_ARG, "b and x must not alias");
    hmc_ctx* c = &hb->c;
    rc = cg_dispatch_batch(c, phi, static_cast<const double2*>(b), static_cast<double2*>(x), (hipStream_t)stream);
    if (rc == HMC_OK || rc == HMC_ERR_NOT_CONVERGED || rc == HMC_ERR_NONFINITE) {
        for (int j = 0; j < c->nunits; ++j) {
            if (iterations) iterations[j] = c->h_st[j].iters;
            if (true_resid) true_resid[j] = true_resid_of(c->h_st[j]);
        }
    }
    return rc;
}

int hmc_batch_autotune(hmc_batch* hb, const double* phi, const void* b, hmc_tune_result* out, void* stream) {
    int rc = check_batch(hb, {phi, b});
    if (rc) return rc;
    if (out == nullptr) return fail(HMC_ERR_INVALID_ARG, "out is NULL");
    hmc_ctx* c = &hb->c;
    if (reuse_cached()) {
        TuneChoice ch;
        if (tune_cache_lookup(tune_key(c), ch)) {
            apply_choice(c, ch);
            rc = set_cg_shape(c, HMC_FP64, ch.bpr[0]);
            if (rc == HMC_OK) rc = set_cg_shape(c, HMC_MIXED, ch.bpr[1]);
            if (rc) return rc;
            choice_result(ch, out);
            return HMC_OK;
        }
    }
    rc = autotune_common(c, phi, static_cast<const double2*>(b), c->nunits, out, (hipStream_t)stream);
    if (rc) return rc;
    tune_cache_store(tune_key(c), current_choice(c));
    return HMC_OK;
}

int hmc_batch_trajectory(hmc_batch* hb, double* phi, const double* pi0, const void* eta,
                         const double* u, double* dH, int* accepted, hmc_traj_stats* totals,
                         void* stream) {
    int rc = check_batch(hb, {phi, pi0, eta});
    if (rc) return rc;
    if (u == nullptr || dH == nullptr || accepted == nullptr || totals == nullptr)
        return fail(HMC_ERR_INVALID_ARG, "NULL host argument");
    hmc_ctx* c = &hb->c;
    BatchInfo& b = c->bi;
    hipStream_t s = (hipStream_t)stream;
    std::memset(totals, 0, sizeof(*totals));
    const size_t phib = 3 * size_t(c->phi_sites) * sizeof(double);
    const int npf = b.nrhs;
    HIPCHK(hipMemcpyAsync(c->phi_save, phi, phib, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(c->pi, pi0, phib, hipMemcpyDeviceToDevice, s));
    rc = launch_apply<double, true>(c, phi, eta, c->chi, 1, s);
    if (rc) return rc;
    rc = dot_re(c, static_cast<const double2*>(eta), static_cast<const double2*>(eta), npf, SL_SPF0, s);
    if (rc) return rc;
    rc = energy(c, c->pi, phi, SL_K0, s);
    if (rc) return rc;
    auto restore_all = [&](int code) -> int {
        (void)hipMemcpyAsync(phi, c->phi_save, phib, hipMemcpyDeviceToDevice, s);
        (void)hipStreamSynchronize(s);
        for (int i = 0; i < b.nchains; ++i) accepted[i] = 0;
        totals->status = code;
        return code;
    };
    rc = md_integrate(c, phi, c->pi, c->chi, npf, false, totals, s);
    if (rc) return restore_all(rc);
    rc = energy(c, c->pi, phi, SL_K1, s);
    if (rc) return restore_all(rc);
    rc = read_slots(c, s);
    if (rc) return restore_all(rc);
    int nacc = 0;
    for (int i = 0; i < b.nchains; ++i) {
        hmc_traj_stats one{};
        fill_energies(b.h_cslots + size_t(i) * kChainSlots, npf, &one);
        dH[i] = one.dH;
        accepted[i] = (std::isfinite(one.dH) && u[i] < std::exp(-one.dH)) ? 1 : 0;
        nacc += accepted[i];
        if (!accepted[i]) {
            const size_t off = size_t(b.phi_off[size_t(i)]);
            const size_t bytes = size_t(b.phi_off[size_t(i) + 1] - b.phi_off[size_t(i)]) * sizeof(double);
            HIPCHK(hipMemcpyAsync(phi + off, c->phi_save + off, bytes, hipMemcpyDeviceToDevice, s));
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    totals->accepted = nacc;
    totals->status = HMC_OK;
    return HMC_OK;
}

}  // extern "C"
