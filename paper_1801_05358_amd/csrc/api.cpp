// C ABI of libdmwf (include/dmwf.h): plan lifecycle, input validation, the
// dual messenger solve (Algorithm 1) orchestrated as a sequence of HIP
// kernels on one stream, the diagnostics, and constrained realizations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dmwf_internal.h"

using namespace dmwf;

// Work memory of the allocation-free analysis (dm_map2alm_device_noalloc):
// the ring Fourier data and the partial-sum slots of one call live in this
// array, which the code object brings along, so that the call itself needs
// no device allocation.  Every GPU the library runs on holds its own copy,
// at its own address, until the process ends.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

// Device addresses of `scratch`, one per device, looked up once with that
// device current (the array's name is only a host-side stand-in).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Called at plan creation with `device` current.
void scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_scratch_done[device] = true;
}

void* scratch_of(int device, hipError_t* err) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *err = g_scratch_err[device];
    return g_scratch_ptr[device];
}

thread_local std::string g_create_err;

struct Fail {
    dm_status st;
};

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            p->err = std::string(#expr) + ": " + hipGetErrorString(e_);                           \
            throw Fail{e_ == hipErrorOutOfMemory ? DM_ENOMEM : DM_EDEVICE};                       \
        }                                                                                         \
    } while (0)

#define REQUIRE(cond, code, msg)         \
    do {                                 \
        if (!(cond)) {                   \
            p->err = (msg);              \
            throw Fail{code};            \
        }                                \
    } while (0)

template <class T>
void dalloc(dm_plan* p, T*& ptr, size_t count) {
    if (ptr) {
        (void)hipFree(ptr);
        ptr = nullptr;
    }
    if (count == 0) count = 1;
    HIPCHK(hipMalloc((void**)&ptr, count * sizeof(T)));
}

template <class T>
void dfree(T*& ptr) {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
}

template <class T>
void upload(dm_plan* p, T* dst, const T* src, size_t count) {
    HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, p->stream));
}

bool all_finite(const double* x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

// --------------------------------------------------------------------------
// timing of kernel classes with HIP events
// --------------------------------------------------------------------------
struct Timed {
    dm_plan* p;
    int cls;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(dm_plan* p_, int c, hipStream_t s_) : p(p_), cls(c), s(s_) {
        if (p->profiling) {
            HIPCHK(hipEventCreate(&a));
            HIPCHK(hipEventCreate(&b));
            HIPCHK(hipEventRecord(a, s));
        }
    }
    void done() {
        if (p->profiling) {
            HIPCHK(hipEventRecord(b, s));
            p->ev.start.push_back(a);
            p->ev.stop.push_back(b);
            p->ev.cls.push_back(cls);
        }
    }
};

void collect_events(dm_plan* p) {
    for (size_t i = 0; i < p->ev.start.size(); ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev.start[i], p->ev.stop[i]) == hipSuccess) {
            p->kc_ms[p->ev.cls[i]] += ms;
            p->kc_n[p->ev.cls[i]] += 1;
        }
        (void)hipEventDestroy(p->ev.start[i]);
        (void)hipEventDestroy(p->ev.stop[i]);
    }
    p->ev.start.clear();
    p->ev.stop.clear();
    p->ev.cls.clear();
}

// --------------------------------------------------------------------------
// transform building blocks
// --------------------------------------------------------------------------
// integer setting from the environment (tuning and test knobs)
int env_int(const char* k, int dflt) {
    const char* v = std::getenv(k);
    return v ? std::atoi(v) : dflt;
}

bool use_mfma(dm_plan* p, int nrhs);

// ring Fourier data: FP32 storage for the mixed matrix-core transforms
// (their products round the data to FP32 anyway), FP64 otherwise (the
// vector kernels, FP64 plans, a mixed plan's FP64 epilogue)
bool phase32(dm_plan* p, int nrhs) { return p->precision == DM_MIXED && p->d_phase32 && use_mfma(p, nrhs); }
void* phase_of(dm_plan* p, int nrhs) { return phase32(p, nrhs) ? (void*)p->d_phase32 : (void*)p->d_phase; }

void ring(dm_plan* p, int mode, int nrhs, const double* in, double* out, const double* b, hipStream_t s) {
    Timed t(p, KC_RING, s);
    const double* K = mode == RING_ANALYSIS6 ? p->d_tn6 : p->d_K;
    HIPCHK(launch_ring(p, mode, nrhs, in, out, K, b, phase_of(p, nrhs), phase32(p, nrhs), s));
    t.done();
}

// the pixel step of one iteration (eq 9): ring Fourier data of u_x -> the
// messenger t = K u_x + b -> ring Fourier data of t; t_out (nullable)
// receives t.  Diagonal noise runs it in one ring pass per field; 3x3 noise
// couples the three fields of a pixel, which one ring pass holds one at a
// time, so there it is synthesis, then analysis with the 3x3 update applied
// as each field is loaded (from the three fields of u_x), or (when t itself
// is wanted, or with DMWF_FUSE6=0) the update as a pass of its own.
void messenger_step(dm_plan* p, int nrhs, double* t_out, hipStream_t s) {
    if (p->ncov_layout != DM_NCOV_SYM6) {
        ring(p, RING_ITERATE, nrhs, nullptr, t_out, p->d_b, s);
        return;
    }
    ring(p, RING_SYNTH, nrhs, nullptr, p->d_ux, nullptr, s);
    if (!t_out && p->fuse6) {
        ring(p, RING_ANALYSIS6, nrhs, p->d_ux, nullptr, p->d_b, s);
        return;
    }
    {
        Timed t(p, KC_PIXEL, s);
        HIPCHK(launch_update6(p, nrhs, p->d_ux, p->d_b, t_out, s));
        t.done();
    }
    ring(p, RING_ANALYSIS, nrhs, p->d_ux, nullptr, nullptr, s);
}

// analysis + combine: alm = filter(A t) in (T, E, B); spin (nullable)
// receives the same coefficients in the spin basis for the synthesis
// batched matrix-core Legendre kernels: for DM_MIXED from 2 right-hand
// sides on (a single RHS fills 2 of the 16 product columns, and the FP64
// vector kernels are faster: 70 against 51 iterations/s at Nside 1024,
// lmax 2048), for DM_FP64 from 8 on; DMWF_MFMA=0/1 forces it off/on
bool use_mfma(dm_plan* p, int nrhs) {
    if (p->mfma_mode >= 0) return p->mfma_mode == 1;
    return nrhs >= (p->precision == DM_MIXED ? 2 : 8);
}


void leg_analysis(dm_plan* p, int nrhs, bool weighted, const double* filter, double* alm, double* spin,
                  hipStream_t s, double* cpart = nullptr) {
    const void* phase = phase_of(p, nrhs);
    const double* w = weighted ? p->d_pair_w : p->d_pair_one;
    int nslots = p->ana_chunks;
    const bool partial32 = use_mfma(p, nrhs) && p->precision == DM_MIXED;
    {
        Timed t(p, KC_LEG_ANALYSIS, s);
        if (use_mfma(p, nrhs)) {
            p->mfma_nct = 1;
            nslots = batched_analysis_slots(p);
            HIPCHK(launch_bana(p, nrhs, phase, w, p->d_partial, s));
        } else {
            HIPCHK(launch_leg_analysis(p, nrhs, static_cast<const double*>(phase), w, p->d_partial, s));
        }
        t.done();
    }
    Timed t(p, KC_COMBINE, s);
    // every Legendre kernel (vector and matrix-core) carries the scaled
    // recursions mu = lam / S: the scales multiply the partial sums here and
    // the spin-basis copy the synthesis reads
    HIPCHK(launch_combine(p, nrhs, nslots, p->d_partial, partial32, use_mfma(p, nrhs) ? p->d_slot_lo : nullptr,
                          filter, alm, spin, cpart, p->d_scale, s));
    t.done();
}

// synthesis from spin-basis coefficients
void leg_synthesis(dm_plan* p, int nrhs, const double* spin, hipStream_t s) {
    void* phase = phase_of(p, nrhs);
    Timed t(p, KC_LEG_SYNTHESIS, s);
    if (use_mfma(p, nrhs)) {
        p->mfma_nct = 1;
        HIPCHK(launch_bsyn(p, nrhs, spin, phase, s));
    } else {
        HIPCHK(launch_leg_synthesis(p, nrhs, spin, static_cast<double*>(phase), s));
    }
    t.done();
}

// map (device) -> alm (device): A = Y^T W (weighted) or Y^T
void map2alm_dev(dm_plan* p, int nrhs, const double* map, double* alm, bool weighted, hipStream_t s) {
    ring(p, RING_ANALYSIS, nrhs, map, nullptr, nullptr, s);
    leg_analysis(p, nrhs, weighted, nullptr, alm, nullptr, s);
}

void alm2map_dev(dm_plan* p, int nrhs, const double* alm, double* map, hipStream_t s) {
    HIPCHK(launch_to_spin(p, nrhs, alm, p->d_alm_spin, p->d_scale, s));
    leg_synthesis(p, nrhs, p->d_alm_spin, s);
    ring(p, RING_SYNTH, nrhs, nullptr, map, nullptr, s);
}

// the band limit of the transforms launched in a scope (adaptive working
// resolution: a cooling step's limit; 0 = the full band)
struct LcutScope {
    dm_plan* p;
    int saved;
    LcutScope(dm_plan* p_, int lcut) : p(p_), saved(p_->lcut) { p->lcut = lcut; }
    ~LcutScope() { p->lcut = saved; }
};

// band limit of cooling step k of the prepared schedule
int step_lcut(const dm_plan* p, int64_t k) {
    return (k >= 0 && k < (int64_t)p->step_lcut.size()) ? p->step_lcut[k] : 0;
}

// runs the transforms of a scope in another precision (the mixed plan's
// FP64 epilogue: the returned map and the residual)
struct PrecisionScope {
    dm_plan* p;
    dm_precision saved;
    PrecisionScope(dm_plan* p_, dm_precision pr) : p(p_), saved(p_->precision) { p->precision = pr; }
    ~PrecisionScope() { p->precision = saved; }
};

void check_rhs(dm_plan* p, int nrhs) {
    REQUIRE(nrhs >= 1 && nrhs <= p->max_rhs, DM_EINVAL,
            "nrhs must be in [1, max_rhs=" + std::to_string(p->max_rhs) + "]");
}

// The largest l whose prior S_l has an eigenvalue >= mu (-1 if none): above
// it the prior clamped at mu is mu 1 in every field (the truncation of the
// text after eq 9), and the filter carries no signal information.
int ell_iter(const dm_plan* p, double mu) {
    const int L = p->lmax + 1;
    for (int l = p->lmax; l >= 0; --l) {
        const double tt = p->cl[l], ee = p->cl[L + l], bb = p->cl[2 * L + l], te = p->cl[3 * L + l];
        const double h = 0.5 * (tt - ee);
        const double top = std::max(0.5 * (tt + ee) + std::sqrt(h * h + te * te), bb);
        if (top >= mu) return l;
    }
    return -1;
}

// Working band limit of a cooling step (Sec. 4: the working resolution
// follows ell_iter with its Nyquist frequency a little above it):
// min(lmax, max(2, ceil(factor ell_iter))); lmax when adaptive resolution is off.
int working_lmax(const dm_plan* p, double mu, double factor) {
    if (!(factor >= 1.0)) return p->lmax;
    const int li = ell_iter(p, mu);
    const double c = std::ceil(factor * li - 1e-9);
    return (int)std::min<double>(p->lmax, std::max(2.0, c));
}

// upload all cooling-step filters [nsteps][lmax+1][4] for the schedule; with
// `adaptive`, each step's rows above its working band limit are zero (the
// harmonic update u = P_L F t_hat) and the limits go to p->step_lcut
void prepare_filters(dm_plan* p, const std::vector<double>& lambdas, bool adaptive = false) {
    const size_t per = (size_t)(p->lmax + 1) * 4;
    const size_t need = per * lambdas.size();
    if ((int)lambdas.size() > p->filters_cap) {
        dalloc(p, p->d_filters, need);
        p->filters_cap = (int)lambdas.size();
    }
    if (p->h_pinned_len < need) {
        HIPCHK(hipStreamSynchronize(p->stream));
        if (p->h_pinned) (void)hipHostFree(p->h_pinned);
        p->h_pinned = nullptr;
        HIPCHK(hipHostMalloc((void**)&p->h_pinned, need * sizeof(double), hipHostMallocDefault));
        p->h_pinned_len = need;
    }
    std::vector<double> F;
    p->step_lcut.assign(lambdas.size(), p->lmax);
    for (size_t k = 0; k < lambdas.size(); ++k) {
        const double mu = (lambdas[k] - 1.0) * p->tau;
        build_filter(p->cl, p->lmax, mu, p->tau, F);
        if (adaptive) {
            const int L = working_lmax(p, mu, p->adaptive);
            p->step_lcut[k] = L;
            for (size_t i = (size_t)(L + 1) * 4; i < per; ++i) F[i] = 0.0;
        }
        std::memcpy(p->h_pinned + k * per, F.data(), per * sizeof(double));
    }
    HIPCHK(hipMemcpyAsync(p->d_filters, p->h_pinned, need * sizeof(double), hipMemcpyHostToDevice, p->stream));
}

bool eps_mode(const dm_schedule& sc) { return sc.iters_per_step <= 0; }

std::vector<double> schedule_lambdas(const dm_schedule& sc) {
    if (eps_mode(sc)) {
        // lambda_j = lambda_start beta^j while above 1, then 1
        std::vector<double> lam;
        for (double v = sc.lambda_start; v > 1.0; v *= sc.beta) lam.push_back(v);
        lam.push_back(1.0);
        return lam;
    }
    std::vector<double> lam(sc.nsteps, 1.0);
    if (sc.nsteps > 1)
        for (int k = 0; k < sc.nsteps - 1; ++k)
            lam[k] = std::pow(sc.lambda_start, 1.0 - (double)k / (sc.nsteps - 1));
    return lam;
}

void sync_plan_stream_to(dm_plan* p, hipStream_t s) {
    if (s == p->stream) return;
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipEventRecord(e, p->stream));
    HIPCHK(hipStreamWaitEvent(s, e, 0));
    HIPCHK(hipEventDestroy(e));
}

// Fixed-mode cooling steps run as HIP graphs: the step's iterations (all but
// the solve's last) are recorded on the plan's own stream (capture is not
// possible on the legacy default stream a caller may pass) and launched on
// s.  The executable graphs are kept until the solve has synchronised.
// Profiling (per-kernel events) and DMWF_GRAPHS=0 run the launches directly.
struct StepGraphs {
    hipStream_t s;
    std::vector<hipGraphExec_t> keep;
    explicit StepGraphs(hipStream_t st) : s(st) {}
    ~StepGraphs() {
        if (keep.empty()) return;
        (void)hipStreamSynchronize(s);          // every launch has finished (also on error paths)
        for (hipGraphExec_t e : keep) (void)hipGraphExecDestroy(e);
    }
};

void messenger_step(dm_plan* p, int nrhs, double* t_out, hipStream_t s);

// Diagnostics of the iterate (Fig. 4), with the FP64 transforms in either
// precision: chi^2 = (d0 - Y u)^T P (d0 - Y u) + u^T S^+ u (eq 3) and the
// Appendix C residual ||S^+1/2 u + S^1/2 Y^T P (Y u - d0)|| / ||S^1/2 Y^T P d0||.
// diag_prepare computes -Y^T P d0 into d_alm_y once per solve (only its norm
// through S^1/2 enters); diag_record evaluates both for u = alm after
// iteration `iter`.  Both run between an iteration's analysis and its
// synthesis, where the map and ring buffers they use hold nothing live.
void diag_prepare(dm_plan* p, int nrhs, hipStream_t s) {
    PrecisionScope fp64(p, DM_FP64);
    LcutScope full(p, 0);
    HIPCHK(hipMemsetAsync(p->d_ux, 0, (size_t)nrhs * 3 * p->npix * sizeof(double), s));
    HIPCHK(launch_residual_maps(p, nrhs, p->d_ux, p->d_d0, nullptr, p->d_red + 64, s));
    map2alm_dev(p, nrhs, p->d_ux, p->d_alm_y, false, s);
}

void diag_record(dm_plan* p, int nrhs, const double* alm, int64_t iter, hipStream_t s) {
    PrecisionScope fp64(p, DM_FP64);
    LcutScope full(p, 0);
    alm2map_dev(p, nrhs, alm, p->d_ux, s);
    double* chi = p->d_red + 64;
    HIPCHK(launch_residual_maps(p, nrhs, p->d_ux, p->d_d0, nullptr, chi, s));
    map2alm_dev(p, nrhs, p->d_ux, p->d_alm_r, false, s);
    const int nb = alm_norm_blocks(p);
    double* parts = chi + (int64_t)nrhs * p->nrings;
    HIPCHK(launch_alm_norms(p, nrhs, alm, nullptr, p->d_alm_r, p->d_alm_y, p->d_mats, parts, s));
    std::vector<double> hchi((size_t)nrhs * p->nrings), hparts((size_t)nrhs * nb * kNormQ);
    HIPCHK(hipMemcpyAsync(hchi.data(), chi, hchi.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hparts.data(), parts, hparts.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    p->diag_iter.push_back((int)iter);
    for (int r = 0; r < nrhs; ++r) {
        double q[kNormQ] = {0, 0, 0, 0, 0};
        for (int b = 0; b < nb; ++b)
            for (int k = 0; k < kNormQ; ++k) q[k] += hparts[((size_t)r * nb + b) * kNormQ + k];
        double c = 0;
        for (int j = 0; j < p->nrings; ++j) c += hchi[(size_t)r * p->nrings + j];
        p->diag_chi2.push_back(c + q[4]);
        p->diag_resid.push_back(q[3] > 0 ? std::sqrt(q[2] / q[3]) : 0.0);
    }
}

// one more iteration of the solve has produced alm: record it if due
void diag_after_analysis(dm_plan* p, int nrhs, const double* alm, bool last, hipStream_t s) {
    if (!p->diag_active) return;
    ++p->diag_count;
    if (last || p->diag_count % p->diag_every == 0) diag_record(p, nrhs, alm, p->diag_count, s);
}

void run_iterations(dm_plan* p, int nrhs, const double* F, double* alm, int count, hipStream_t s, StepGraphs& g) {
    if (p->diag_active) {
        // traced: direct launches, the iterate stored after every analysis
        for (int i = 0; i < count; ++i) {
            leg_analysis(p, nrhs, true, F, alm, p->d_alm_spin, s);
            diag_after_analysis(p, nrhs, alm, false, s);
            leg_synthesis(p, nrhs, p->d_alm_spin, s);
            messenger_step(p, nrhs, nullptr, s);
        }
        return;
    }
    auto body = [&](hipStream_t st) {
        for (int i = 0; i < count; ++i) {
            // t_hat = A t ; u = F t_hat   (eq 8) ; u_x = Y u ; t = K u_x + b ; next t_hat's ring data (eq 9).
            // The next synthesis reads u through the spin-basis copy, so u
            // itself is stored only by the run's last iteration
            leg_analysis(p, nrhs, true, F, i == count - 1 ? alm : nullptr, p->d_alm_spin, st);
            leg_synthesis(p, nrhs, p->d_alm_spin, st);
            messenger_step(p, nrhs, nullptr, st);
        }
    };
    if (count <= 0) return;
    if (!p->graphs || p->profiling || count < 2) {
        body(s);
        return;
    }
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    try {
        body(p->stream);
    } catch (...) {
        (void)hipStreamEndCapture(p->stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    HIPCHK(hipStreamEndCapture(p->stream, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t st = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(st);
    g.keep.push_back(exec);
    HIPCHK(hipGraphLaunch(exec, s));
}

// fingerprint of a device buffer (blocks on s)
uint64_t device_hash(dm_plan* p, const void* buf, int64_t n, int elem_bytes, hipStream_t s) {
    uint64_t* acc = reinterpret_cast<uint64_t*>(p->d_red + 8);
    HIPCHK(hipMemsetAsync(acc, 0, sizeof(uint64_t), s));
    HIPCHK(launch_hash(buf, n, elem_bytes, acc, s));
    uint64_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, acc, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return hash_mix(h ^ (uint64_t)n);
}

// the same fingerprint of host doubles
uint64_t host_hash(const double* x, size_t n) {
    uint64_t h = 0;
    for (size_t i = 0; i < n; ++i) {
        uint64_t v;
        std::memcpy(&v, x + i, sizeof v);
        h += hash_mix(v + (uint64_t)i * 0x9E3779B97F4A7C15ull);
    }
    return hash_mix(h ^ (uint64_t)n);
}

// two schedules that produce the same iterates (max_iters only stops early)
bool same_schedule(const dm_schedule& a, const dm_schedule& b) {
    if (eps_mode(a) != eps_mode(b) || a.lambda_start != b.lambda_start) return false;
    if (!eps_mode(a)) return a.nsteps == b.nsteps && a.iters_per_step == b.iters_per_step;
    return a.beta == b.beta && a.eps_start == b.eps_start && a.eps_end == b.eps_end && a.eps_eta == b.eps_eta;
}

// The dual messenger solve on device buffers (Algorithm 1).
//   d: [nrhs][3][npix] device; alm: [nrhs][3][nalm] complex device;
//   map: nullable device [nrhs][3][npix] (receives Y u).
// resumable: a Wiener filter solve, which continues a loaded checkpoint
// and leaves its own state for dm_checkpoint_save.
// Iterations [from, end) of the fixed schedule on the iterate alm, from the
// ring Fourier data of the current messenger t; the solve's last iteration
// keeps the previous iterate in d_alm_prev and ends with u_x = Y u in d_ux.
void fixed_loop(dm_plan* p, int nrhs, double* alm, int64_t from, int64_t end, hipStream_t s, StepGraphs& graphs) {
    const size_t per = (size_t)(p->lmax + 1) * 4;
    const int niter = p->sched.iters_per_step;
    const size_t alm_bytes = (size_t)nrhs * 3 * p->nalm * 2 * sizeof(double);
    for (int64_t it = from; it < end;) {
        const int64_t k = it / niter;
        const double* F = p->d_filters + per * k;
        LcutScope band(p, step_lcut(p, k));
        // this cooling step's iterations before the solve's last one
        const int64_t stop = std::min<int64_t>((k + 1) * niter, end - 1);
        if (it < stop) {
            run_iterations(p, nrhs, F, alm, (int)(stop - it), s, graphs);
            it = stop;
            continue;
        }
        // the last iteration: keep the previous iterate (final Cauchy
        // ratio) and end with u_x = Y u
        HIPCHK(hipMemcpyAsync(p->d_alm_prev, alm, alm_bytes, hipMemcpyDeviceToDevice, s));
        leg_analysis(p, nrhs, true, F, alm, p->d_alm_spin, s);
        diag_after_analysis(p, nrhs, alm, true, s);
        leg_synthesis(p, nrhs, p->d_alm_spin, s);
        ring(p, RING_SYNTH, nrhs, nullptr, p->d_ux, nullptr, s);
        ++it;
    }
}

// The messenger run with counts[k] iterations at cooling step k (the
// iterations an epsilon-mode solve spent there), from the ring Fourier data
// of the current messenger; it ends like fixed_loop.
void counted_loop(dm_plan* p, int nrhs, double* alm, const std::vector<int>& counts, hipStream_t s,
                  StepGraphs& graphs) {
    const size_t per = (size_t)(p->lmax + 1) * 4;
    const size_t alm_bytes = (size_t)nrhs * 3 * p->nalm * 2 * sizeof(double);
    int64_t total = 0, done = 0;
    for (int c : counts) total += c;
    for (size_t k = 0; k < counts.size(); ++k) {
        if (counts[k] <= 0) continue;
        const double* F = p->d_filters + per * k;
        LcutScope band(p, step_lcut(p, (int64_t)k));
        const bool last_step = done + counts[k] == total;
        const int run = last_step ? counts[k] - 1 : counts[k];
        run_iterations(p, nrhs, F, alm, run, s, graphs);
        done += run;
        if (last_step) {
            HIPCHK(hipMemcpyAsync(p->d_alm_prev, alm, alm_bytes, hipMemcpyDeviceToDevice, s));
            leg_analysis(p, nrhs, true, F, alm, p->d_alm_spin, s);
            leg_synthesis(p, nrhs, p->d_alm_spin, s);
            ring(p, RING_SYNTH, nrhs, nullptr, p->d_ux, nullptr, s);
            ++done;
        }
    }
}

// Appendix A's refinement (a modified Jacobi relaxation), on the sphere:
// with W~ the fixed-schedule messenger run, p->refine corrections
//   s <- s + W~(g),  g = W Y r,  r = Pi Y^T P (d0 - Y s) - S^+ s,
// r the residual of the Wiener filter equation on the range of S (FP64
// transforms, whatever the plan's precision) and W Y a right inverse of the
// adjoint Y^T where the quadrature is exact.  W~(g) runs the same schedule
// from t = 0 with b = T_p g = -tau Y r~ (r~ = -r), so that every correction
// applies one linear operator, and its fixed point solves the Wiener filter
// equation exactly.  Records ||r|| / ||Pi Y^T P d0|| before each correction
// and after the last in p->refine_hist.  Returns the last iterate, as
// Appendix A's relaxation does, or with p->refine_best per RHS the iterate
// of smallest residual norm (the first of equal ones): the corrections
// converge only where W~ is close enough to the inverse.  p->refine_chosen
// records which one each RHS returned.
void refine_dev(dm_plan* p, int nrhs, double* alm, int64_t full, const std::vector<int>* counts, hipStream_t s) {
    const int64_t na2 = (int64_t)nrhs * 3 * p->nalm * 2;
    const int64_t nmap = (int64_t)nrhs * 3 * p->npix;
    const size_t alm_bytes = (size_t)na2 * sizeof(double);
    const int nb = alm_norm_blocks(p);
    double* parts = p->d_red + 64 + (int64_t)nrhs * p->nrings;
    std::vector<double> hparts((size_t)nrhs * nb * 2), ynorm(nrhs, 0.0);
    p->refine_hist.assign((size_t)(p->refine + 1) * nrhs, 0.0);
    p->refine_nrhs = nrhs;
    // r~ = -r into d_alm_r, its relative norm into refine_hist[k]
    auto residual = [&](int k) {
        PrecisionScope fp64(p, DM_FP64);
        alm2map_dev(p, nrhs, alm, p->d_ux, s);
        // d_ux <- P (Y s - d0); d_b2 <- P d0 (used at k = 0)
        HIPCHK(launch_residual_maps(p, nrhs, p->d_ux, p->d_d0, p->d_b2, p->d_red + 64, s));
        map2alm_dev(p, nrhs, p->d_ux, p->d_alm_r, false, s);
        if (k == 0) map2alm_dev(p, nrhs, p->d_b2, p->d_alm_y, false, s);
        HIPCHK(launch_refine_residual(p, nrhs, p->d_alm_r, alm, k == 0 ? p->d_alm_y : nullptr, parts, s));
        HIPCHK(hipMemcpyAsync(hparts.data(), parts, hparts.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int r = 0; r < nrhs; ++r) {
            double q0 = 0.0, q1 = 0.0;
            for (int b = 0; b < nb; ++b) {
                q0 += hparts[((size_t)r * nb + b) * 2];
                q1 += hparts[((size_t)r * nb + b) * 2 + 1];
            }
            if (k == 0) ynorm[r] = std::sqrt(q1);
            p->refine_hist[(size_t)k * nrhs + r] = ynorm[r] > 0.0 ? std::sqrt(q0) / ynorm[r] : 0.0;
        }
    };
    // with refine_best: the best iterate so far per RHS (smallest residual
    // norm), returned at the end
    std::vector<double> best_r(nrhs);
    p->refine_chosen.assign(nrhs, 0);
    const size_t slice = (size_t)3 * p->nalm * 2;
    auto keep_best = [&](int k) {
        for (int r = 0; r < nrhs; ++r) {
            const double h = p->refine_hist[(size_t)k * nrhs + r];
            if (!p->refine_best) {
                p->refine_chosen[r] = k;
                continue;
            }
            if (k > 0 && !(h < best_r[r])) continue;
            best_r[r] = h;
            p->refine_chosen[r] = k;
            HIPCHK(hipMemcpyAsync(p->d_alm_best + slice * r, alm + slice * r, slice * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
        }
    };
    residual(0);
    keep_best(0);
    for (int n = 0; n < p->refine; ++n) {
        // d_alm_r holds r~ of the current iterate
        {
            PrecisionScope fp64(p, DM_FP64);
            alm2map_dev(p, nrhs, p->d_alm_r, p->d_ux, s);
        }
        HIPCHK(launch_scale(p->d_b2, p->d_ux, -p->tau, nmap, s));
        // W~(g): the schedule from t = 0, with b = d_b2 in place of the data's
        std::swap(p->d_b, p->d_b2);
        try {
            HIPCHK(hipMemsetAsync(p->d_ux, 0, (size_t)nmap * sizeof(double), s));
            ring(p, RING_ANALYSIS, nrhs, p->d_ux, nullptr, nullptr, s);
            HIPCHK(hipMemsetAsync(p->d_alm_corr, 0, alm_bytes, s));
            StepGraphs graphs(s);
            if (counts)
                counted_loop(p, nrhs, p->d_alm_corr, *counts, s, graphs);
            else
                fixed_loop(p, nrhs, p->d_alm_corr, 0, full, s, graphs);
        } catch (...) {
            std::swap(p->d_b, p->d_b2);
            throw;
        }
        std::swap(p->d_b, p->d_b2);
        HIPCHK(launch_axpby(alm, p->d_alm_corr, 1.0, 1.0, na2, s));
        residual(n + 1);
        keep_best(n + 1);
    }
    if (p->refine_best) HIPCHK(hipMemcpyAsync(alm, p->d_alm_best, alm_bytes, hipMemcpyDeviceToDevice, s));
}

void solve_dev(dm_plan* p, int nrhs, const double* d, double* alm, double* map, hipStream_t s, dm_stats* stats,
               bool resumable) {
    REQUIRE(p->noise_set, DM_ESTATE, "dm_set_noise must be called before solving");
    REQUIRE(p->spectra_set, DM_ESTATE, "dm_set_spectra must be called before solving");
    check_rhs(p, nrhs);
    const auto t0 = std::chrono::steady_clock::now();
    if (p->refine > 0) {
        REQUIRE(eps_mode(p->sched) || p->sched.max_iters <= 0, DM_EUNSUPPORTED,
                "refinement does not combine with an iteration cap on the fixed schedule");
        REQUIRE(!p->resume.pending, DM_EUNSUPPORTED, "refinement does not resume from a checkpoint");
        // a refined solve leaves nothing to checkpoint
        p->state.valid = false;
        resumable = false;
    }
    const std::vector<double> lam = schedule_lambdas(p->sched);
    prepare_filters(p, lam, p->adaptive >= 1.0);
    sync_plan_stream_to(p, s);
    const size_t per = (size_t)(p->lmax + 1) * 4;
    const int64_t alm_len = (int64_t)nrhs * 3 * p->nalm * 2;
    const size_t alm_bytes = (size_t)alm_len * sizeof(double);
    if (resumable) p->state.valid = false;
    StepGraphs graphs(s);

    // setup: d0 = mask(d), b = T N^-1 d0
    HIPCHK(launch_data_setup(p, nrhs, d, p->d_d0, p->d_b, s));
    // diagnostics trace of this solve's own iterations (a resumed solve
    // counts on from its checkpoint)
    p->diag_active = false;
    p->diag_iter.clear();
    p->diag_chi2.clear();
    p->diag_resid.clear();
    p->diag_nrhs = nrhs;
    if (p->diag_every > 0) {
        diag_prepare(p, nrhs, s);
        p->diag_count = (resumable && p->resume.pending) ? p->resume.st.iterations : 0;
        p->diag_active = true;
    }
    const int nsteps = (int)lam.size();
    const bool eps = eps_mode(p->sched);
    const uint64_t hash_data = resumable ? device_hash(p, p->d_d0, (int64_t)nrhs * 3 * p->npix, 8, s) : 0;

    // a loaded checkpoint: the same inputs and schedule, then its iterate
    dm_plan::Resume* rs = (resumable && p->resume.pending) ? &p->resume : nullptr;
    if (rs) {
        REQUIRE(rs->st.nrhs == nrhs, DM_EINVAL,
                "the loaded checkpoint holds " + std::to_string(rs->st.nrhs) + " right-hand sides, not " +
                    std::to_string(nrhs));
        REQUIRE(same_schedule(rs->st.sched, p->sched), DM_EINVAL, "the schedule differs from the checkpoint's");
        REQUIRE(rs->st.hash_data == hash_data, DM_EINVAL, "the data differ from the checkpoint's");
        REQUIRE(p->hash_noise == rs->st.hash_noise && p->hash_cl == rs->st.hash_cl, DM_EINVAL,
                "the noise or the spectra differ from the checkpoint's");
        HIPCHK(hipMemcpyAsync(alm, rs->u.data(), alm_bytes, hipMemcpyHostToDevice, s));
        if (rs->has_prev)
            HIPCHK(hipMemcpyAsync(p->d_alm_prev, rs->uprev.data(), alm_bytes, hipMemcpyHostToDevice, s));
    }
    // resuming from u: the ring Fourier data of the next messenger t (or, with
    // nothing left to run, the final Y u), by the same kernels an
    // uninterrupted run uses after its analysis, so the result is the same to
    // the last bit
    auto restart_from_u = [&](bool final_map) {
        HIPCHK(launch_to_spin(p, nrhs, alm, p->d_alm_spin, p->d_scale, s));
        leg_synthesis(p, nrhs, p->d_alm_spin, s);
        if (final_map)
            ring(p, RING_SYNTH, nrhs, nullptr, p->d_ux, nullptr, s);
        else
            messenger_step(p, nrhs, nullptr, s);
    };
    if (!rs) {
        // t_0 = d0; u_0 = 0 (the reference of the first Cauchy ratio)
        ring(p, RING_ANALYSIS, nrhs, p->d_d0, nullptr, nullptr, s);
        HIPCHK(hipMemsetAsync(alm, 0, alm_bytes, s));
    }
    std::vector<double> last_c(nrhs, 0.0);
    int64_t total = rs ? rs->st.iterations : 0;
    int next_step = 0;
    bool finished = false;
    if (!eps) {
        const int niter = p->sched.iters_per_step;
        const int64_t full = (int64_t)nsteps * niter;
        const int64_t end = p->sched.max_iters > 0 ? std::min<int64_t>(full, p->sched.max_iters) : full;
        if (rs) restart_from_u(total >= end);
        fixed_loop(p, nrhs, alm, total, end, s, graphs);
        p->diag_active = false;
        total = std::max(total, end);
        finished = total >= full;
        if (p->refine > 0) {
            refine_dev(p, nrhs, alm, full, nullptr, s);
            total *= 1 + p->refine;
        }
    } else {
        // Algorithm 1's loop: per cooling step, repeat until the Cauchy ratio
        // (largest over the RHS) is below that step's threshold.  The ratio
        // of iteration i comes from the combine kernel; the host reads it
        // while the GPU runs the iteration's synthesis, then picks the ring
        // step: the pixel update, or (at the end) the final map.
        const dm_schedule& sc = p->sched;
        struct Ev {
            hipEvent_t e = nullptr;
            ~Ev() { if (e) (void)hipEventDestroy(e); }
        } ev;
        HIPCHK(hipEventCreateWithFlags(&ev.e, hipEventDisableTiming));
        int k0 = 0;
        bool done = false;
        if (rs) {
            p->trace_cauchy = rs->trace_cauchy;
            p->trace_step = rs->trace_step;
            last_c = rs->st.last_c;
            k0 = rs->st.next_step;
            finished = rs->st.finished;
            done = finished || total >= sc.max_iters;
            restart_from_u(done);
        } else {
            p->trace_cauchy.clear();
            p->trace_step.clear();
        }
        next_step = k0;
        for (int k = k0; k < nsteps && !done; ++k) {
            const double* F = p->d_filters + per * k;
            LcutScope band(p, step_lcut(p, k));
            const double thr = (k == nsteps - 1) ? sc.eps_end
                                                 : std::max(sc.eps_end, sc.eps_start * std::pow(sc.eps_eta, -(double)k));
            for (;;) {
                leg_analysis(p, nrhs, true, F, alm, p->d_alm_spin, s, p->d_cpart);
                HIPCHK(launch_cauchy_reduce(p, nrhs, p->d_cpart, p->d_cout, s));
                HIPCHK(hipMemcpyAsync(p->h_cout, p->d_cout, (size_t)nrhs * 2 * sizeof(double), hipMemcpyDeviceToHost,
                                      s));
                HIPCHK(hipEventRecord(ev.e, s));
                // traced: the diagnostics of this iterate go before its
                // synthesis, once the ratio says whether it is the last
                if (!p->diag_active) leg_synthesis(p, nrhs, p->d_alm_spin, s);
                HIPCHK(hipEventSynchronize(ev.e));
                double c = 0.0;
                for (int r = 0; r < nrhs; ++r) {
                    const double num = p->h_cout[2 * r], den = p->h_cout[2 * r + 1];
                    last_c[r] = den > 0.0 ? std::sqrt(num / den) : 0.0;
                    c = std::max(c, last_c[r]);
                }
                REQUIRE(std::isfinite(c), DM_ENONFINITE, "the iterate became non-finite");
                p->trace_cauchy.push_back(c);
                p->trace_step.push_back(k);
                ++total;
                const bool conv = c < thr;
                next_step = conv ? k + 1 : k;
                finished = conv && k == nsteps - 1;
                if (p->diag_active) {
                    diag_after_analysis(p, nrhs, alm, finished || total >= sc.max_iters, s);
                    leg_synthesis(p, nrhs, p->d_alm_spin, s);
                }
                if (finished || total >= sc.max_iters) {
                    ring(p, RING_SYNTH, nrhs, nullptr, p->d_ux, nullptr, s);
                    done = true;
                    break;
                }
                messenger_step(p, nrhs, nullptr, s);
                if (conv) break;
            }
        }
        p->diag_active = false;
        if (p->refine > 0) {
            // Appendix A's prescription: every correction runs the
            // iterations this solve spent at each cooling step
            std::vector<int> counts(nsteps, 0);
            for (int k : p->trace_step) ++counts[k];
            refine_dev(p, nrhs, alm, 0, &counts, s);
            total *= 1 + p->refine;
        }
    }
    if (resumable) {
        // where this solve stopped, for dm_checkpoint_save
        HIPCHK(hipMemcpyAsync(p->d_state_u, alm, alm_bytes, hipMemcpyDeviceToDevice, s));
        dm_plan::SolveState& st = p->state;
        st.nrhs = nrhs;
        st.iterations = total;
        st.next_step = next_step;
        st.finished = finished;
        st.hash_data = hash_data;
        st.hash_noise = p->hash_noise;
        st.hash_cl = p->hash_cl;
        st.sched = p->sched;
        st.last_c = last_c;
    }
    // epilogue in FP64 (section a8): a mixed plan recomputes s_x = Y u with
    // the FP64 transforms before it is returned or enters the residual
    std::unique_ptr<PrecisionScope> fp64;
    if ((p->precision == DM_MIXED || p->refine > 0) && (map || stats)) {
        fp64.reset(new PrecisionScope(p, DM_FP64));
        alm2map_dev(p, nrhs, alm, p->d_ux, s);
    }
    if (map) HIPCHK(hipMemcpyAsync(map, p->d_ux, (size_t)nrhs * 3 * p->npix * sizeof(double),
                                   hipMemcpyDeviceToDevice, s));
    // non-finite check of the iterate
    int* d_cnt = reinterpret_cast<int*>(p->d_red);
    HIPCHK(hipMemsetAsync(d_cnt, 0, sizeof(int), s));
    HIPCHK(launch_count_nonfinite(alm, alm_len, d_cnt, s));
    int cnt = 0;
    if (stats) {
        // residual maps, their adjoints, and the norms
        double* chi = p->d_red + 64;
        HIPCHK(launch_residual_maps(p, nrhs, p->d_ux, p->d_d0, p->d_b, chi, s));
        map2alm_dev(p, nrhs, p->d_ux, p->d_alm_r, false, s);
        map2alm_dev(p, nrhs, p->d_b, p->d_alm_y, false, s);
        const int nb = alm_norm_blocks(p);
        double* parts = chi + (int64_t)nrhs * p->nrings;
        HIPCHK(launch_alm_norms(p, nrhs, alm, (eps || p->refine > 0) ? nullptr : p->d_alm_prev, p->d_alm_r, p->d_alm_y,
                                p->d_mats,
                                parts, s));
        std::vector<double> hchi((size_t)nrhs * p->nrings), hparts((size_t)nrhs * nb * kNormQ);
        HIPCHK(hipMemcpyAsync(hchi.data(), chi, hchi.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hparts.data(), parts, hparts.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&cnt, d_cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int r = 0; r < nrhs; ++r) {
            double q[kNormQ] = {0, 0, 0, 0, 0};
            for (int b = 0; b < nb; ++b)
                for (int k = 0; k < kNormQ; ++k) q[k] += hparts[((size_t)r * nb + b) * kNormQ + k];
            double c = 0;
            for (int j = 0; j < p->nrings; ++j) c += hchi[(size_t)r * p->nrings + j];
            stats[r].iterations = (int)total;
            stats[r].cauchy = p->refine > 0 ? 0.0 : eps ? last_c[r] : (q[1] > 0 ? std::sqrt(q[0] / q[1]) : 0.0);
            stats[r].residual = q[3] > 0 ? std::sqrt(q[2] / q[3]) : 0.0;
            stats[r].chi2 = c + q[4];
            stats[r].seconds = secs;
        }
    } else {
        HIPCHK(hipMemcpyAsync(&cnt, d_cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (p->profiling) collect_events(p);
    REQUIRE(cnt == 0, DM_ENONFINITE, "the iterate became non-finite");
    if (rs) p->resume = dm_plan::Resume();
    if (resumable) p->state.valid = true;
}

void free_plan(dm_plan* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    for (size_t i = 0; i < p->ev.start.size(); ++i) {
        (void)hipEventDestroy(p->ev.start[i]);
        (void)hipEventDestroy(p->ev.stop[i]);
    }
    dfree(p->d_pair_x); dfree(p->d_pair_w); dfree(p->d_pair_one); dfree(p->d_pairs); dfree(p->d_fftlen);
    dfree(p->d_plist_whole); dfree(p->d_plist_split); dfree(p->d_plist_small); dfree(p->d_plist_big);
    dfree(p->d_chirp); dfree(p->d_bhat); dfree(p->d_tw);
    dfree(p->d_tw3); dfree(p->d_tw332);
    dfree(p->d_chirp32); dfree(p->d_bhat32); dfree(p->d_tw32); dfree(p->d_coef); dfree(p->d_coef_s); dfree(p->d_scale); dfree(p->d_lstart); dfree(p->d_slot_lo); dfree(p->d_seed);
    dfree(p->d_lp0); dfree(p->d_lp2); dfree(p->d_K); dfree(p->d_tn); dfree(p->d_ninv); dfree(p->d_obs);
    dfree(p->d_ninv6); dfree(p->d_tn6); dfree(p->d_state_u);
    dfree(p->d_ring_w); dfree(p->d_ring_off); dfree(p->d_ring_n); dfree(p->d_phase); dfree(p->d_phase32); dfree(p->d_partial);
    dfree(p->d_alm); dfree(p->d_alm_prev); dfree(p->d_alm_spin); dfree(p->d_d0); dfree(p->d_b); dfree(p->d_ux); dfree(p->d_alm_r);
    dfree(p->d_alm_y); dfree(p->d_filters); dfree(p->d_mats); dfree(p->d_red);
    dfree(p->d_b2); dfree(p->d_alm_corr); dfree(p->d_alm_best);
    dfree(p->d_cpart); dfree(p->d_cout);
    if (p->h_cout) (void)hipHostFree(p->h_cout);
    if (p->h_pinned) (void)hipHostFree(p->h_pinned);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

template <class F>
dm_status guarded(dm_plan* p, F&& f) {
    if (!p) return DM_EINVAL;
    try {
        HIPCHK(hipSetDevice(p->device));
        p->err.clear();
        f();
        return DM_OK;
    } catch (const Fail& e) {
        return e.st;
    } catch (const std::bad_alloc&) {
        p->err = "host allocation failed";
        return DM_ENOMEM;
    } catch (...) {
        p->err = "internal error";
        return DM_EDEVICE;
    }
}

}  // namespace

// ==========================================================================
// ABI
// ==========================================================================
extern "C" {

int dm_abi_version(void) { return DMWF_ABI_VERSION; }

int dm_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

const char* dm_last_error(const dm_plan* p) { return p ? p->err.c_str() : g_create_err.c_str(); }

dm_status dm_plan_create(dm_plan** out, const dm_grid* grid, int lmax, int max_rhs, dm_precision precision,
                         int device) {
    g_create_err.clear();
    if (!out || !grid) {
        g_create_err = "null argument";
        return DM_EINVAL;
    }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        g_create_err = "no HIP device available";
        return DM_EDEVICE;
    }
    if (device < 0 || device >= ndev) {
        g_create_err = "device index out of range";
        return DM_EINVAL;
    }
    dm_plan* p = new (std::nothrow) dm_plan();
    if (!p) {
        g_create_err = "host allocation failed";
        return DM_ENOMEM;
    }
    p->device = device;
    p->grid = *grid;
    p->lmax = lmax;
    p->mmax = lmax;
    p->max_rhs = max_rhs;
    p->precision = precision;
    try {
        HIPCHK(hipSetDevice(device));
        scratch_setup(device);
        REQUIRE(precision == DM_FP64 || precision == DM_MIXED, DM_EINVAL, "unknown precision");
        REQUIRE(max_rhs >= 1 && max_rhs <= 4096, DM_EINVAL, "max_rhs must be in [1, 4096]");
        REQUIRE(lmax >= 2 && lmax <= 16384, DM_EINVAL, "lmax must be in [2, 16384]");
        std::string e;
        REQUIRE(build_rings(*grid, p->rings, p->npix, e), DM_EINVAL, e);
        if (grid->kind == DM_GRID_HEALPIX_RING)
            REQUIRE(lmax <= 3 * grid->nside - 1, DM_EINVAL, "lmax must be <= 3 nside - 1 on HEALPix");
        else
            REQUIRE(lmax <= grid->ntheta - 1 && 2 * lmax + 1 <= grid->nphi, DM_EINVAL,
                    "Gauss-Legendre needs ntheta >= lmax + 1 and nphi >= 2 lmax + 1");
        p->nrings = (int)p->rings.z.size();
        p->npairs = (int)p->rings.pair_n.size();
        p->nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
        // the largest padded FP64 transform buffer within one workgroup's
        // 160 KB of LDS (DMWF_FFT_MAX_ELEMS lowers it, to exercise the split
        // transform on small grids)
        const int max_elems = std::max(8, std::min(8192, env_int("DMWF_FFT_MAX_ELEMS", 8192)));
        REQUIRE(build_fft_tables(p->rings, p->mmax, max_elems, p->fft, e), DM_EINVAL, e);
        for (size_t i = 0; i < p->fft.n.size(); ++i) {
            if (!p->fft.split[i]) continue;
            const int i4 = p->fft.n[i] / 4;
            REQUIRE(i4 <= 4 * p->fft_threads, DM_EUNSUPPORTED,
                    "ring length " + std::to_string(p->fft.n[i]) + " is too long for the split transform");
            if (i4 > 2 * p->fft_threads) p->split_k = 4;
        }
        const int lds_max = std::max(p->fft.lds_elems, p->fft.lds_split);
        p->fft_lds_bytes = (size_t)(lds_max + lds_max / 8 + 32) * 16;  // padded layout (ringfft.hip)
        REQUIRE(p->fft_lds_bytes <= 160 * 1024, DM_EUNSUPPORTED,
                "ring length needs a transform buffer of " + std::to_string(lds_max) +
                    " points, beyond the LDS of one workgroup in double precision");
        // Whole-ring workgroups: when one transform buffer takes more than
        // half the LDS, a CU holds one workgroup, and 1024 threads (four
        // waves per SIMD) hide more LDS latency than 512; otherwise two
        // 512-thread workgroups fit.  DMWF_RING_THREADS overrides (256, 512
        // or 1024).
        p->ring_threads = p->fft_lds_bytes > 80 * 1024 ? 1024 : 512;
        {
            const int rt = env_int("DMWF_RING_THREADS", 0);
            if (rt == 256 || rt == 512 || rt == 1024) p->ring_threads = rt;
            const int rb = env_int("DMWF_RING_BIG_THREADS", 1024), rs = env_int("DMWF_RING_SMALL_THREADS", 512);
            if (rb == 256 || rb == 512 || rb == 1024) p->ring_big_threads = rb;
            if (rs == 256 || rs == 512 || rs == 1024) p->ring_small_threads = rs;
            const int sw = env_int("DMWF_SYN_WAVES", 4);
            if (sw == 1 || sw == 2 || sw == 4 || sw == 8) p->syn_waves = sw;
        }
        HIPCHK(hipStreamCreate(&p->stream));
        p->graphs = env_int("DMWF_GRAPHS", 1) != 0;
        p->fuse6 = env_int("DMWF_FUSE6", 1) != 0;

        // ring and pair tables
        std::vector<double> px(p->npairs), pw(p->npairs), one(p->npairs, 1.0);
        std::vector<RingPairDev> pd(p->npairs);
        for (int q = 0; q < p->npairs; ++q) {
            const int rn = p->rings.pair_n[q], rs = p->rings.pair_s[q];
            px[q] = p->rings.z[rn];
            pw[q] = p->rings.w[rn];
            RingPairDev& d = pd[q];
            d.nphi = p->rings.nphi[rn];
            d.len_idx = (int)(std::lower_bound(p->fft.n.begin(), p->fft.n.end(), d.nphi) - p->fft.n.begin());
            d.has_s = rs >= 0;
            d.off_n = p->rings.offset[rn];
            d.off_s = rs >= 0 ? p->rings.offset[rs] : 0;
            // phi0 = pi / den for HEALPix (den = 4i or 4 nside), 0 otherwise
            d.phi0_den = 0;
            const double ph = p->rings.phi0[rn];
            if (ph > 0) d.phi0_den = (int)std::lround(M_PI / ph);
        }
        std::vector<FftLenDev> fl(p->fft.n.size());
        for (size_t i = 0; i < fl.size(); ++i) {
            fl[i].n = p->fft.n[i];
            fl[i].M = p->fft.M[i];
            fl[i].logM = p->fft.logM[i];
            fl[i].bluestein = p->fft.chirp_off[i] >= 0;
            fl[i].split = p->fft.split[i];
            fl[i].r3 = p->fft.r3[i];
            fl[i].chirp_off = std::max<int64_t>(p->fft.chirp_off[i], 0);
            fl[i].bhat_off = std::max<int64_t>(p->fft.bhat_off[i], 0);
        }
        {
            std::vector<int> whole, split;
            for (int q = 0; q < p->npairs; ++q) (p->fft.split[pd[q].len_idx] ? split : whole).push_back(q);
            p->n_whole = (int)whole.size();
            p->n_split = (int)split.size();
            if (p->n_split) {
                dalloc(p, p->d_plist_whole, std::max<size_t>(whole.size(), 1));
                dalloc(p, p->d_plist_split, split.size());
                if (!whole.empty()) upload(p, p->d_plist_whole, whole.data(), whole.size());
                upload(p, p->d_plist_split, split.data(), split.size());
                HIPCHK(hipStreamSynchronize(p->stream));
            }
            // size classes of the unsplit pairs (DMWF_RING_CLASSES=0 turns them off)
            std::vector<int> small, big;
            // (4096 + 512 + 32) x 16 B = 72.5 KB; DMWF_RING_SMALL_M lowers the
            // bound, to exercise the two launches on small grids
            const int kSmallM = std::max(4, std::min(4096, env_int("DMWF_RING_SMALL_M", 4096)));
            for (int q : whole) (p->fft.M[pd[q].len_idx] <= kSmallM ? small : big).push_back(q);
            if (env_int("DMWF_RING_CLASSES", 1) == 1 && !small.empty() && !big.empty()) {
                p->ring_classes = 1;
                p->n_small = (int)small.size();
                p->n_big = (int)big.size();
                for (int q : small) p->lds_small = std::max(p->lds_small, p->fft.M[pd[q].len_idx]);
                for (int q : big) p->lds_big = std::max(p->lds_big, p->fft.M[pd[q].len_idx]);
                dalloc(p, p->d_plist_small, small.size());
                dalloc(p, p->d_plist_big, big.size());
                upload(p, p->d_plist_small, small.data(), small.size());
                upload(p, p->d_plist_big, big.data(), big.size());
                HIPCHK(hipStreamSynchronize(p->stream));
            }
        }
        dalloc(p, p->d_pair_x, p->npairs);
        dalloc(p, p->d_pair_w, p->npairs);
        dalloc(p, p->d_pair_one, p->npairs);
        dalloc(p, p->d_pairs, p->npairs);
        dalloc(p, p->d_fftlen, fl.size());
        dalloc(p, p->d_chirp, p->fft.chirp.size());
        dalloc(p, p->d_bhat, p->fft.bhat.size());
        dalloc(p, p->d_tw, p->fft.tw.size());
        dalloc(p, p->d_tw3, p->fft.tw3.size());
        upload(p, p->d_pair_x, px.data(), px.size());
        upload(p, p->d_pair_w, pw.data(), pw.size());
        upload(p, p->d_pair_one, one.data(), one.size());
        upload(p, p->d_pairs, pd.data(), pd.size());
        upload(p, p->d_fftlen, fl.data(), fl.size());
        if (!p->fft.chirp.empty()) upload(p, p->d_chirp, p->fft.chirp.data(), p->fft.chirp.size());
        if (!p->fft.bhat.empty()) upload(p, p->d_bhat, p->fft.bhat.data(), p->fft.bhat.size());
        upload(p, p->d_tw, p->fft.tw.data(), p->fft.tw.size());
        upload(p, p->d_tw3, p->fft.tw3.data(), p->fft.tw3.size());
        // FP32 ring transforms for a mixed plan: opt-in (DMWF_RING_FP32=1).
        // At Nside 1024, lmax 2048 they take the B-mode error of the mixed
        // solve from 4e-6 to 1.2e-5 relative, past the 1e-5 bar, so the
        // default keeps the ring step in FP64.
        const char* rf = std::getenv("DMWF_RING_FP32");
        if (precision == DM_MIXED && rf && std::atoi(rf) == 1) {
            auto to32 = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
            const std::vector<float> c32 = to32(p->fft.chirp), b32 = to32(p->fft.bhat), t32 = to32(p->fft.tw),
                                     t332 = to32(p->fft.tw3);
            dalloc(p, p->d_chirp32, c32.size());
            dalloc(p, p->d_bhat32, b32.size());
            dalloc(p, p->d_tw32, t32.size());
            dalloc(p, p->d_tw332, t332.size());
            if (!c32.empty()) upload(p, p->d_chirp32, c32.data(), c32.size());
            if (!b32.empty()) upload(p, p->d_bhat32, b32.data(), b32.size());
            upload(p, p->d_tw32, t32.data(), t32.size());
            upload(p, p->d_tw332, t332.data(), t332.size());
            HIPCHK(hipStreamSynchronize(p->stream));           // the host copies go out of scope
        }
        HIPCHK(ring_set_lds_limit(p->fft_lds_bytes));
        std::vector<int64_t> roff(p->rings.offset.begin(), p->rings.offset.end());
        dalloc(p, p->d_ring_w, p->nrings);
        dalloc(p, p->d_ring_off, p->nrings);
        dalloc(p, p->d_ring_n, p->nrings);
        upload(p, p->d_ring_w, p->rings.w.data(), p->nrings);
        upload(p, p->d_ring_off, roff.data(), p->nrings);
        upload(p, p->d_ring_n, p->rings.nphi.data(), p->nrings);

        // recursion coefficients and seeds
        std::vector<double> coef, lp0, lp2;
        build_coefficients(lmax, coef, lp0, lp2);
        dalloc(p, p->d_coef, coef.size());
        dalloc(p, p->d_lp0, lp0.size());
        dalloc(p, p->d_lp2, lp2.size());
        upload(p, p->d_coef, coef.data(), coef.size());
        {
            std::vector<double> coef_s, scale;
            build_scaled_coefficients(lmax, coef_s, scale);
            dalloc(p, p->d_coef_s, coef_s.size());
            dalloc(p, p->d_scale, scale.size());
            upload(p, p->d_coef_s, coef_s.data(), coef_s.size());
            upload(p, p->d_scale, scale.data(), scale.size());
            HIPCHK(hipStreamSynchronize(p->stream));
        }
        upload(p, p->d_lp0, lp0.data(), lp0.size());
        upload(p, p->d_lp2, lp2.data(), lp2.size());
        const size_t sn = (size_t)(p->mmax + 1) * p->npairs;
        dalloc(p, p->d_lstart, sn);
        dalloc(p, p->d_seed, sn * kSeedFields);
        HIPCHK(launch_seeds(p, p->stream));
        dalloc(p, p->d_slot_lo, (size_t)(p->mmax + 1) * batched_analysis_slots(p));
        HIPCHK(launch_slot_starts(p, p->d_slot_lo, p->stream));

        // tiling of the Legendre kernels (ring pairs per lane R); the
        // DMWF_ANA_R / DMWF_SYN_R / DMWF_SYN_THREADS / DMWF_*_MCHUNK
        // environment variables override the defaults for tuning sweeps
        int ar = env_int("DMWF_ANA_R", p->npairs >= 2048 ? 2 : 1);
        if (ar != 1 && ar != 2 && ar != 4) ar = 2;
        set_analysis_tiling(p, ar);
        p->syn_R = env_int("DMWF_SYN_R", 1);
        if (p->syn_R != 1 && p->syn_R != 2 && p->syn_R != 4) p->syn_R = 1;
        p->syn_threads = env_int("DMWF_SYN_THREADS", 128);
        if (p->syn_threads != 64 && p->syn_threads != 128 && p->syn_threads != 256) p->syn_threads = 128;
        p->mfma_mode = env_int("DMWF_MFMA", -1);
        // batched kernels: consecutive m per XCD chunk (0 = plain order)
        p->syn_mchunk = std::max(0, std::min(16, env_int("DMWF_SYN_MCHUNK", 4)));
        // (measured at Nside 1024, lmax 2048, B = 8: synthesis gains from
        // chunks of 4 in both precisions, the FP64 analysis from chunks of 2,
        // the FP32 analysis runs best in plain order)
        p->ana_mchunk = std::max(0, std::min(16, env_int("DMWF_ANA_MCHUNK", precision == DM_MIXED ? 0 : 2)));

        // work buffers
        const size_t B = (size_t)max_rhs;
        dalloc(p, p->d_phase, B * 3 * p->npairs * (p->mmax + 1) * 4);
        if (precision == DM_MIXED) dalloc(p, p->d_phase32, B * 3 * p->npairs * (p->mmax + 1) * 4);
        // partial-sum slots for every analysis the plan may run: a call of n
        // RHS takes a slot set of n RHS per slot, from the batched kernels'
        // slots or the vector kernel's chunks (which of the two runs depends
        // on n); a mixed plan also runs the FP64 kernels for its FP64
        // epilogue
        size_t slot_rhs = 0;
        {
            const dm_precision pr = p->precision;
            for (dm_precision q : {pr, DM_FP64}) {
                p->precision = q;
                for (size_t n : {B, std::min(B, (size_t)7), (size_t)1}) {
                    const size_t ns = use_mfma(p, (int)n) ? (size_t)batched_analysis_slots(p) : (size_t)p->ana_chunks;
                    slot_rhs = std::max(slot_rhs, ns * n);
                }
            }
            p->precision = pr;
        }
        dalloc(p, p->d_partial, slot_rhs * 3 * p->nalm * 2);
        dalloc(p, p->d_alm, B * 3 * p->nalm * 2);
        dalloc(p, p->d_alm_prev, B * 3 * p->nalm * 2);
        dalloc(p, p->d_state_u, B * 3 * p->nalm * 2);
        dalloc(p, p->d_alm_spin, B * 3 * p->nalm * 2);
        dalloc(p, p->d_alm_r, B * 3 * p->nalm * 2);
        dalloc(p, p->d_alm_y, B * 3 * p->nalm * 2);
        dalloc(p, p->d_d0, B * 3 * p->npix);
        dalloc(p, p->d_b, B * 3 * p->npix);
        dalloc(p, p->d_ux, B * 3 * p->npix);
        dalloc(p, p->d_K, 3 * p->npix);
        dalloc(p, p->d_tn, 3 * p->npix);
        dalloc(p, p->d_ninv, 3 * p->npix);
        dalloc(p, p->d_obs, p->npix);
        dalloc(p, p->d_mats, 3 * (size_t)(lmax + 1) * 4);
        dalloc(p, p->d_cpart, B * (size_t)cauchy_blocks(p) * 2);
        dalloc(p, p->d_cout, B * 2);
        HIPCHK(hipHostMalloc((void**)&p->h_cout, B * 2 * sizeof(double), hipHostMallocDefault));
        p->red_len = 64 + B * p->nrings + B * (size_t)alm_norm_blocks(p) * kNormQ + p->nrings;
        dalloc(p, p->d_red, p->red_len);
        HIPCHK(hipStreamSynchronize(p->stream));
        p->cl.assign(4 * (size_t)(lmax + 1), 0.0);
    } catch (const Fail& f) {
        g_create_err = p->err;
        free_plan(p);
        return f.st;
    } catch (...) {
        g_create_err = "internal error during plan creation";
        free_plan(p);
        return DM_EDEVICE;
    }
    *out = p;
    return DM_OK;
}

dm_status dm_plan_destroy(dm_plan* p) {
    if (!p) return DM_EINVAL;
    free_plan(p);
    return DM_OK;
}

dm_status dm_plan_info(const dm_plan* p, int64_t* npix, int64_t* nalm, int* nrings) {
    if (!p) return DM_EINVAL;
    if (npix) *npix = p->npix;
    if (nalm) *nalm = p->nalm;
    if (nrings) *nrings = p->nrings;
    return DM_OK;
}

dm_status dm_set_spectra(dm_plan* p, const double* cl) {
    return guarded(p, [&] {
        REQUIRE(cl != nullptr, DM_EINVAL, "cl is null");
        const int L = p->lmax + 1;
        REQUIRE(all_finite(cl, 4 * (size_t)L), DM_EINVAL, "spectra must be finite");
        std::vector<double> c(cl, cl + 4 * (size_t)L);
        for (int l = 0; l < L; ++l) {
            if (l < 2) {
                c[1 * L + l] = c[2 * L + l] = c[3 * L + l] = 0.0;   // no E, B below l = 2
            }
            const double TT = c[l], EE = c[L + l], BB = c[2 * L + l], TE = c[3 * L + l];
            REQUIRE(TT >= 0 && EE >= 0 && BB >= 0 && TE * TE <= TT * EE * (1 + 1e-12), DM_EINVAL,
                    "S_l must be positive semi-definite at l = " + std::to_string(l));
        }
        p->cl = c;
        std::vector<double> m1, m2, m3, all;
        build_matrix_function(p->cl, p->lmax, 1, m1);
        build_matrix_function(p->cl, p->lmax, 2, m2);
        build_matrix_function(p->cl, p->lmax, 3, m3);
        all.insert(all.end(), m1.begin(), m1.end());
        all.insert(all.end(), m2.begin(), m2.end());
        all.insert(all.end(), m3.begin(), m3.end());
        upload(p, p->d_mats, all.data(), all.size());
        HIPCHK(hipStreamSynchronize(p->stream));
        p->hash_cl = host_hash(p->cl.data(), p->cl.size());
        p->spectra_set = true;
    });
}

dm_status dm_set_noise(dm_plan* p, const double* ncov, dm_ncov layout, const uint8_t* obs) {
    return dm_set_noise_masks(p, ncov, layout, obs, obs);
}

dm_status dm_set_noise_masks(dm_plan* p, const double* ncov, dm_ncov layout, const uint8_t* obs_t,
                             const uint8_t* obs_p) {
    return guarded(p, [&] {
        REQUIRE(ncov != nullptr, DM_EINVAL, "ncov is null");
        REQUIRE(layout == DM_NCOV_DIAG3 || layout == DM_NCOV_SYM6, DM_EUNSUPPORTED, "unknown noise layout");
        const int64_t n = p->npix;
        const int rows = layout == DM_NCOV_SYM6 ? 6 : 3;
        // observation bits: 1 = I, 2 = Q and U
        std::vector<uint8_t> bits(n);
        int64_t nobs = 0;
        for (int64_t q = 0; q < n; ++q) {
            const int m = ((!obs_t || obs_t[q]) ? 1 : 0) | ((!obs_p || obs_p[q]) ? 2 : 0);
            bits[q] = (uint8_t)m;
            if (!m) continue;
            ++nobs;
            if (layout == DM_NCOV_DIAG3) {
                for (int f = 0; f < 3; ++f) {
                    if (!(m & (f == 0 ? 1 : 2))) continue;
                    const double v = ncov[f * n + q];
                    REQUIRE(std::isfinite(v) && v > 0, DM_EINVAL,
                            "observed noise variances must be finite and > 0 (pixel " + std::to_string(q) + ")");
                }
            } else {
                double e[6];
                for (int k = 0; k < 6; ++k) e[k] = ncov[k * n + q];
                bool ok = true;
                for (int k = 0; k < 6; ++k) ok = ok && std::isfinite(e[k]);
                // Sylvester: leading minors of [[II IQ IU] [IQ QQ QU] [IU QU UU]] > 0
                const double m1 = e[0], m2 = e[0] * e[3] - e[1] * e[1];
                const double m3 = e[0] * (e[3] * e[5] - e[4] * e[4]) - e[1] * (e[1] * e[5] - e[4] * e[2]) +
                                  e[2] * (e[1] * e[4] - e[3] * e[2]);
                REQUIRE(ok && m1 > 0 && m2 > 0 && m3 > 0, DM_EINVAL,
                        "the 3x3 noise covariance must be finite and positive definite on pixels with an "
                        "observed component (pixel " + std::to_string(q) + ")");
            }
        }
        REQUIRE(nobs > 0, DM_EINVAL, "every pixel is masked");
        p->noise_set = false;
        if (layout == DM_NCOV_SYM6 && !p->d_ninv6) {
            dalloc(p, p->d_ninv6, 6 * (size_t)n);
            dalloc(p, p->d_tn6, 6 * (size_t)n);
        }
        p->ncov_layout = layout;
        double* d_ncov = nullptr;
        HIPCHK(hipMalloc((void**)&d_ncov, rows * n * sizeof(double)));
        std::unique_ptr<double, void (*)(double*)> guard(d_ncov, [](double* x) { (void)hipFree(x); });
        upload(p, d_ncov, ncov, rows * n);
        upload(p, p->d_obs, bits.data(), n);
        double* ring_min = p->d_red + 64;
        HIPCHK(launch_tau_parts(p, d_ncov, ring_min, p->stream));
        std::vector<double> rm(p->nrings);
        HIPCHK(hipMemcpyAsync(rm.data(), ring_min, rm.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        double tau = INFINITY;
        for (double v : rm) tau = std::min(tau, v);
        REQUIRE(std::isfinite(tau) && tau > 0, DM_EINVAL, "no valid observed pixel");
        p->tau = tau;
        HIPCHK(launch_noise_setup(p, d_ncov, tau, p->stream));
        // fingerprint: the mask bits and T N^-1 (which carries tau)
        const bool sym = layout == DM_NCOV_SYM6;
        const uint64_t h_obs = device_hash(p, p->d_obs, n, 1, p->stream);
        const uint64_t h_tn = device_hash(p, sym ? p->d_tn6 : p->d_tn, (sym ? 6 : 3) * n, 8, p->stream);
        p->hash_noise = hash_mix(h_obs + 3 * hash_mix(h_tn + (uint64_t)layout));
        p->noise_set = true;
    });
}

dm_status dm_set_schedule(dm_plan* p, const dm_schedule* sc) {
    return guarded(p, [&] {
        REQUIRE(sc != nullptr, DM_EINVAL, "schedule is null");
        REQUIRE(std::isfinite(sc->lambda_start) && sc->lambda_start >= 1.0, DM_EINVAL, "lambda_start must be >= 1");
        if (sc->iters_per_step >= 1) {
            REQUIRE(sc->nsteps >= 1 && sc->nsteps <= 100000, DM_EINVAL, "nsteps must be in [1, 100000]");
            REQUIRE(sc->iters_per_step <= 10000000, DM_EINVAL, "iters_per_step must be <= 1e7");
            REQUIRE(sc->max_iters >= 0, DM_EINVAL, "max_iters must be >= 0 (0: no cap)");
        } else {
            REQUIRE(std::isfinite(sc->beta) && sc->beta > 0.0 && sc->beta < 1.0, DM_EINVAL,
                    "epsilon mode: beta must be in (0, 1)");
            REQUIRE(std::isfinite(sc->eps_end) && sc->eps_end > 0.0, DM_EINVAL, "epsilon mode: eps_end must be > 0");
            REQUIRE(std::isfinite(sc->eps_start) && sc->eps_start >= sc->eps_end, DM_EINVAL,
                    "epsilon mode: eps_start must be >= eps_end");
            REQUIRE(std::isfinite(sc->eps_eta) && sc->eps_eta >= 1.0, DM_EINVAL, "epsilon mode: eps_eta must be >= 1");
            REQUIRE(sc->max_iters >= 1 && sc->max_iters <= 100000000, DM_EINVAL,
                    "epsilon mode: max_iters must be in [1, 1e8]");
            REQUIRE(std::log(sc->lambda_start) / -std::log(sc->beta) < 100000.0, DM_EINVAL,
                    "epsilon mode: more than 1e5 cooling steps");
        }
        p->sched = *sc;
    });
}

}  // extern "C"

// --------------------------------------------------------------------------
// checkpoint files: a fixed little header, the state, and a checksum of
// every byte before it.  Written to path + ".tmp", then renamed.
// --------------------------------------------------------------------------
namespace {

constexpr char kCkMagic[8] = {'D', 'M', 'W', 'F', 'C', 'K', 'P', 'T'};
constexpr uint32_t kCkVersion = 1;

struct CkSum {
    uint64_t h = 0x6A09E667F3BCC909ull;
    void add(const void* buf, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(buf);
        size_t i = 0;
        for (; i + 8 <= n; i += 8) {
            uint64_t w;
            std::memcpy(&w, b + i, 8);
            h = dmwf::hash_mix(h ^ w);
        }
        uint64_t w = 0;
        std::memcpy(&w, b + i, n - i);
        h = dmwf::hash_mix(h ^ w ^ ((uint64_t)(n - i) << 56));
    }
};

struct CkWriter {
    std::FILE* f;
    CkSum sum;
    bool ok = true;
    void put(const void* buf, size_t n) {
        sum.add(buf, n);
        if (n && std::fwrite(buf, 1, n, f) != n) ok = false;
    }
    template <typename T>
    void val(T v) { put(&v, sizeof v); }
};

struct CkReader {
    std::FILE* f;
    CkSum sum;
    bool ok = true;
    void get(void* buf, size_t n) {
        if (n && std::fread(buf, 1, n, f) != n) {
            ok = false;
            std::memset(buf, 0, n);
        }
        sum.add(buf, n);
    }
    template <typename T>
    T val() {
        T v;
        get(&v, sizeof v);
        return v;
    }
};

void put_schedule(CkWriter& w, const dm_schedule& sc) {
    w.val(sc.lambda_start);
    w.val<int32_t>(sc.nsteps);
    w.val<int32_t>(sc.iters_per_step);
    w.val(sc.beta);
    w.val(sc.eps_start);
    w.val(sc.eps_end);
    w.val(sc.eps_eta);
    w.val<int32_t>(sc.max_iters);
}

dm_schedule get_schedule(CkReader& r) {
    dm_schedule sc{};
    sc.lambda_start = r.val<double>();
    sc.nsteps = r.val<int32_t>();
    sc.iters_per_step = r.val<int32_t>();
    sc.beta = r.val<double>();
    sc.eps_start = r.val<double>();
    sc.eps_end = r.val<double>();
    sc.eps_eta = r.val<double>();
    sc.max_iters = r.val<int32_t>();
    return sc;
}

}  // namespace

extern "C" {

dm_status dm_checkpoint_save(const dm_plan* cp, const char* path) {
    dm_plan* p = const_cast<dm_plan*>(cp);
    return guarded(p, [&] {
        REQUIRE(path != nullptr && path[0], DM_EINVAL, "path is empty");
        REQUIRE(p->state.valid, DM_ESTATE, "no completed Wiener filter solve to checkpoint");
        const dm_plan::SolveState& st = p->state;
        const bool eps = eps_mode(st.sched);
        const size_t n = (size_t)st.nrhs * 3 * p->nalm * 2;
        std::vector<double> u(n), up;
        HIPCHK(hipMemcpyAsync(u.data(), p->d_state_u, n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        if (!eps) {
            up.resize(n);
            HIPCHK(hipMemcpyAsync(up.data(), p->d_alm_prev, n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        }
        HIPCHK(hipStreamSynchronize(p->stream));
        const std::string tmp = std::string(path) + ".tmp";
        std::FILE* f = std::fopen(tmp.c_str(), "wb");
        REQUIRE(f != nullptr, DM_EINVAL, "cannot open " + tmp + " for writing");
        CkWriter w{f, CkSum{}};
        w.put(kCkMagic, sizeof kCkMagic);
        w.val<uint32_t>(kCkVersion);
        w.val<int32_t>(p->grid.kind);
        w.val<int32_t>(p->grid.nside);
        w.val<int32_t>(p->grid.ntheta);
        w.val<int32_t>(p->grid.nphi);
        w.val<int32_t>(p->lmax);
        w.val<int32_t>(p->precision);
        w.val<int32_t>(p->ncov_layout);
        w.val<int32_t>(st.nrhs);
        w.val<int64_t>(p->nalm);
        put_schedule(w, st.sched);
        w.val<uint64_t>(st.hash_cl);
        w.val<uint64_t>(st.hash_noise);
        w.val<uint64_t>(st.hash_data);
        w.val<int64_t>(st.iterations);
        w.val<int32_t>(st.next_step);
        w.val<int32_t>(st.finished ? 1 : 0);
        w.val<int32_t>(eps ? 0 : 1);
        const std::vector<double>& tc = p->trace_cauchy;
        const std::vector<int>& ts = p->trace_step;
        const int64_t ntr = eps ? (int64_t)tc.size() : 0;
        w.val<int64_t>(ntr);
        for (int64_t i = 0; i < ntr; ++i) w.val<double>(tc[i]);
        for (int64_t i = 0; i < ntr; ++i) w.val<int32_t>(ts[i]);
        for (int r = 0; r < st.nrhs; ++r) w.val<double>(r < (int)st.last_c.size() ? st.last_c[r] : 0.0);
        w.put(u.data(), n * sizeof(double));
        if (!eps) w.put(up.data(), n * sizeof(double));
        const uint64_t sum = w.sum.h;
        if (std::fwrite(&sum, sizeof sum, 1, f) != 1) w.ok = false;
        if (std::fclose(f) != 0) w.ok = false;
        if (!w.ok) std::remove(tmp.c_str());
        REQUIRE(w.ok, DM_EINVAL, "writing " + tmp + " failed");
        REQUIRE(std::rename(tmp.c_str(), path) == 0, DM_EINVAL, std::string("cannot rename to ") + path);
    });
}

dm_status dm_checkpoint_load(dm_plan* p, const char* path) {
    return guarded(p, [&] {
        REQUIRE(path != nullptr && path[0], DM_EINVAL, "path is empty");
        std::FILE* f = std::fopen(path, "rb");
        REQUIRE(f != nullptr, DM_EINVAL, std::string("cannot open ") + path);
        std::unique_ptr<std::FILE, int (*)(std::FILE*)> guard(f, &std::fclose);
        CkReader r{f, CkSum{}};
        char magic[8];
        r.get(magic, sizeof magic);
        REQUIRE(r.ok && std::memcmp(magic, kCkMagic, 8) == 0, DM_EINVAL, "not a checkpoint file");
        REQUIRE(r.val<uint32_t>() == kCkVersion, DM_EINVAL, "unsupported checkpoint version");
        const int kind = r.val<int32_t>(), nside = r.val<int32_t>(), ntheta = r.val<int32_t>(),
                  nphi = r.val<int32_t>(), lmax = r.val<int32_t>(), prec = r.val<int32_t>();
        (void)r.val<int32_t>();                          // noise layout (part of the noise fingerprint)
        const int nrhs = r.val<int32_t>();
        const int64_t nalm = r.val<int64_t>();
        REQUIRE(r.ok, DM_EINVAL, "truncated checkpoint");
        const bool same_grid = kind == p->grid.kind &&
                               (kind == DM_GRID_HEALPIX_RING ? nside == p->grid.nside
                                                             : (ntheta == p->grid.ntheta && nphi == p->grid.nphi));
        REQUIRE(same_grid && lmax == p->lmax && nalm == p->nalm, DM_EINVAL,
                "the checkpoint was written for another grid or lmax");
        REQUIRE(prec == p->precision, DM_EINVAL, "the checkpoint was written with another precision");
        REQUIRE(nrhs >= 1 && nrhs <= p->max_rhs, DM_EINVAL, "the checkpoint holds more RHS than max_rhs");
        dm_plan::Resume rs;
        dm_plan::SolveState& st = rs.st;
        st.nrhs = nrhs;
        st.sched = get_schedule(r);
        st.hash_cl = r.val<uint64_t>();
        st.hash_noise = r.val<uint64_t>();
        st.hash_data = r.val<uint64_t>();
        st.iterations = r.val<int64_t>();
        st.next_step = r.val<int32_t>();
        st.finished = r.val<int32_t>() != 0;
        rs.has_prev = r.val<int32_t>() != 0;
        const int64_t ntr = r.val<int64_t>();
        REQUIRE(r.ok && st.iterations >= 0 && st.iterations <= 100000000 && ntr >= 0 && ntr <= st.iterations &&
                    st.next_step >= 0 && rs.has_prev == !eps_mode(st.sched),
                DM_EINVAL, "corrupt checkpoint header");
        rs.trace_cauchy.resize(ntr);
        rs.trace_step.resize(ntr);
        for (int64_t i = 0; i < ntr; ++i) rs.trace_cauchy[i] = r.val<double>();
        for (int64_t i = 0; i < ntr; ++i) rs.trace_step[i] = r.val<int32_t>();
        st.last_c.resize(nrhs);
        for (int k = 0; k < nrhs; ++k) st.last_c[k] = r.val<double>();
        const size_t n = (size_t)nrhs * 3 * p->nalm * 2;
        rs.u.resize(n);
        r.get(rs.u.data(), n * sizeof(double));
        if (rs.has_prev) {
            rs.uprev.resize(n);
            r.get(rs.uprev.data(), n * sizeof(double));
        }
        const uint64_t want = r.sum.h;
        uint64_t sum = 0;
        REQUIRE(r.ok && std::fread(&sum, sizeof sum, 1, f) == 1, DM_EINVAL, "truncated checkpoint");
        REQUIRE(sum == want, DM_EINVAL, "checkpoint checksum mismatch");
        rs.pending = true;
        p->resume = std::move(rs);
    });
}

dm_status dm_set_refinement(dm_plan* p, int ncorrections) {
    return guarded(p, [&] {
        REQUIRE(ncorrections >= 0 && ncorrections <= 1000, DM_EINVAL, "ncorrections must be in [0, 1000]");
        if (ncorrections > 0 && !p->d_b2) {
            dalloc(p, p->d_b2, (size_t)p->max_rhs * 3 * p->npix);
            dalloc(p, p->d_alm_corr, (size_t)p->max_rhs * 3 * p->nalm * 2);
            dalloc(p, p->d_alm_best, (size_t)p->max_rhs * 3 * p->nalm * 2);
        }
        p->refine = ncorrections;
    });
}

dm_status dm_set_refinement_select(dm_plan* p, int keep_best) {
    return guarded(p, [&] {
        REQUIRE(keep_best == 0 || keep_best == 1, DM_EINVAL, "keep_best must be 0 or 1");
        p->refine_best = keep_best;
    });
}

dm_status dm_refinement_selected(const dm_plan* p, int* index, int cap, int* n) {
    if (!p || !n) return DM_EINVAL;
    const int cnt = (int)p->refine_chosen.size();
    const int k = std::max(0, std::min(cap, cnt));
    if (index) std::copy(p->refine_chosen.begin(), p->refine_chosen.begin() + k, index);
    *n = cnt;
    return DM_OK;
}

dm_status dm_refinement_trace(const dm_plan* p, double* history, int cap, int* n, int* nrhs) {
    if (!p || !n) return DM_EINVAL;
    const int cnt = (int)p->refine_hist.size();
    const int k = std::max(0, std::min(cap, cnt));
    if (history) std::copy(p->refine_hist.begin(), p->refine_hist.begin() + k, history);
    *n = cnt;
    if (nrhs) *nrhs = cnt ? p->refine_nrhs : 0;
    return DM_OK;
}

dm_status dm_transform_work(dm_plan* p, int64_t* points, int64_t* executed) {
    return guarded(p, [&] {
        REQUIRE(points && executed, DM_EINVAL, "null argument");
        const size_t sn = (size_t)(p->mmax + 1) * p->npairs;
        std::vector<int> ls(sn);
        HIPCHK(hipMemcpyAsync(ls.data(), p->d_lstart, sn * sizeof(int), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        int64_t ex = 0;
        for (int m = 0; m <= p->mmax; ++m)
            for (int q = 0; q < p->npairs; ++q) {
                const int l0 = std::max(ls[(size_t)m * p->npairs + q], m);
                if (l0 <= p->lmax) ex += p->lmax + 1 - l0;
            }
        *points = (int64_t)p->npairs * p->nalm;
        *executed = ex;
    });
}

dm_status dm_set_adaptive_resolution(dm_plan* p, double factor) {
    return guarded(p, [&] {
        REQUIRE(factor == 0.0 || (std::isfinite(factor) && factor >= 1.0), DM_EINVAL,
                "factor must be 0 (off) or >= 1");
        p->adaptive = factor;
    });
}

dm_status dm_step_band_limits(const dm_plan* p, int* lcut, int cap, int* n) {
    if (!p || !n) return DM_EINVAL;
    const int cnt = (int)p->step_lcut.size();
    const int k = std::max(0, std::min(cap, cnt));
    if (lcut) std::copy(p->step_lcut.begin(), p->step_lcut.begin() + k, lcut);
    *n = cnt;
    return DM_OK;
}

dm_status dm_set_diagnostics(dm_plan* p, int every) {
    return guarded(p, [&] {
        REQUIRE(every >= 0, DM_EINVAL, "every must be >= 0 (0: off)");
        p->diag_every = every;
    });
}

dm_status dm_diagnostics_trace(const dm_plan* p, int* iteration, double* chi2, double* residual, int cap, int* n,
                               int* nrhs) {
    if (!p || !n) return DM_EINVAL;
    const int cnt = (int)p->diag_iter.size();
    const int k = std::max(0, std::min(cap, cnt));
    const size_t w = (size_t)std::max(p->diag_nrhs, 1);
    if (iteration) std::copy(p->diag_iter.begin(), p->diag_iter.begin() + k, iteration);
    if (chi2) std::copy(p->diag_chi2.begin(), p->diag_chi2.begin() + k * w, chi2);
    if (residual) std::copy(p->diag_resid.begin(), p->diag_resid.begin() + k * w, residual);
    *n = cnt;
    if (nrhs) *nrhs = cnt ? p->diag_nrhs : 0;
    return DM_OK;
}

dm_status dm_schedule_trace(const dm_plan* p, double* cauchy, int* step, int cap, int* n) {
    if (!p || !n) return DM_EINVAL;
    const int cnt = (int)p->trace_cauchy.size();
    const int k = std::max(0, std::min(cap, cnt));
    if (cauchy) std::copy(p->trace_cauchy.begin(), p->trace_cauchy.begin() + k, cauchy);
    if (step) std::copy(p->trace_step.begin(), p->trace_step.begin() + k, step);
    *n = cnt;
    return DM_OK;
}

dm_status dm_wiener_filter(dm_plan* p, int nrhs, const double* d, double* alm, double* map, dm_stats* stats) {
    return guarded(p, [&] {
        REQUIRE(d && alm, DM_EINVAL, "d and alm must not be null");
        check_rhs(p, nrhs);
        const size_t nmap = (size_t)nrhs * 3 * p->npix;
        REQUIRE(all_finite(d, nmap), DM_EINVAL, "d must be finite");
        double *dd = nullptr, *da = nullptr, *dm = nullptr;
        auto del = [](double* x) { if (x) (void)hipFree(x); };
        HIPCHK(hipMalloc((void**)&dd, nmap * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g1(dd, del);
        HIPCHK(hipMalloc((void**)&da, (size_t)nrhs * 3 * p->nalm * 2 * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g2(da, del);
        if (map) HIPCHK(hipMalloc((void**)&dm, nmap * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g3(dm, del);
        upload(p, dd, d, nmap);
        solve_dev(p, nrhs, dd, da, dm, p->stream, stats, true);
        HIPCHK(hipMemcpyAsync(alm, da, (size_t)nrhs * 3 * p->nalm * 2 * sizeof(double), hipMemcpyDeviceToHost,
                              p->stream));
        if (map) HIPCHK(hipMemcpyAsync(map, dm, nmap * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
    });
}

dm_status dm_wiener_filter_device(dm_plan* p, int nrhs, const void* d, void* alm, void* map, void* hip_stream,
                                  dm_stats* stats) {
    return guarded(p, [&] {
        REQUIRE(d && alm, DM_EINVAL, "d and alm must not be null");
        check_rhs(p, nrhs);
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : p->stream;
        // the data must be finite (checked on the device)
        int* d_cnt = reinterpret_cast<int*>(p->d_red);
        sync_plan_stream_to(p, s);
        HIPCHK(hipMemsetAsync(d_cnt, 0, sizeof(int), s));
        HIPCHK(launch_count_nonfinite((const double*)d, (int64_t)nrhs * 3 * p->npix, d_cnt, s));
        int cnt = 0;
        HIPCHK(hipMemcpyAsync(&cnt, d_cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        REQUIRE(cnt == 0, DM_EINVAL, "d must be finite");
        solve_dev(p, nrhs, (const double*)d, (double*)alm, (double*)map, s, stats, true);
    });
}

dm_status dm_wiener_filter_device_f32(dm_plan* p, int nrhs, const void* d, void* alm, void* map, void* hip_stream,
                                      dm_stats* stats) {
    return guarded(p, [&] {
        REQUIRE(d && alm, DM_EINVAL, "d and alm must not be null");
        check_rhs(p, nrhs);
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : p->stream;
        const int64_t nmap = (int64_t)nrhs * 3 * p->npix, nalm2 = (int64_t)nrhs * 3 * p->nalm * 2;
        double *dd = nullptr, *da = nullptr, *dm = nullptr;
        auto del = [](double* x) { if (x) (void)hipFree(x); };
        HIPCHK(hipMalloc((void**)&dd, (size_t)nmap * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g1(dd, del);
        HIPCHK(hipMalloc((void**)&da, (size_t)nalm2 * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g2(da, del);
        if (map) HIPCHK(hipMalloc((void**)&dm, (size_t)nmap * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g3(dm, del);
        sync_plan_stream_to(p, s);
        HIPCHK(launch_widen(dd, static_cast<const float*>(d), nmap, s));
        // the data must be finite (checked on the device)
        int* d_cnt = reinterpret_cast<int*>(p->d_red);
        HIPCHK(hipMemsetAsync(d_cnt, 0, sizeof(int), s));
        HIPCHK(launch_count_nonfinite(dd, nmap, d_cnt, s));
        int cnt = 0;
        HIPCHK(hipMemcpyAsync(&cnt, d_cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        REQUIRE(cnt == 0, DM_EINVAL, "d must be finite");
        solve_dev(p, nrhs, dd, da, dm, s, stats, true);
        HIPCHK(launch_narrow(static_cast<float*>(alm), da, nalm2, s));
        if (map) HIPCHK(launch_narrow(static_cast<float*>(map), dm, nmap, s));
        // the scratch is freed when the guards go: wait for the narrowing
        HIPCHK(hipStreamSynchronize(s));
    });
}

dm_status dm_constrained_realizations(dm_plan* p, int nreal, const double* d, const double* shat_alm,
                                      const double* dhat, double* scr_alm, double* f_alm) {
    return guarded(p, [&] {
        REQUIRE(d && shat_alm && dhat && scr_alm, DM_EINVAL, "null argument");
        REQUIRE(nreal >= 1, DM_EINVAL, "nreal must be >= 1");
        const int B = nreal + 1;
        check_rhs(p, B);
        const size_t nm = (size_t)3 * p->npix, na = (size_t)3 * p->nalm * 2;
        REQUIRE(all_finite(d, nm) && all_finite(dhat, nm * nreal) && all_finite(shat_alm, na * nreal), DM_EINVAL,
                "inputs must be finite");
        double *dd = nullptr, *da = nullptr, *ds = nullptr;
        auto del = [](double* x) { if (x) (void)hipFree(x); };
        HIPCHK(hipMalloc((void**)&dd, nm * B * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g1(dd, del);
        HIPCHK(hipMalloc((void**)&da, na * B * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g2(da, del);
        HIPCHK(hipMalloc((void**)&ds, na * nreal * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g3(ds, del);
        // right-hand sides: d, then d - d_hat_k   (eq 19)
        upload(p, dd, d, nm);
        upload(p, dd + nm, dhat, nm * nreal);
        for (int k = 0; k < nreal; ++k)
            HIPCHK(launch_axpby(dd + nm * (k + 1), dd, 1.0, -1.0, (int64_t)nm, p->stream));
        upload(p, ds, shat_alm, na * nreal);
        solve_dev(p, B, dd, da, nullptr, p->stream, nullptr, false);
        // s_CR,k = W(d - d_hat_k) + s_hat_k
        HIPCHK(launch_axpby(da + na, ds, 1.0, 1.0, (int64_t)(na * nreal), p->stream));
        HIPCHK(hipMemcpyAsync(scr_alm, da + na, na * nreal * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        if (f_alm) {
            // f_k = s_CR,k - W d
            for (int k = 0; k < nreal; ++k)
                HIPCHK(launch_axpby(da + na * (k + 1), da, -1.0, 1.0, (int64_t)na, p->stream));
            HIPCHK(hipMemcpyAsync(f_alm, da + na, na * nreal * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        }
        HIPCHK(hipStreamSynchronize(p->stream));
    });
}

static dm_status transform_host(dm_plan* p, int nrhs, const double* in, double* out, int which) {
    return guarded(p, [&] {
        REQUIRE(in && out, DM_EINVAL, "null argument");
        check_rhs(p, nrhs);
        const size_t nm = (size_t)nrhs * 3 * p->npix, na = (size_t)nrhs * 3 * p->nalm * 2;
        const size_t nin = which == 0 ? na : nm, nout = which == 0 ? nm : na;
        REQUIRE(all_finite(in, nin), DM_EINVAL, "input must be finite");
        double *di = nullptr, *dout = nullptr;
        auto del = [](double* x) { if (x) (void)hipFree(x); };
        HIPCHK(hipMalloc((void**)&di, nin * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g1(di, del);
        HIPCHK(hipMalloc((void**)&dout, nout * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g2(dout, del);
        upload(p, di, in, nin);
        if (which == 0) alm2map_dev(p, nrhs, di, dout, p->stream);
        else map2alm_dev(p, nrhs, di, dout, which == 1, p->stream);
        HIPCHK(hipMemcpyAsync(out, dout, nout * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        if (p->profiling) collect_events(p);
    });
}

dm_status dm_alm2map(dm_plan* p, int nrhs, const double* alm, double* map) { return transform_host(p, nrhs, alm, map, 0); }
dm_status dm_map2alm(dm_plan* p, int nrhs, const double* map, double* alm) { return transform_host(p, nrhs, map, alm, 1); }
dm_status dm_alm2map_adjoint(dm_plan* p, int nrhs, const double* map, double* alm) {
    return transform_host(p, nrhs, map, alm, 2);
}

dm_status dm_alm2map_device(dm_plan* p, int nrhs, const void* alm, void* map, void* hip_stream) {
    return guarded(p, [&] {
        REQUIRE(alm && map, DM_EINVAL, "null argument");
        check_rhs(p, nrhs);
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : p->stream;
        sync_plan_stream_to(p, s);
        alm2map_dev(p, nrhs, (const double*)alm, (double*)map, s);
        if (p->profiling) {
            HIPCHK(hipStreamSynchronize(s));
            collect_events(p);
        }
    });
}

dm_status dm_map2alm_device(dm_plan* p, int nrhs, const void* map, void* alm, void* hip_stream) {
    return guarded(p, [&] {
        REQUIRE(alm && map, DM_EINVAL, "null argument");
        check_rhs(p, nrhs);
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : p->stream;
        sync_plan_stream_to(p, s);
        map2alm_dev(p, nrhs, (const double*)map, (double*)alm, true, s);
        if (p->profiling) {
            HIPCHK(hipStreamSynchronize(s));
            collect_events(p);
        }
    });
}

dm_status dm_map2alm_device_noalloc(dm_plan* p, int nrhs, const void* map, void* alm, void* hip_stream) {
    return guarded(p, [&] {
        REQUIRE(alm && map, DM_EINVAL, "null argument");
        check_rhs(p, nrhs);
        hipError_t serr = hipSuccess;
        char* base = static_cast<char*>(scratch_of(p->device, &serr));
        REQUIRE(base != nullptr, DM_EDEVICE,
                std::string("the device address of the scratch array is unknown: ") + hipGetErrorString(serr));
        // the work memory map2alm_dev uses: ring Fourier data, then the
        // analysis partial-sum slots, each as the plan's buffers would hold
        // them for nrhs right-hand sides
        const bool batched = use_mfma(p, nrhs);
        const bool ring32 = phase32(p, nrhs);
        const bool part32 = batched && p->precision == DM_MIXED;
        const size_t phase_bytes = (size_t)nrhs * 3 * p->npairs * (p->mmax + 1) * 4 * (ring32 ? 4 : 8);
        const size_t nslots = (size_t)(batched ? batched_analysis_slots(p) : p->ana_chunks);
        const size_t part_bytes = nslots * nrhs * 3 * p->nalm * 2 * (part32 ? 4 : 8);
        const size_t off = (phase_bytes + 255) / 256 * 256;
        REQUIRE(off + part_bytes <= kScratchBytes, DM_EINVAL,
                "this analysis needs " + std::to_string(off + part_bytes) + " bytes of work memory, more than the " +
                    std::to_string(kScratchBytes) + " bytes of the allocation-free path: use dm_map2alm_device");
        // the plan's work buffers stand aside for the call; per-kernel event
        // timing (which creates events) is off during it
        struct Swap {
            dm_plan* p;
            double* phase;
            float* phase32;
            double* partial;
            bool profiling;
            ~Swap() {
                p->d_phase = phase;
                p->d_phase32 = phase32;
                p->d_partial = partial;
                p->profiling = profiling;
            }
        } keep{p, p->d_phase, p->d_phase32, p->d_partial, p->profiling};
        if (ring32)
            p->d_phase32 = reinterpret_cast<float*>(base);
        else
            p->d_phase = reinterpret_cast<double*>(base);
        p->d_partial = reinterpret_cast<double*>(base + off);
        p->profiling = false;
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : p->stream;
        map2alm_dev(p, nrhs, (const double*)map, (double*)alm, true, s);
    });
}

dm_status dm_iterate(dm_plan* p, int nrhs, const double* d, const double* t_in, double lambda, int niter, double* alm,
                     double* t_out) {
    return guarded(p, [&] {
        REQUIRE(d && t_in && alm, DM_EINVAL, "null argument");
        REQUIRE(p->noise_set && p->spectra_set, DM_ESTATE, "noise and spectra must be set");
        REQUIRE(niter >= 1, DM_EINVAL, "niter must be >= 1");
        REQUIRE(std::isfinite(lambda) && lambda >= 1.0, DM_EINVAL, "lambda must be >= 1");
        check_rhs(p, nrhs);
        const size_t nm = (size_t)nrhs * 3 * p->npix, na = (size_t)nrhs * 3 * p->nalm * 2;
        REQUIRE(all_finite(d, nm) && all_finite(t_in, nm), DM_EINVAL, "inputs must be finite");
        prepare_filters(p, std::vector<double>{lambda});
        double *dd = nullptr, *dt = nullptr;
        auto del = [](double* x) { if (x) (void)hipFree(x); };
        HIPCHK(hipMalloc((void**)&dd, nm * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g1(dd, del);
        HIPCHK(hipMalloc((void**)&dt, nm * sizeof(double)));
        std::unique_ptr<double, decltype(del)> g2(dt, del);
        upload(p, dd, d, nm);
        upload(p, dt, t_in, nm);
        HIPCHK(launch_data_setup(p, nrhs, dd, p->d_d0, p->d_b, p->stream));
        ring(p, RING_ANALYSIS, nrhs, dt, nullptr, nullptr, p->stream);
        for (int i = 0; i < niter; ++i) {
            leg_analysis(p, nrhs, true, p->d_filters, p->d_alm, p->d_alm_spin, p->stream);
            leg_synthesis(p, nrhs, p->d_alm_spin, p->stream);
            messenger_step(p, nrhs, (i == niter - 1) ? dt : nullptr, p->stream);
        }
        HIPCHK(hipMemcpyAsync(alm, p->d_alm, na * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        if (t_out) HIPCHK(hipMemcpyAsync(t_out, dt, nm * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        if (p->profiling) collect_events(p);
    });
}

// current choices [syn mchunk, ana mchunk, syn waves, ring big threads, ring small threads]
static void tune_choice(const dm_plan* p, int* choice) {
    if (!choice) return;
    choice[0] = p->syn_mchunk;
    choice[1] = p->ana_mchunk;
    choice[2] = p->syn_waves;
    choice[3] = p->ring_big_threads;
    choice[4] = p->ring_small_threads;
}

dm_status dm_autotune(dm_plan* p, int nrhs, int* choice, double* ms) {
    return guarded(p, [&] {
        check_rhs(p, nrhs);
        if (ms) ms[0] = ms[1] = ms[2] = 0.0;
        const bool batched = use_mfma(p, nrhs);
        const bool classes = p->ring_classes && nrhs >= 4;
        if (!batched && !classes) {
            tune_choice(p, choice);
            return;
        }
        // cache key: grid, lmax, precision, column tiles of 8 RHS, ring classes in use
        char key[160];
        std::snprintf(key, sizeof key, "g%d_%d_%d_%d_l%d_p%d_t%d_c%d", p->grid.kind, p->grid.nside, p->grid.ntheta,
                      p->grid.nphi, p->lmax, (int)p->precision, (nrhs + 7) / 8, classes ? 1 : 0);
        const char* cache = std::getenv("DMWF_TUNE_CACHE");
        if (cache && cache[0]) {
            if (std::FILE* f = std::fopen(cache, "r")) {
                char k[160];
                int v[5];
                bool hit = false;
                while (std::fscanf(f, "%159s %d %d %d %d %d", k, &v[0], &v[1], &v[2], &v[3], &v[4]) == 6)
                    if (std::strcmp(k, key) == 0 && v[0] >= 0 && v[0] <= 16 && v[1] >= 0 && v[1] <= 16 &&
                        (v[2] == 1 || v[2] == 2 || v[2] == 4 || v[2] == 8) && (v[3] == 512 || v[3] == 1024) &&
                        (v[4] == 256 || v[4] == 512 || v[4] == 1024)) {
                        p->syn_mchunk = v[0];
                        p->ana_mchunk = v[1];
                        p->syn_waves = v[2];
                        p->ring_big_threads = v[3];
                        p->ring_small_threads = v[4];
                        hit = true;
                    }
                std::fclose(f);
                if (hit) {
                    tune_choice(p, choice);
                    return;
                }
            }
        }
        HIPCHK(hipStreamSynchronize(p->stream));
        const void* phase = phase_of(p, nrhs);
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        struct Ev2 {
            hipEvent_t a, b;
            ~Ev2() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
        } guard{e0, e1};
        // best of three launches after a warm-up
        auto timeit = [&](auto launch) {
            HIPCHK(launch());
            float best = 1e30f;
            for (int r = 0; r < 3; ++r) {
                HIPCHK(hipEventRecord(e0, p->stream));
                HIPCHK(launch());
                HIPCHK(hipEventRecord(e1, p->stream));
                HIPCHK(hipEventSynchronize(e1));
                float t = 0.f;
                HIPCHK(hipEventElapsedTime(&t, e0, e1));
                best = std::min(best, t);
            }
            return (double)best;
        };
        double best_syn = 0.0, best_ana = 0.0, best_ring = 0.0;
        if (batched) {
            // synthesis: waves per block x m-chunk; analysis: m-chunk.  Both
            // only move work between waves, blocks and XCDs: the arithmetic
            // of every output stays the same, to the last bit
            const int cand[] = {0, 1, 2, 4, 8};
            const int waves[] = {1, 2, 4, 8};
            best_syn = best_ana = 1e300;
            int syn = p->syn_mchunk, ana = p->ana_mchunk, sw = p->syn_waves;
            p->mfma_nct = 1;
            for (int w : waves)
                for (int c : cand) {
                    p->syn_waves = w;
                    p->syn_mchunk = c;
                    const double t =
                        timeit([&] { return launch_bsyn(p, nrhs, p->d_alm_spin, const_cast<void*>(phase), p->stream); });
                    if (t < best_syn) { best_syn = t; syn = c; sw = w; }
                }
            for (int c : cand) {
                p->ana_mchunk = c;
                const double t = timeit([&] { return launch_bana(p, nrhs, phase, p->d_pair_w, p->d_partial, p->stream); });
                if (t < best_ana) { best_ana = t; ana = c; }
            }
            p->syn_mchunk = syn;
            p->ana_mchunk = ana;
            p->syn_waves = sw;
        }
        if (classes) {
            // the ring step's two launches: workgroup widths of the large and
            // the small transforms (a width changes the order in which a few
            // first-pixel rotations are accumulated: results move by FP64
            // rounding only), timed on the pixel-update pass
            const int bigc[] = {512, 1024}, smallc[] = {256, 512, 1024};
            best_ring = 1e300;
            int rb = p->ring_big_threads, rs = p->ring_small_threads;
            for (int b : bigc)
                for (int c : smallc) {
                    p->ring_big_threads = b;
                    p->ring_small_threads = c;
                    const double t = timeit([&] {
                        return launch_ring(p, RING_ITERATE, nrhs, nullptr, nullptr, p->d_K, p->d_b,
                                           const_cast<void*>(phase), phase32(p, nrhs), p->stream);
                    });
                    if (t < best_ring) { best_ring = t; rb = b; rs = c; }
                }
            p->ring_big_threads = rb;
            p->ring_small_threads = rs;
        }
        tune_choice(p, choice);
        if (ms) { ms[0] = best_syn; ms[1] = best_ana; ms[2] = best_ring; }
        if (cache && cache[0])
            if (std::FILE* f = std::fopen(cache, "a")) {
                std::fprintf(f, "%s %d %d %d %d %d\n", key, p->syn_mchunk, p->ana_mchunk, p->syn_waves,
                             p->ring_big_threads, p->ring_small_threads);
                std::fclose(f);
            }
    });
}

dm_status dm_profile_enable(dm_plan* p, int enable) {
    return guarded(p, [&] {
        HIPCHK(hipStreamSynchronize(p->stream));
        collect_events(p);
        p->profiling = enable != 0;
        for (int k = 0; k < KC_COUNT; ++k) {
            p->kc_ms[k] = 0;
            p->kc_n[k] = 0;
        }
    });
}

dm_status dm_kernel_times(dm_plan* p, double* ms, int64_t* launches, int* count) {
    return guarded(p, [&] {
        REQUIRE(ms && launches && count, DM_EINVAL, "null argument");
        HIPCHK(hipDeviceSynchronize());
        collect_events(p);
        const int n = std::min(*count, (int)KC_COUNT);
        for (int k = 0; k < n; ++k) {
            ms[k] = p->kc_ms[k];
            launches[k] = p->kc_n[k];
        }
        *count = KC_COUNT;
    });
}

}  // extern "C"
