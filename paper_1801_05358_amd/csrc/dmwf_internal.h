// Internal declarations of libdmwf: the plan, its device tables and the
// kernel launchers.  Not part of the public ABI (include/dmwf.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmwf.h"

namespace dmwf {

// Recursion coefficients per packed (l, m), producing the value at l from
// the values at l-1 and l-2 (see legendre.hip).
constexpr int kCoefStride = 6;   // A0, B0, alpha, alpha*beta, gamma, pad
constexpr int kCoefSStride = 4;  // scaled recursions: A0', alpha', (alpha*beta)', pad

// Per-(m, ring pair) recursion seeds: values at (ls-1, ls) of
// lam, (+2)lam, (-2)lam (for m < 2 the spin-2 slots hold l = 1, 2).
constexpr int kSeedFields = 6;

// Kernel classes for the optional event timing.
enum KernelClass { KC_LEG_ANALYSIS = 0, KC_LEG_SYNTHESIS = 1, KC_RING = 2, KC_COMBINE = 3, KC_PIXEL = 4, KC_COUNT = 5 };

struct RingTables {
    // per ring
    std::vector<double> z;        // cos(theta)
    std::vector<double> phi0;     // first pixel longitude
    std::vector<double> w;        // per-pixel quadrature weight
    std::vector<int> nphi;
    std::vector<int64_t> offset;
    // per ring pair (north ring p, south ring mirror or -1)
    std::vector<int> pair_n, pair_s;
};

struct FftTables {
    // distinct ring lengths
    std::vector<int> n;           // length
    std::vector<int> split;       // 1: n = 4 i transformed as four length-i DFTs
    std::vector<int> M;           // transform size: n for n = 2^k or 3 2^k (direct), else the
                                  // Bluestein size of n (or of n/4 when split): the smaller of
                                  // 2^a and 3 2^b that is >= 2n - 1
    std::vector<int> logM;        // log2 of M's power-of-two factor
    std::vector<int> r3;          // 1: M = 3 2^logM (a radix-3 pass and three 2^logM blocks)
    std::vector<int64_t> chirp_off;   // offset into chirp (complex) or -1
    std::vector<int64_t> bhat_off;    // offset into bhat (complex) or -1
    int Mmax = 1;                 // largest power-of-two transform (the twiddle table's size)
    int lds_elems = 1;            // largest transform buffer of the unsplit lengths (complex elements)
    int lds_split = 1;            // the same for the split lengths: max(n, M)
    std::vector<double> chirp;    // interleaved complex, exp(-i pi j^2 / n)
    std::vector<double> bhat;     // interleaved complex, FFT_M(b) / M
    std::vector<double> tw;       // interleaved complex, exp(-2 pi i k / Mmax), k < Mmax/2
    int P3max = 1;                // largest power-of-two factor P of a radix-3 size 3P
    std::vector<double> tw3;      // interleaved complex, exp(-2 pi i e / (3 P3max)), e < 3 P3max
};

// Device view of everything the ring (FFT) kernel needs per pair.
struct RingPairDev {
    int nphi;
    int len_idx;      // index into the FFT length tables
    int has_s;        // south ring present
    int phi0_den;     // first-pixel longitude phi0 = pi / phi0_den (0: phi0 = 0)
    int64_t off_n, off_s;
};

struct FftLenDev {
    int n, M, logM, bluestein, split, r3;
    int64_t chirp_off, bhat_off;
};

struct GpuEvents {
    std::vector<hipEvent_t> start, stop;
    std::vector<int> cls;
};

}  // namespace dmwf

struct dm_plan {
    int device = 0;
    hipStream_t stream = nullptr;       // plan-owned stream (default priority)
    dm_grid grid{};
    int lmax = 0, mmax = 0;
    int64_t nalm = 0, npix = 0;
    int nrings = 0, npairs = 0;
    int max_rhs = 1;
    dm_precision precision = DM_FP64;
    std::string err;

    dmwf::RingTables rings;
    dmwf::FftTables fft;

    // device tables
    double* d_pair_x = nullptr;        // [npairs] cos theta of the north ring
    double* d_pair_w = nullptr;        // [npairs] pixel weight
    double* d_pair_one = nullptr;      // [npairs] ones (unweighted adjoint)
    dmwf::RingPairDev* d_pairs = nullptr;
    dmwf::FftLenDev* d_fftlen = nullptr;
    double* d_chirp = nullptr;
    double* d_bhat = nullptr;
    double* d_tw = nullptr;
    double* d_tw3 = nullptr;           // radix-3 twiddles
    float* d_chirp32 = nullptr;        // FP32 copies of the four tables (mixed plans)
    float* d_bhat32 = nullptr;
    float* d_tw32 = nullptr;
    float* d_tw332 = nullptr;
    double* d_coef = nullptr;          // [nalm][kCoefStride]
    double* d_coef_s = nullptr;        // [nalm][kCoefSStride] scaled recursions (batched kernels)
    double* d_scale = nullptr;         // [nalm][2] their scales S (spin 0, spin 2)
    int* d_lstart = nullptr;           // [mmax+1][npairs]
    int* d_slot_lo = nullptr;          // [mmax+1][batched analysis slots]: first start degree per slot
    double* d_seed = nullptr;          // [kSeedFields][mmax+1][npairs]
    double* d_lp0 = nullptr;           // [mmax+1] log seed prefactors, spin 0
    double* d_lp2 = nullptr;           // [mmax+1] log seed prefactors, spin 2

    // analysis tiling
    int ana_R = 2, ana_blocks = 1, ana_chunks = 1;   // chunks = partial-sum slots
    int mfma_nct = 1;                                 // column tiles (8 RHS each) of the batched kernels
    int mfma_mode = -1;                               // -1 auto, 0 off, 1 on (FP64 plans)
    int syn_threads = 128, syn_R = 1;
    int syn_mchunk = 4, ana_mchunk = 4;               // batched kernels: consecutive m per XCD chunk
    int fft_threads = 512;          // threads of a split-ring workgroup
    int ring_threads = 512;         // threads of a whole-ring workgroup (<= 1024)
    int ring_big_threads = 1024;    // the same for the two size classes' launches
    int ring_small_threads = 512;
    int syn_waves = 4;              // waves per block of the batched synthesis (2, 4 or 8)
    // ring pairs of the unsplit and the split lengths (the split launch runs
    // only when some length is split)
    int n_whole = 0, n_split = 0;
    int split_k = 2;                   // kappa values per lane of the split launch (2 or 4)
    int* d_plist_whole = nullptr;
    // the unsplit pairs in two launches by transform size (ring_classes,
    // used from 4 RHS per launch on): buffers up to 80 KB (two 512-thread
    // workgroups per CU) and the rest (one 1024-thread workgroup per CU)
    int ring_classes = 0;
    int fuse6 = 1;                     // 3x3 update inside the ring analysis pass
    int n_small = 0, n_big = 0, lds_small = 1, lds_big = 1;
    int* d_plist_small = nullptr;
    int* d_plist_big = nullptr;
    int* d_plist_split = nullptr;
    size_t fft_lds_bytes = 0;

    // noise
    bool noise_set = false;
    double tau = 0.0;
    int ncov_layout = DM_NCOV_DIAG3;   // of the last dm_set_noise
    double* d_K = nullptr;             // [3][npix]  1 - T N^-1        (diagonal noise)
    double* d_tn = nullptr;            // [3][npix]  T N^-1            (diagonal noise)
    double* d_ninv = nullptr;          // [3][npix]  N^-1, 0 unobserved (diagonal noise)
    double* d_ninv6 = nullptr;         // [6][npix]  P = N^-1 on observed components (3x3 noise)
    double* d_tn6 = nullptr;           // [6][npix]  T P (3x3 noise)
    uint8_t* d_obs = nullptr;          // [npix] bit 0: I observed, bit 1: Q and U observed
    double* d_ring_w = nullptr;        // [nrings] pixel weight per ring
    int64_t* d_ring_off = nullptr;     // [nrings]
    int* d_ring_n = nullptr;           // [nrings]

    // spectra / schedule
    bool spectra_set = false;
    std::vector<double> cl;            // [4][lmax+1]
    dm_schedule sched{1e3, 20, 10, 0.75, 1e-4, 1e-6, 1.1, 100000};

    // work buffers (sized for max_rhs)
    double* d_phase = nullptr;         // [B][3][npairs][mmax+1][2] complex
    float* d_phase32 = nullptr;        // the same in FP32, for the mixed transforms
    double* d_partial = nullptr;       // [chunks][B][3][nalm] complex
    double* d_alm = nullptr;           // [B][3][nalm] complex
    double* d_alm_prev = nullptr;      // [B][3][nalm] complex
    double* d_alm_spin = nullptr;      // [B][3][nalm] complex, (T, (2)a, (-2)a)
    double* d_d0 = nullptr;            // [B][3][npix]  masked data
    double* d_b = nullptr;             // [B][3][npix]  T N^-1 d
    double* d_ux = nullptr;            // [B][3][npix]  Y u (scratch)
    double* d_alm_r = nullptr;         // [B][3][nalm]  residual adjoint (scratch)
    double* d_alm_y = nullptr;         // [B][3][nalm]
    double* d_filters = nullptr;       // [nsteps][lmax+1][4]
    int filters_cap = 0;
    double* d_mats = nullptr;          // [3][lmax+1][4]  S^1/2, S^+1/2, S^+
    double* h_pinned = nullptr;        // pinned staging for filters
    size_t h_pinned_len = 0;
    double* d_red = nullptr;           // reduction scratch
    size_t red_len = 0;
    // epsilon-mode schedule: Cauchy terms per combine block and per RHS,
    // their pinned host copy, and the per-iteration record of the last solve
    double* d_cpart = nullptr;         // [max_rhs][cauchy_blocks][2]
    double* d_cout = nullptr;          // [max_rhs][2]
    double* h_cout = nullptr;          // pinned [max_rhs][2]
    std::vector<double> trace_cauchy;
    std::vector<int> trace_step;
    // refinement (Appendix A): corrections per solve, the correction's own
    // b and iterate (allocated when first enabled), and the relative
    // residual norms of the last solve, [ncorr + 1][nrhs]
    int refine = 0;
    double* d_b2 = nullptr;            // [B][3][npix]
    double* d_alm_corr = nullptr;      // [B][3][nalm] complex
    double* d_alm_best = nullptr;      // [B][3][nalm] complex (refine_best only)
    std::vector<double> refine_hist;
    int refine_nrhs = 0;
    int refine_best = 0;               // 0: the last iterate (Appendix A), 1: the one of smallest residual
    std::vector<int> refine_chosen;    // [nrhs] index in refine_hist of the returned iterate

    // adaptive working resolution: factor (0 = off) and the band limit of
    // each cooling step of the last prepared schedule
    double adaptive = 0.0;
    std::vector<int> step_lcut;
    int lcut = 0;                      // band limit of the transforms being launched (lmax: full)

    // diagnostics trace (Fig. 4): chi^2 (eq 3) and the Appendix C residual
    // of the iterate after every diag_every-th iteration and after the last;
    // [entries][nrhs] per quantity, the iteration of each entry
    int diag_every = 0;
    bool diag_active = false;          // during a solve's own iterations (not refinement runs)
    int64_t diag_count = 0;            // iterations of the current solve so far
    int diag_nrhs = 0;
    std::vector<int> diag_iter;
    std::vector<double> diag_chi2, diag_resid;

    // input fingerprints (checked when a solve resumes from a checkpoint)
    uint64_t hash_cl = 0, hash_noise = 0;
    // where the last Wiener filter solve stopped: its iterate u in d_state_u,
    // the one before it in d_alm_prev (fixed mode), the position in the
    // schedule and the fingerprint of its masked data
    struct SolveState {
        bool valid = false;
        int nrhs = 0;
        int64_t iterations = 0;        // completed, counted from the schedule's start
        int next_step = 0;             // epsilon mode: cooling step of the next iteration
        bool finished = false;         // the schedule ran to its end
        uint64_t hash_data = 0, hash_noise = 0, hash_cl = 0;
        dm_schedule sched{};
        std::vector<double> last_c;    // epsilon mode: last Cauchy ratio per RHS
    } state;
    double* d_state_u = nullptr;       // [B][3][nalm] complex
    // a loaded checkpoint, consumed by the next Wiener filter solve
    struct Resume {
        bool pending = false;
        SolveState st;
        std::vector<double> trace_cauchy;
        std::vector<int> trace_step;
        std::vector<double> u, uprev;  // [nrhs][3][nalm][2]
        bool has_prev = false;
    } resume;

    // timing
    bool profiling = false;
    bool graphs = true;                // fixed-mode cooling steps as HIP graphs (DMWF_GRAPHS=0: off)
    double kc_ms[dmwf::KC_COUNT] = {0, 0, 0, 0, 0};
    int64_t kc_n[dmwf::KC_COUNT] = {0, 0, 0, 0, 0};
    dmwf::GpuEvents ev;
};

namespace dmwf {

// tables.cpp
bool build_rings(const dm_grid& g, RingTables& rt, int64_t& npix, std::string& err);
void build_scaled_coefficients(int lmax, std::vector<double>& coef_s, std::vector<double>& scale);
void build_coefficients(int lmax, std::vector<double>& coef, std::vector<double>& lp0,
                        std::vector<double>& lp2);
// lengths whose Bluestein buffer would exceed max_elems are split
bool build_fft_tables(const RingTables& rt, int mmax, int max_elems, FftTables& ft, std::string& err);
void build_filter(const std::vector<double>& cl, int lmax, double mu, double tau, std::vector<double>& F);
void build_matrix_function(const std::vector<double>& cl, int lmax, int which, std::vector<double>& F);

// legendre.hip
hipError_t launch_seeds(dm_plan* p, hipStream_t s);
// synthesis reads alm in the spin basis (T, (2)a, (-2)a)
hipError_t launch_leg_synthesis(dm_plan* p, int nrhs, const double* spin_alm, double* phase, hipStream_t s);
// analysis writes chunk partials of (T, (2)a, (-2)a); combine sums them,
// converts to (T, E, B), applies the filter (may be null) and optionally
// writes the spin-basis copy for the next synthesis (spin may be null).
hipError_t launch_leg_analysis(dm_plan* p, int nrhs, const double* phase, const double* pair_w,
                               double* partial, hipStream_t s);
// scale (nullable): the batched kernels' recursion scales, applied to the
// partial sums and to the spin-basis copy; partial32: the slots hold FP32
// (the mixed batched analysis), else FP64; slot_lo (nullable, [mmax+1][nslots]):
// slot c holds degrees l >= slot_lo[m][c] only (the batched analysis)
hipError_t launch_combine(dm_plan* p, int nrhs, int nslots, const double* partial, bool partial32,
                          const int* slot_lo, const double* filter, double* alm, double* spin, double* cpart,
                          const double* scale, hipStream_t s);
int64_t cauchy_blocks(dm_plan* p);   // Cauchy partial sums per RHS written by the combine kernel
hipError_t launch_cauchy_reduce(dm_plan* p, int nrhs, const double* cpart, double* out, hipStream_t s);
hipError_t launch_to_spin(dm_plan* p, int nrhs, const double* alm, double* spin, const double* scale,
                          hipStream_t s);
void set_analysis_tiling(dm_plan* p, int R);

// legendre_mfma.hip: batched Legendre products on the matrix cores
// (FP64 for DM_FP64 plans, FP32 for DM_MIXED); analysis writes one
// partial-sum slot per block of ring pairs
int batched_analysis_slots(dm_plan* p);
// the first start degree of each (m, slot) from the plan's start degrees
hipError_t launch_slot_starts(dm_plan* p, int* slot_lo, hipStream_t s);
// batched kernels: phase is FP32 ring data for DM_MIXED, FP64 otherwise
hipError_t launch_bsyn(dm_plan* p, int nrhs, const double* spin, void* phase, hipStream_t s);
hipError_t launch_bana(dm_plan* p, int nrhs, const void* phase, const double* pair_w, double* partial,
                       hipStream_t s);

// ringfft.hip
enum RingMode { RING_ANALYSIS = 1, RING_SYNTH = 2, RING_ITERATE = 3, RING_ANALYSIS6 = 4 };
// RING_ANALYSIS: map -> phase.  RING_SYNTH: phase -> map.
// RING_ITERATE: phase -> (K x + b) -> phase.
// RING_ITERATE with map_out != null also stores the updated messenger t.
// RING_ANALYSIS6: u_x map -> (the 3x3 update t = u_x - T_p P_p u_x + b) ->
// phase, with K the T_p P_p entries [6][npix] (II IQ IU QQ QU UU).
// phase: FP32 ring data if phase32, else FP64
hipError_t launch_ring(dm_plan* p, int mode, int nrhs, const double* map_in, double* map_out,
                       const double* K, const double* b, void* phase, bool phase32, hipStream_t s);
hipError_t ring_set_lds_limit(size_t bytes);

// pointwise.hip
// alpha_p w_p per pixel with an observed component, min-reduced per ring
// -> ring_min [nrings]; with 3x3 noise also P_p -> d_ninv6.  The mask bits
// are d_obs, the layout p->ncov_layout.
hipError_t launch_tau_parts(dm_plan* p, const double* ncov, double* ring_min, hipStream_t s);
// K, T N^-1 and N^-1 (diagonal) or T P (3x3) from the noise, the mask and tau
hipError_t launch_noise_setup(dm_plan* p, const double* ncov, double tau, hipStream_t s);
// d0 = d on observed components, b = T N^-1 d0
hipError_t launch_data_setup(dm_plan* p, int nrhs, const double* d, double* d0, double* b, hipStream_t s);
// 3x3 noise, in place: ux <- ux - T P ux + b; t_out (nullable) gets a copy
hipError_t launch_update6(dm_plan* p, int nrhs, double* ux, const double* b, double* t_out, hipStream_t s);
// in place: ux <- N^-1 (ux - d0), b <- N^-1 d0 (b nullable: not written);
// chi_parts [nrhs][nrings] = sum (d0-ux)^T N^-1 (d0-ux)
hipError_t launch_residual_maps(dm_plan* p, int nrhs, double* ux, const double* d0, double* b,
                                double* chi_parts, hipStream_t s);
// fingerprint of a buffer of n elements of elem_bytes (1 or 8) bytes:
// sum over i of mix(v_i + i g) mod 2^64, accumulated into *acc (which the
// caller zeroes); integer sums, so the value does not depend on the order
hipError_t launch_hash(const void* buf, int64_t n, int elem_bytes, uint64_t* acc, hipStream_t s);
uint64_t hash_mix(uint64_t x);
// per (rhs, m, block) sums: |u-uprev|^2, |u|^2, |r|^2, |y|^2, u^T S^+ u
constexpr int kNormQ = 5;
int alm_norm_blocks(dm_plan* p);
hipError_t launch_alm_norms(dm_plan* p, int nrhs, const double* u, const double* uprev, const double* r1,
                            const double* y1, const double* mats, double* parts, hipStream_t s);
hipError_t launch_count_nonfinite(const double* x, int64_t n, int* count, hipStream_t s);
// y = (double) x, y = (float) x, elementwise
hipError_t launch_widen(double* y, const float* x, int64_t n, hipStream_t s);
hipError_t launch_narrow(float* y, const double* x, int64_t n, hipStream_t s);
// y = a * x + c * y  (elementwise)
hipError_t launch_axpby(double* y, const double* x, double a, double c, int64_t n, hipStream_t s);
// refinement residual per (l, m): e <- Pi e + S^+ u in place; parts [blocks][2]
// = (|e|^2, |Pi y|^2) per block, blocks as alm_norm_blocks (y nullable)
hipError_t launch_refine_residual(dm_plan* p, int nrhs, double* e, const double* u, const double* y, double* parts,
                                  hipStream_t s);
// y = a x
hipError_t launch_scale(double* y, const double* x, double a, int64_t n, hipStream_t s);

}  // namespace dmwf
