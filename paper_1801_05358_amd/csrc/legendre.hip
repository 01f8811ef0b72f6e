// Legendre step of the spin-0 + spin-2 spherical harmonic transforms
// (the basis change of Algorithm 1, replacing the flat-sky eqs 12-16 on the
// sphere): recursion seeds, synthesis (alm -> ring Fourier coefficients),
// analysis (ring Fourier coefficients -> alm) and the per-(l, m) 3x3
// messenger filter of eq 8, fused into the analysis epilogue.
//
// Functions: for a ring pair (theta, pi - theta) with x = cos(theta):
//   lam_lm(theta)   spin-0 orthonormal Legendre function,
//   p_lm = (+2)lam_lm, q_lm = (-2)lam_lm   spin +-2 functions,
// with lam(pi - theta) = (-1)^(l+m) lam(theta) and p(pi - theta) =
// (-1)^(l+m) q(theta).  The two spin-2 functions are recursed separately:
// near a pole one of them is many orders of magnitude below the other, and
// any sum/difference form would lose it to cancellation.
// Polarization works in the spin basis (+-2)a = -(a^E +- i a^B):
// synthesis per m:  F^T = sum_l a^T lam,  (Q + iU)_m = sum_l (2)a p,
//                   (Q - iU)_m = sum_l (-2)a q;
// analysis per m (w = pixel weight, G = ring Fourier coefficients):
//   a^T = sum_r w lam G^T,  (2)a = sum_r w p G^{Q+iU},  (-2)a = sum_r w q G^{Q-iU},
//   a^E = -((2)a + (-2)a)/2,  a^B = i((2)a - (-2)a)/2.
//
// Each (m, ring pair) starts its recursion at the first l where one of
// lam, p, q exceeds 2^-100 (all earlier terms are below that and are
// skipped).  The seeds at that l are found once per plan by a recursion
// that carries an explicit binary exponent (the values at l = m underflow
// double precision near the poles for large m).
#include "dmwf_internal.h"

namespace dmwf {

namespace {

constexpr double kLn2 = 0.69314718055994530942;
constexpr double kThr = 7.888609052210118e-31;   // 2^-100

__device__ __forceinline__ int64_t mbase(int m, int lmax) {
    return (int64_t)m * (2 * lmax + 1 - m) / 2;
}

__device__ __forceinline__ int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

struct LegArgs {
    int lmax, mmax, npairs;
    int lend;             // band limit of this launch: degrees and orders above it are skipped
    int64_t nalm;
    const double* __restrict__ pair_x;
    const double* __restrict__ coef;    // scaled recursions, [nalm][kCoefSStride]
    const double* __restrict__ scale;   // their scales S, [nalm][2]
    const int* __restrict__ lstart;
    const double* __restrict__ seed;
    int64_t sstride;      // (mmax + 1) * npairs
};

LegArgs leg_args(dm_plan* p) {
    LegArgs a;
    a.lmax = p->lmax;
    a.mmax = p->mmax;
    a.npairs = p->npairs;
    a.nalm = p->nalm;
    a.pair_x = p->d_pair_x;
    a.coef = p->d_coef_s;
    a.scale = p->d_scale;
    a.lstart = p->d_lstart;
    a.seed = p->d_seed;
    a.sstride = (int64_t)(p->mmax + 1) * p->npairs;
    a.lend = (p->lcut > 0 && p->lcut < p->lmax) ? p->lcut : p->lmax;
    return a;
}

// ---------------------------------------------------------------------------
// seeds
// ---------------------------------------------------------------------------
__global__ void seed_kernel(int lmax, int npairs, const double* __restrict__ pair_x,
                            const double* __restrict__ coef, const double* __restrict__ lp0,
                            const double* __restrict__ lp2, int* __restrict__ lstart,
                            double* __restrict__ seed, int64_t sstride) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (p >= npairs) return;
    const double x = pair_x[p];
    const double s = sqrt((1.0 - x) * (1.0 + x));
    const int64_t o = (int64_t)m * npairs + p;
    double v[6];
    int ls;
    if (m < 2) {
        // spin-0 from l = m; spin-2 slots hold (l = 1, l = 2)
        const double fourpi = 4.0 * M_PI;
        ls = m;
        v[0] = 0.0;
        v[1] = (m == 0) ? 1.0 / sqrt(fourpi) : -sqrt(3.0 / (2.0 * fourpi)) * s;
        v[2] = 0.0;
        v[3] = (m == 0) ? sqrt(15.0 / (8.0 * fourpi)) * s * s : -sqrt(5.0 / (4.0 * fourpi)) * s * (1.0 - x);
        v[4] = 0.0;
        v[5] = (m == 0) ? sqrt(15.0 / (8.0 * fourpi)) * s * s : sqrt(5.0 / (4.0 * fourpi)) * s * (1.0 + x);
    } else {
        // l = m:  lam = (-1)^m e^{lp0} s^m,
        //         p = (-1)^m e^{lp2} (s/2)^(m-2) (1 - x)^2 / 4,
        //         q = (-1)^m e^{lp2} (s/2)^(m-2) (1 + x)^2 / 4
        const double lsn = log(s);
        const double logl = lp0[m] + m * lsn;
        const double logw = lp2[m] + (m - 2) * (lsn - kLn2);
        const double sg = (m & 1) ? -1.0 : 1.0;
        int E = (int)floor(fmax(logl, logw) / kLn2);
        double cl = sg * exp(logl - E * kLn2);
        const double ew = sg * exp(logw - E * kLn2) * 0.25;
        double cw = ew * (1.0 - x) * (1.0 - x);
        double cx = ew * (1.0 + x) * (1.0 + x);
        double pl = 0.0, pw = 0.0, px = 0.0;
        const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
        int l = m;
        for (;;) {
            const double mx = fmax(fabs(cl), fmax(fabs(cw), fabs(cx)));
            if (E > -1200 && ldexp(mx, E) > kThr) break;
            if (l == lmax) { l = lmax + 1; break; }
            const double* c = coef + (base + l + 1) * kCoefStride;
            const double ax = c[0] * x, bx = c[2] * x;
            const double nl = ax * cl - c[1] * pl;
            const double nw = (bx + c[3]) * cw - c[4] * pw;
            const double nx = (bx - c[3]) * cx - c[4] * px;
            pl = cl; pw = cw; px = cx;
            cl = nl; cw = nw; cx = nx;
            ++l;
            const double m2 = fmax(fabs(cl), fmax(fabs(cw), fabs(cx)));
            if (m2 > 0x1p400) {
                cl *= 0x1p-400; cw *= 0x1p-400; cx *= 0x1p-400;
                pl *= 0x1p-400; pw *= 0x1p-400; px *= 0x1p-400;
                E += 400;
            }
        }
        ls = l;
        if (l <= lmax) {
            v[0] = ldexp(pl, E); v[1] = ldexp(cl, E);
            v[2] = ldexp(pw, E); v[3] = ldexp(cw, E);
            v[4] = ldexp(px, E); v[5] = ldexp(cx, E);
        } else {
            for (int k = 0; k < 6; ++k) v[k] = 0.0;
        }
    }
    lstart[o] = ls;
    for (int k = 0; k < 6; ++k) seed[k * sstride + o] = v[k];
}

// One step to degree l of the scaled recursions (mu = lam / S, the degree
// l-2 term with coefficient 1; the combine step and the spin-basis copy
// apply S) for R ring pairs: lam (l0, l1), p = (+2)lam (w0, w1),
// q = (-2)lam (q0, q1) hold degrees (l-2, l-1).
template <int R>
__device__ __forceinline__ void advance(const double* __restrict__ c, const double* x, double* l0,
                                        double* l1, double* w0, double* w1, double* q0, double* q1) {
    const double A0 = c[0], al = c[1], ab = c[2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double ax = A0 * x[r];
        const double cw = al * x[r] + ab, cq = al * x[r] - ab;
        const double nl = ax * l1[r] - l0[r];
        const double nw = cw * w1[r] - w0[r];
        const double nq = cq * q1[r] - q0[r];
        l0[r] = l1[r]; l1[r] = nl;
        w0[r] = w1[r]; w1[r] = nw;
        q0[r] = q1[r]; q1[r] = nq;
    }
}

// Activation of lanes whose recursion starts at degree l.
template <int R>
__device__ __forceinline__ void activate(const LegArgs& A, int m, int l, const int* ls, const int* pr,
                                         double* l0, double* l1, double* w0, double* w1, double* q0,
                                         double* q1) {
    // seeds lam at (l-1, l) become mu = lam / S (a degree below m holds 0)
    const double* sc = A.scale + mbase(m, A.lmax) * 2;
    auto inv = [&](int d, int k) { return 1.0 / sc[(int64_t)min(max(d, m), A.lmax) * 2 + k]; };
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t o = (int64_t)m * A.npairs + pr[r];
        if (l == ls[r]) {
            l0[r] = A.seed[0 * A.sstride + o] * inv(l - 1, 0);
            l1[r] = A.seed[1 * A.sstride + o] * inv(l, 0);
            if (m >= 2) {
                w0[r] = A.seed[2 * A.sstride + o] * inv(l - 1, 1);
                w1[r] = A.seed[3 * A.sstride + o] * inv(l, 1);
                q0[r] = A.seed[4 * A.sstride + o] * inv(l - 1, 1);
                q1[r] = A.seed[5 * A.sstride + o] * inv(l, 1);
            }
        }
        if (m < 2 && l == 2 && ls[r] <= A.lmax) {
            w0[r] = A.seed[2 * A.sstride + o] * inv(1, 1);
            w1[r] = A.seed[3 * A.sstride + o] * inv(2, 1);
            q0[r] = A.seed[4 * A.sstride + o] * inv(1, 1);
            q1[r] = A.seed[5 * A.sstride + o] * inv(2, 1);
        }
    }
}

// Recursion state of R ring pairs held by one thread.
template <int R>
struct RecState {
    double x[R], l0[R], l1[R], w0[R], w1[R], q0[R], q1[R];
    int ls[R], pr[R];
};

template <int R>
__device__ __forceinline__ void rec_init(RecState<R>& S, const LegArgs& A, int m, int p0, int stride, int& lo,
                                         int& hi) {
    lo = A.lmax + 1;
    hi = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int p = p0 + r * stride;
        const bool ok = p < A.npairs;
        S.pr[r] = ok ? p : 0;
        S.x[r] = ok ? A.pair_x[p] : 0.0;
        S.ls[r] = ok ? A.lstart[(int64_t)m * A.npairs + p] : A.lmax + 1;
        S.l0[r] = S.l1[r] = S.w0[r] = S.w1[r] = S.q0[r] = S.q1[r] = 0.0;
        lo = min(lo, S.ls[r]);
        hi = max(hi, S.ls[r] <= A.lmax ? S.ls[r] : 0);
    }
}

// ---------------------------------------------------------------------------
// synthesis: spin-basis alm [B][3][nalm] complex -> phase [B][3][npairs][mmax+1][2]
// ---------------------------------------------------------------------------
// acc[r][PAR*10 + k], PAR = (l + m) & 1:  k = 0,1 a^T lam;  2,3 (2)a p;
// 4,5 (-2)a q;  6,7 (2)a q;  8,9 (-2)a p   (re, im)
template <int R, int PAR, bool ADV, bool ACT>
__device__ __forceinline__ void synth_step(const LegArgs& A, int m, int l, const double* __restrict__ cf,
                                           const double2* __restrict__ aT, const double2* __restrict__ aP,
                                           const double2* __restrict__ aM, RecState<R>& S, double (&acc)[R][20]) {
    if (ADV) advance<R>(cf + (int64_t)l * kCoefSStride, S.x, S.l0, S.l1, S.w0, S.w1, S.q0, S.q1);
    if (ACT) activate<R>(A, m, l, S.ls, S.pr, S.l0, S.l1, S.w0, S.w1, S.q0, S.q1);
    const double2 t = aT[l], e = aP[l], b = aM[l];
    constexpr int o = PAR * 10;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double lam = S.l1[r], pp = S.w1[r], qq = S.q1[r];
        acc[r][o + 0] = fma(lam, t.x, acc[r][o + 0]);
        acc[r][o + 1] = fma(lam, t.y, acc[r][o + 1]);
        acc[r][o + 2] = fma(pp, e.x, acc[r][o + 2]);
        acc[r][o + 3] = fma(pp, e.y, acc[r][o + 3]);
        acc[r][o + 4] = fma(qq, b.x, acc[r][o + 4]);
        acc[r][o + 5] = fma(qq, b.y, acc[r][o + 5]);
        acc[r][o + 6] = fma(qq, e.x, acc[r][o + 6]);
        acc[r][o + 7] = fma(qq, e.y, acc[r][o + 7]);
        acc[r][o + 8] = fma(pp, b.x, acc[r][o + 8]);
        acc[r][o + 9] = fma(pp, b.y, acc[r][o + 9]);
    }
}

template <int R>
__global__ __launch_bounds__(256) void leg_synth_kernel(LegArgs A, const double2* __restrict__ alm,
                                                        double2* __restrict__ phase) {
    const int m = blockIdx.y;
    const int rhs = blockIdx.z;
    const int lmax = A.lmax;
    const int lend = A.lend;          // degrees above it contribute nothing (zero coefficients)
    const int64_t base = mbase(m, lmax);
    const double2* __restrict__ aT = alm + (int64_t)rhs * 3 * A.nalm + base;
    const double2* __restrict__ aP = aT + A.nalm;
    const double2* __restrict__ aM = aP + A.nalm;
    const double* __restrict__ cf = A.coef + base * kCoefSStride;
    const int nt = blockDim.x, tid = threadIdx.x;

    RecState<R> S;
    double acc[R][20];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < 20; ++k) acc[r][k] = 0.0;
    int lo, hi;
    rec_init<R>(S, A, m, blockIdx.x * R * nt + tid, nt, lo, hi);
    // the degree loop is uniform across the wave
    lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    if (m < 2) hi = max(hi, 2);

    int l = lo;
    if (l <= lend) {
        // activation phase: some lanes start their recursion at l
        if ((l + m) & 1) synth_step<R, 1, false, true>(A, m, l, cf, aT, aP, aM, S, acc);
        else synth_step<R, 0, false, true>(A, m, l, cf, aT, aP, aM, S, acc);
        ++l;
        const int h = min(hi, lend);
        for (; l <= h; ++l) {
            if ((l + m) & 1) synth_step<R, 1, true, true>(A, m, l, cf, aT, aP, aM, S, acc);
            else synth_step<R, 0, true, true>(A, m, l, cf, aT, aP, aM, S, acc);
        }
        // steady state: every lane active, parity unrolled
        if (l <= lend && ((l + m) & 1)) {
            synth_step<R, 1, true, false>(A, m, l, cf, aT, aP, aM, S, acc);
            ++l;
        }
        for (; l + 1 <= lend; l += 2) {
            synth_step<R, 0, true, false>(A, m, l, cf, aT, aP, aM, S, acc);
            synth_step<R, 1, true, false>(A, m, l + 1, cf, aT, aP, aM, S, acc);
        }
        if (l <= lend) synth_step<R, 0, true, false>(A, m, l, cf, aT, aP, aM, S, acc);
    }

    const int64_t fstride = (int64_t)A.npairs * (A.mmax + 1) * 2;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int p = blockIdx.x * R * nt + r * nt + tid;
        if (p >= A.npairs) continue;
        const double* e = acc[r];       // even l+m: [0..9], odd: [10..19]
        // T on the north and south rings
        const double TNr = e[0] + e[10], TNi = e[1] + e[11];
        const double TSr = e[0] - e[10], TSi = e[1] - e[11];
        // (Q + iU) = P, (Q - iU) = M; south ring: p(pi-theta) = (-1)^(l+m) q(theta)
        const double PNr = e[2] + e[12], PNi = e[3] + e[13];
        const double MNr = e[4] + e[14], MNi = e[5] + e[15];
        const double PSr = e[6] - e[16], PSi = e[7] - e[17];
        const double MSr = e[8] - e[18], MSi = e[9] - e[19];
        // Q = (P + M)/2, U = (P - M)/(2i)
        double2* out = phase + (((int64_t)rhs * 3) * A.npairs + p) * (A.mmax + 1) * 2 + (int64_t)m * 2;
        out[0] = make_double2(TNr, TNi);
        out[1] = make_double2(TSr, TSi);
        out += fstride;
        out[0] = make_double2(0.5 * (PNr + MNr), 0.5 * (PNi + MNi));
        out[1] = make_double2(0.5 * (PSr + MSr), 0.5 * (PSi + MSi));
        out += fstride;
        out[0] = make_double2(0.5 * (PNi - MNi), -0.5 * (PNr - MNr));
        out[1] = make_double2(0.5 * (PSi - MSi), -0.5 * (PSr - MSr));
    }
}

// ---------------------------------------------------------------------------
// analysis: phase -> partial sums [slot][B][3][nalm] complex of
// (a^T, (2)a, (-2)a), one slot per wave of 64 lanes x R ring pairs.
// Each wave reduces its own lanes through a private LDS tile every kAnaL
// degrees, so no block-wide barrier sits inside the degree loop.
// ---------------------------------------------------------------------------
constexpr int kAnaThreads = 256;               // 4 independent waves
constexpr int kAnaL = 4;                       // degrees per reduction round
constexpr int kAnaRow = 66;                    // padded LDS row (64 lanes)
constexpr int kAnaTile = kAnaL * 6 * kAnaRow;  // doubles per wave

// weighted ring data of R ring pairs: T sum/difference; P = Q + iU and
// M = Q - iU on the north (n) and south (s) rings
template <int R>
struct AnaData {
    double Ts[R][2], Ta[R][2], Pn[R][2], Ps[R][2], Mn[R][2], Ms[R][2];
};

// c = (a^T, (2)a, (-2)a) contributions at degree l, summed over the lane's
// ring pairs:  (2)a += p P_n + eps q P_s,  (-2)a += q M_n + eps p M_s,
// eps = (-1)^(l+m); written to the lane's column of the degree's rows.
template <int R, int PAR, bool ADV, bool ACT>
__device__ __forceinline__ void ana_step(const LegArgs& A, int m, int l, const double* __restrict__ cf,
                                         RecState<R>& S, const AnaData<R>& D, double* slot) {
    if (ADV) advance<R>(cf + (int64_t)l * kCoefSStride, S.x, S.l0, S.l1, S.w0, S.w1, S.q0, S.q1);
    if (ACT) activate<R>(A, m, l, S.ls, S.pr, S.l0, S.l1, S.w0, S.w1, S.q0, S.q1);
    double c[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double lam = S.l1[r], pp = S.w1[r], qq = S.q1[r];
        if (PAR) {
            c[0] = fma(lam, D.Ta[r][0], c[0]);
            c[1] = fma(lam, D.Ta[r][1], c[1]);
            c[2] = fma(pp, D.Pn[r][0], fma(-qq, D.Ps[r][0], c[2]));
            c[3] = fma(pp, D.Pn[r][1], fma(-qq, D.Ps[r][1], c[3]));
            c[4] = fma(qq, D.Mn[r][0], fma(-pp, D.Ms[r][0], c[4]));
            c[5] = fma(qq, D.Mn[r][1], fma(-pp, D.Ms[r][1], c[5]));
        } else {
            c[0] = fma(lam, D.Ts[r][0], c[0]);
            c[1] = fma(lam, D.Ts[r][1], c[1]);
            c[2] = fma(pp, D.Pn[r][0], fma(qq, D.Ps[r][0], c[2]));
            c[3] = fma(pp, D.Pn[r][1], fma(qq, D.Ps[r][1], c[3]));
            c[4] = fma(qq, D.Mn[r][0], fma(pp, D.Ms[r][0], c[4]));
            c[5] = fma(qq, D.Mn[r][1], fma(pp, D.Ms[r][1], c[5]));
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) slot[k * kAnaRow] = c[k];
}

template <int R>
__device__ __forceinline__ void ana_step_any(const LegArgs& A, int m, int l, int lo, int hi,
                                             const double* __restrict__ cf, RecState<R>& S, const AnaData<R>& D,
                                             double* slot) {
    const bool par = (l + m) & 1;
    if (l > lo) {
        if (l <= hi) {
            if (par) ana_step<R, 1, true, true>(A, m, l, cf, S, D, slot);
            else ana_step<R, 0, true, true>(A, m, l, cf, S, D, slot);
        } else {
            if (par) ana_step<R, 1, true, false>(A, m, l, cf, S, D, slot);
            else ana_step<R, 0, true, false>(A, m, l, cf, S, D, slot);
        }
    } else {
        if (par) ana_step<R, 1, false, true>(A, m, l, cf, S, D, slot);
        else ana_step<R, 0, false, true>(A, m, l, cf, S, D, slot);
    }
}

// a full round of kAnaL degrees in the steady state (no activation)
template <int R, int P0>
__device__ __forceinline__ void ana_round(const LegArgs& A, int m, int lc, const double* __restrict__ cf,
                                          RecState<R>& S, const AnaData<R>& D, double* tile, int lane) {
#pragma unroll
    for (int j = 0; j < kAnaL; ++j) {
        if ((P0 + j) & 1) ana_step<R, 1, true, false>(A, m, lc + j, cf, S, D, tile + j * 6 * kAnaRow + lane);
        else ana_step<R, 0, true, false>(A, m, lc + j, cf, S, D, tile + j * 6 * kAnaRow + lane);
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int R>
__global__ __launch_bounds__(kAnaThreads) void leg_analysis_kernel(LegArgs A, const double2* __restrict__ phase,
                                                                   const double* __restrict__ pair_w,
                                                                   double* __restrict__ partial) {
    __shared__ double red[(kAnaThreads / 64) * kAnaTile];
    const int m = blockIdx.y;
    const int rhs = blockIdx.z;
    const int nrhs = gridDim.z;
    const int lmax = A.lmax;
    const int lend = A.lend;
    // orders above the band limit: nothing to sum (the combine writes zeros)
    if (m > lend) return;
    const int64_t base = mbase(m, lmax);
    const double* __restrict__ cf = A.coef + base * kCoefSStride;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (kAnaThreads / 64) + (threadIdx.x >> 6);   // partial-sum slot
    double* tile = red + (threadIdx.x >> 6) * kAnaTile;
    const int p0 = wave * 64 * R + lane;

    RecState<R> S;
    AnaData<R> D;
    int lo, hi;
    rec_init<R>(S, A, m, p0, 64, lo, hi);
    const int64_t fstride = (int64_t)A.npairs * (A.mmax + 1) * 2;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int p = p0 + r * 64;
        const bool ok = p < A.npairs;
        double2 g[3][2];
        if (ok) {
            const double2* in = phase + (((int64_t)rhs * 3) * A.npairs + p) * (A.mmax + 1) * 2 + (int64_t)m * 2;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                g[f][0] = in[f * fstride];
                g[f][1] = in[f * fstride + 1];
            }
        } else {
#pragma unroll
            for (int f = 0; f < 3; ++f) g[f][0] = g[f][1] = make_double2(0.0, 0.0);
        }
        const double w = ok ? pair_w[p] : 0.0;
        D.Ts[r][0] = w * (g[0][0].x + g[0][1].x); D.Ts[r][1] = w * (g[0][0].y + g[0][1].y);
        D.Ta[r][0] = w * (g[0][0].x - g[0][1].x); D.Ta[r][1] = w * (g[0][0].y - g[0][1].y);
        D.Pn[r][0] = w * (g[1][0].x - g[2][0].y); D.Pn[r][1] = w * (g[1][0].y + g[2][0].x);
        D.Ps[r][0] = w * (g[1][1].x - g[2][1].y); D.Ps[r][1] = w * (g[1][1].y + g[2][1].x);
        D.Mn[r][0] = w * (g[1][0].x + g[2][0].y); D.Mn[r][1] = w * (g[1][0].y - g[2][0].x);
        D.Ms[r][0] = w * (g[1][1].x + g[2][1].y); D.Ms[r][1] = w * (g[1][1].y - g[2][1].x);
    }
    lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    if (m < 2) hi = max(hi, 2);

    double* out = partial + ((((int64_t)wave * nrhs + rhs) * 3) * A.nalm) * 2;
    // degrees below the wave's first active one get zero partial sums
    const int lz = min(lo, lend + 1);
    for (int q = lane; q < (lz - m) * 6; q += 64) {
        const int l = m + q / 6, k = q % 6;
        out[((int64_t)(k >> 1) * A.nalm + base + l) * 2 + (k & 1)] = 0.0;
    }

    // reduction roles: 2 lanes per (degree, component) row
    const int o = lane >> 1, q = lane & 1;
    for (int lc = lo; lc <= lend; lc += kAnaL) {
        const int ln = min(kAnaL, lend + 1 - lc);
        if (ln == kAnaL && lc > hi) {
            if ((lc + m) & 1) ana_round<R, 1>(A, m, lc, cf, S, D, tile, lane);
            else ana_round<R, 0>(A, m, lc, cf, S, D, tile, lane);
        } else {
            for (int j = 0; j < ln; ++j)
                ana_step_any<R>(A, m, lc + j, lo, hi, cf, S, D, tile + j * 6 * kAnaRow + lane);
        }
        wave_sync();
        const int nout = ln * 6;
        double s = 0.0;
        if (o < nout) {
            const double* row = tile + o * kAnaRow + q * 32;
#pragma unroll 8
            for (int i = 0; i < 32; ++i) s += row[i];
        }
        s += __shfl_xor(s, 1, 64);
        if (o < nout && q == 0) {
            const int ll = lc + o / 6, k = o % 6;
            out[((int64_t)(k >> 1) * A.nalm + base + ll) * 2 + (k & 1)] = s;
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// combine chunk partials, convert the spin-2 pair to E/B, apply the
// messenger filter (eq 8); optionally also write the filtered result in the
// spin basis (T, (2)a, (-2)a) that the synthesis consumes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void eb_to_spin(double2 e, double2 b, double2& p2, double2& m2) {
    // (+-2)a = -(E +- i B)
    p2 = make_double2(-(e.x - b.y), -(e.y + b.x));
    m2 = make_double2(-(e.x + b.y), -(e.y - b.x));
}

// the spin-basis copy (T, (2)a, (-2)a), each times its recursion scale
// (1 for the vector kernels)
__device__ __forceinline__ void spin_scale(double s0, double s2, double2 t, double2 p2, double2 m2,
                                           double2* __restrict__ q, int64_t nalm) {
    q[0] = make_double2(s0 * t.x, s0 * t.y);
    q[nalm] = make_double2(s2 * p2.x, s2 * p2.y);
    q[2 * nalm] = make_double2(s2 * m2.x, s2 * m2.y);
}

// fixed-order sum of (a, b) over the 256 threads of a combine block into
// cpart[rhs][block][2]; every thread of the block must call it once
__device__ void cauchy_block_sum(double a, double b, double* __restrict__ cpart, int nrhs) {
    __shared__ double sa[256], sb[256];
    const int t = threadIdx.x;
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            sa[t] += sa[t + h];
            sb[t] += sb[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        const int64_t nblk = (int64_t)gridDim.x * gridDim.y;
        double* o = cpart + ((int64_t)blockIdx.z * nblk + (int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        o[0] = sa[0];
        o[1] = sb[0];
    }
}

// per RHS: fixed-order sum of the combine blocks' Cauchy terms -> out[rhs][2]
__global__ __launch_bounds__(256) void cauchy_reduce_kernel(const double* __restrict__ cpart, int64_t nblk,
                                                            double* __restrict__ out) {
    __shared__ double sa[256], sb[256];
    const int t = threadIdx.x, rhs = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t i = t; i < nblk; i += 256) {
        a += cpart[((int64_t)rhs * nblk + i) * 2];
        b += cpart[((int64_t)rhs * nblk + i) * 2 + 1];
    }
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            sa[t] += sa[t + h];
            sb[t] += sb[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[rhs * 2] = sa[0];
        out[rhs * 2 + 1] = sb[0];
    }
}

// cpart (nullable): per-block sums of w |u_new - u_old|^2 and w |u_new|^2
// over T, E, B (w = 2 for m > 0), the Cauchy ratio's terms; the old value
// is what alm holds on entry.  scale (nullable, [nalm][2]): the batched
// kernels' recursion scales S (spin 0, spin 2); the partial sums are
// multiplied by S, and so is the spin-basis copy (the batched synthesis
// contracts the scaled functions with it).
template <typename PV>
__global__ __launch_bounds__(256) void combine_kernel(int lmax, int lend, int64_t nalm, int nchunks, int nrhs,
                                                      const PV* __restrict__ partial,
                                                      const int* __restrict__ slot_lo,
                                                      const double* __restrict__ filt, double2* __restrict__ alm,
                                                      double2* __restrict__ spin, double* __restrict__ cpart,
                                                      const double* __restrict__ scale) {
    const int m = blockIdx.y;
    const int rhs = blockIdx.z;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    double dd = 0.0, nn = 0.0;                         // Cauchy terms of this thread
    if (l <= lmax) {
        const int64_t idx = mbase(m, lmax) + l;
        double2 a[3];
        // above the band limit the analysis wrote nothing: the coefficient is 0
        const int nc = (l <= lend && m <= lend) ? nchunks : 0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            double2 s = make_double2(0.0, 0.0);
            for (int c = 0; c < nc; ++c) {
                // a slot holds degrees from its first start degree on
                if (slot_lo && l < slot_lo[(int64_t)m * nchunks + c]) continue;
                const PV v = partial[(((int64_t)c * nrhs + rhs) * 3 + f) * nalm + idx];
                s.x += (double)v.x;
                s.y += (double)v.y;
            }
            a[f] = s;
        }
        double s0 = 1.0, s2 = 1.0;
        if (scale) {
            s0 = scale[2 * idx];
            s2 = scale[2 * idx + 1];
            a[0] = make_double2(s0 * a[0].x, s0 * a[0].y);
            a[1] = make_double2(s2 * a[1].x, s2 * a[1].y);
            a[2] = make_double2(s2 * a[2].x, s2 * a[2].y);
        }
        // E = -((2)a + (-2)a)/2,  B = i((2)a - (-2)a)/2
        double2 E = make_double2(-0.5 * (a[1].x + a[2].x), -0.5 * (a[1].y + a[2].y));
        double2 B = make_double2(-0.5 * (a[1].y - a[2].y), 0.5 * (a[1].x - a[2].x));
        if (l < 2) E = B = make_double2(0.0, 0.0);
        double2 T = a[0];
        if (filt) {
            const double ftt = filt[4 * l], fte = filt[4 * l + 1], fee = filt[4 * l + 2], fbb = filt[4 * l + 3];
            const double2 t2 = make_double2(ftt * T.x + fte * E.x, ftt * T.y + fte * E.y);
            const double2 e2 = make_double2(fte * T.x + fee * E.x, fte * T.y + fee * E.y);
            B = make_double2(fbb * B.x, fbb * B.y);
            T = t2;
            E = e2;
        }
        // alm may be null (a fixed-schedule iteration whose iterate only the
        // next synthesis reads, through the spin-basis copy)
        if (alm) {
            double2* o = alm + ((int64_t)rhs * 3) * nalm + idx;
            if (cpart) {
                const double w = m > 0 ? 2.0 : 1.0;
                const double2 n3[3] = {T, E, B};
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const double2 old = o[f * nalm];
                    const double dx = n3[f].x - old.x, dy = n3[f].y - old.y;
                    dd += w * (dx * dx + dy * dy);
                    nn += w * (n3[f].x * n3[f].x + n3[f].y * n3[f].y);
                }
            }
            o[0] = T;
            o[nalm] = E;
            o[2 * nalm] = B;
        }
        if (spin) {
            double2* q = spin + ((int64_t)rhs * 3) * nalm + idx;
            double2 p2, m2;
            eb_to_spin(E, B, p2, m2);
            spin_scale(s0, s2, T, p2, m2, q, nalm);
        }
    }
    // cpart is uniform over the grid, so the whole block takes this branch
    if (cpart) cauchy_block_sum(dd, nn, cpart, nrhs);
}

// (T, E, B) -> (T, (2)a, (-2)a), times the recursion scales if scale is
// given (the same arithmetic as the combine kernel's spin-basis copy)
__global__ void to_spin_kernel(int64_t nalm, int64_t total, const double2* __restrict__ alm,
                               double2* __restrict__ spin, const double* __restrict__ scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rhs = i / nalm, idx = i % nalm;
        const double2* a = alm + rhs * 3 * nalm + idx;
        double2* q = spin + rhs * 3 * nalm + idx;
        double2 p2, m2;
        eb_to_spin(a[nalm], a[2 * nalm], p2, m2);
        const double s0 = scale ? scale[2 * idx] : 1.0, s2 = scale ? scale[2 * idx + 1] : 1.0;
        spin_scale(s0, s2, a[0], p2, m2, q, nalm);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_seeds(dm_plan* p, hipStream_t s) {
    dim3 grid((p->npairs + 127) / 128, p->mmax + 1);
    hipLaunchKernelGGL(seed_kernel, grid, dim3(128), 0, s, p->lmax, p->npairs, p->d_pair_x, p->d_coef,
                       p->d_lp0, p->d_lp2, p->d_lstart, p->d_seed, (int64_t)(p->mmax + 1) * p->npairs);
    return hipGetLastError();
}

hipError_t launch_leg_synthesis(dm_plan* p, int nrhs, const double* alm, double* phase, hipStream_t s) {
    LegArgs A = leg_args(p);
    const int nt = p->syn_threads, R = p->syn_R;
    dim3 grid((p->npairs + nt * R - 1) / (nt * R), p->mmax + 1, nrhs);
    const double2* a = reinterpret_cast<const double2*>(alm);
    double2* ph = reinterpret_cast<double2*>(phase);
    if (R == 1) hipLaunchKernelGGL(leg_synth_kernel<1>, grid, dim3(nt), 0, s, A, a, ph);
    else if (R == 2) hipLaunchKernelGGL(leg_synth_kernel<2>, grid, dim3(nt), 0, s, A, a, ph);
    else hipLaunchKernelGGL(leg_synth_kernel<4>, grid, dim3(nt), 0, s, A, a, ph);
    return hipGetLastError();
}

hipError_t launch_leg_analysis(dm_plan* p, int nrhs, const double* phase, const double* pair_w, double* partial,
                               hipStream_t s) {
    LegArgs A = leg_args(p);
    const int R = p->ana_R;
    dim3 grid(p->ana_blocks, p->mmax + 1, nrhs);
    const double2* ph = reinterpret_cast<const double2*>(phase);
    if (R == 1) hipLaunchKernelGGL(leg_analysis_kernel<1>, grid, dim3(kAnaThreads), 0, s, A, ph, pair_w, partial);
    else if (R == 2) hipLaunchKernelGGL(leg_analysis_kernel<2>, grid, dim3(kAnaThreads), 0, s, A, ph, pair_w, partial);
    else hipLaunchKernelGGL(leg_analysis_kernel<4>, grid, dim3(kAnaThreads), 0, s, A, ph, pair_w, partial);
    return hipGetLastError();
}

// analysis tiling: R ring pairs per lane, 4 waves per workgroup; one
// partial-sum slot per wave
void set_analysis_tiling(dm_plan* p, int R) {
    p->ana_R = R;
    const int per_wave = 64 * R;
    const int waves = (p->npairs + per_wave - 1) / per_wave;
    p->ana_blocks = (waves + kAnaThreads / 64 - 1) / (kAnaThreads / 64);
    p->ana_chunks = p->ana_blocks * (kAnaThreads / 64);
}

hipError_t launch_combine(dm_plan* p, int nrhs, int nslots, const double* partial, bool partial32,
                          const int* slot_lo, const double* filter, double* alm, double* spin, double* cpart,
                          const double* scale, hipStream_t s) {
    dim3 grid((p->lmax + 1 + 255) / 256, p->mmax + 1, nrhs);
    const int lend = (p->lcut > 0 && p->lcut < p->lmax) ? p->lcut : p->lmax;
    if (partial32)
        hipLaunchKernelGGL(combine_kernel<float2>, grid, dim3(256), 0, s, p->lmax, lend, p->nalm, nslots, nrhs,
                           reinterpret_cast<const float2*>(partial), slot_lo, filter, reinterpret_cast<double2*>(alm),
                           reinterpret_cast<double2*>(spin), cpart, scale);
    else
        hipLaunchKernelGGL(combine_kernel<double2>, grid, dim3(256), 0, s, p->lmax, lend, p->nalm, nslots, nrhs,
                           reinterpret_cast<const double2*>(partial), slot_lo, filter, reinterpret_cast<double2*>(alm),
                           reinterpret_cast<double2*>(spin), cpart, scale);
    return hipGetLastError();
}

int64_t cauchy_blocks(dm_plan* p) { return (int64_t)((p->lmax + 1 + 255) / 256) * (p->mmax + 1); }

hipError_t launch_cauchy_reduce(dm_plan* p, int nrhs, const double* cpart, double* out, hipStream_t s) {
    hipLaunchKernelGGL(cauchy_reduce_kernel, dim3(nrhs), dim3(256), 0, s, cpart, cauchy_blocks(p), out);
    return hipGetLastError();
}

hipError_t launch_to_spin(dm_plan* p, int nrhs, const double* alm, double* spin, const double* scale,
                          hipStream_t s) {
    const int64_t total = (int64_t)nrhs * p->nalm;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(to_spin_kernel, dim3((int)g), dim3(256), 0, s, p->nalm, total,
                       reinterpret_cast<const double2*>(alm), reinterpret_cast<double2*>(spin), scale);
    return hipGetLastError();
}


}  // namespace dmwf
