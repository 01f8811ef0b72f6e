// Batched Legendre step on the matrix cores: for B right-hand sides the
// contractions of the spherical harmonic transform become dense products
// (the batching of constrained realizations, Sec. 2.2, eq 19):
//
//   synthesis  Out[(pair, side), (rhs, re/im)] += sum_l A_f[(pair, side), l] D_f[l, (rhs, re/im)]
//   analysis   Out[l, (rhs, re/im)]            += sum_(pair, side) A_f[(pair, side), l] G_f[(pair, side), (rhs, re/im)]
//
// with three products f = T, +2, -2 and rows (pair, side) = the north ring
// and its mirror:  A_T = (lam, eps lam),  A_+2 = (p, eps q),
// A_-2 = (q, eps p),  eps = (-1)^(l+m),  p = (+2)lam, q = (-2)lam.
// D_f are the spin-basis coefficients (a^T, (2)a, (-2)a); G_f are the
// weighted ring Fourier data (G^T, G^Q + i G^U, G^Q - i G^U).
//
// One lane runs the FP64 recursions of one ring pair (seeds and start
// degrees as in the single-RHS kernels); the values of a few consecutive
// degrees go through a double-buffered, wave-private LDS tile into the
// operand layout of v_mfma_*_16x16x4 (A: lane = row + 16 k, B: lane =
// col + 16 k).  T = double uses the FP64 matrix instruction; T = float
// converts the functions and data to FP32 and accumulates in FP32 (the
// mixed-precision path; the iterate itself stays FP64).
#include <type_traits>

#include "dmwf_internal.h"

namespace dmwf {

namespace {

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output element v of a lane sits at row (lane / 16) + 4 v
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // output element v of a lane sits at row 4 (lane / 16) + v
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// complex values of the ring Fourier data, stored in the kernel's own
// precision (FP32 ring data for the mixed plans: the products round it to
// FP32 anyway)
template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    typedef float2 t;
};
template <>
struct Vec2<double> {
    typedef double2 t;
};

template <typename T>
__device__ __forceinline__ typename Vec2<T>::t vec2(double x, double y) {
    typename Vec2<T>::t v;
    v.x = (T)x;
    v.y = (T)y;
    return v;
}

__device__ __forceinline__ int64_t mbase(int m, int lmax) { return (int64_t)m * (2 * lmax + 1 - m) / 2; }

__device__ __forceinline__ int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Workgroup placement.  Workgroups go to the 8 XCDs (each with its own L2)
// in turn by linear index, so a plain (pair block, m) grid spreads the
// blocks of one m, which share their harmonic coefficients, recursion
// coefficients and 128-byte lines of the ring data of neighbouring m, over
// all XCDs.  The 1-D grid is decoded instead so that XCD c receives, in
// order, chunks of kMChunk consecutive m with all their pair blocks:
// m = R (8 j + c) + r, R = mchunk.  Indices past mmax return at once.
// mchunk = 0 keeps the plain order (pair block fastest, then m).
constexpr int kXcd = 8;

struct BlockPos {
    int x, m;
};

__device__ __forceinline__ BlockPos block_pos(int nx, int R) {
    const int id = blockIdx.x;
    if (R == 0) return BlockPos{id % nx, id / nx};
    const int c = id % kXcd, k = id / kXcd;
    const int j = k / (R * nx), r = (k / nx) % R, x = k % nx;
    return BlockPos{x, R * (kXcd * j + c) + r};
}

inline unsigned grid_blocks(int nx, int mmax, int R) {
    if (R == 0) return (unsigned)(nx * (mmax + 1));
    const int chunks = (mmax + 1 + kXcd * R - 1) / (kXcd * R);
    return (unsigned)(chunks * kXcd * R * nx);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct BatchArgs {
    int lmax, mmax, npairs, nrhs;
    int lend;                       // band limit of this launch: degrees and orders above it are skipped
    int nx;                         // ring-pair blocks per m
    int mchunk;                     // consecutive m per XCD chunk (0: plain order)
    int64_t nalm;
    const double* __restrict__ pair_x;
    const double* __restrict__ coef;    // scaled recursions, [nalm][kCoefSStride]
    const double* __restrict__ scale;   // their scales S, [nalm][2]
    const int* __restrict__ lstart;
    const double* __restrict__ seed;
    int64_t sstride;
};

// FP64 recursion of one ring pair: lam, p, q at (l-1, l), and the pair's
// seeds, loaded once at the start so that taking them needs no memory wait
// (a load at activation time waits, through the in-order vector memory
// counter, for every load issued before it: 2 % of both kernels' time)
struct Rec {
    double x, l0, l1, w0, w1, q0, q1;
    double sd[6];
    int ls, pr;
};

// coefficients of one degree of the scaled recursions: spin 0 (A0'), spin 2
// (alpha', (alpha beta)'); the degree l-2 term has coefficient 1.  The
// functions carried are mu = lam / S (S per (l, m), spin 0 and spin 2): the
// contraction inputs and outputs are multiplied by S outside these kernels.
struct Coef {
    double a, al, ab;
};

__device__ __forceinline__ Coef coef_at(const double* __restrict__ c) { return Coef{c[0], c[1], c[2]}; }

__device__ __forceinline__ void rec_advance(const Coef& c, Rec& s) {
    const double ax = c.a * s.x;
    const double cw = c.al * s.x + c.ab, cq = c.al * s.x - c.ab;
    const double nl = ax * s.l1 - s.l0;
    const double nw = cw * s.w1 - s.w0;
    const double nq = cq * s.q1 - s.q0;
    s.l0 = s.l1; s.l1 = nl;
    s.w0 = s.w1; s.w1 = nw;
    s.q0 = s.q1; s.q1 = nq;
}

__device__ __forceinline__ void rec_advance(const double* __restrict__ c, Rec& s) { rec_advance(coef_at(c), s); }

// The recursion coefficients reach the steady loops through LDS rather than
// scalar loads: scalar and LDS loads share one wait counter and scalar loads
// return out of order, so every wait for an LDS operand would also wait for
// the coefficient loads.  A group of G degrees (3 coefficients each) is
// loaded one round ahead by lane t < 5G (one double each, vector loads),
// stored to LDS in the following round and read as broadcasts in the round
// after.  Every lane loads and stores (lanes >= 5G repeat the last value
// into their own slot), so the loop body has no branch and the wait for the
// load stays precise; degrees past lmax are clamped to lmax (a group past
// lmax is loaded but never used).
constexpr int kCoefN = 3;

__device__ __forceinline__ double coef_fetch(const double* __restrict__ cf, int l0, int lmax, int t, int G) {
    const int tc = min(t, G * kCoefN - 1);
    const int d = tc / kCoefN, i = tc - d * kCoefN;
    // a uniform base (cf points at the order's first degree) and a 32-bit
    // byte offset per lane
    const unsigned off = (unsigned)((min(l0 + d, lmax) * kCoefSStride + i) * 8);
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(cf) + off);
}

__device__ __forceinline__ Coef coef_lds(const double* c) { return Coef{c[0], c[1], c[2]}; }

__device__ __forceinline__ void rec_activate(const BatchArgs& A, int m, int l, Rec& s) {
    if (l == s.ls) {
        s.l0 = s.sd[0];
        s.l1 = s.sd[1];
        if (m >= 2) {
            s.w0 = s.sd[2];
            s.w1 = s.sd[3];
            s.q0 = s.sd[4];
            s.q1 = s.sd[5];
        }
    }
    if (m < 2 && l == 2 && s.ls <= A.lmax) {
        s.w0 = s.sd[2];
        s.w1 = s.sd[3];
        s.q0 = s.sd[4];
        s.q1 = s.sd[5];
    }
}

// call before the kernel's other global loads: the seeds then arrive first,
// and waiting for them does not wait for the loads issued after them.  The
// seeds (lam at the degrees before and at the start) become mu = lam / S.
__device__ __forceinline__ void rec_init(Rec& s, const BatchArgs& A, int m, int p) {
    const bool ok = p < A.npairs;
    s.pr = ok ? p : 0;
    s.x = ok ? A.pair_x[p] : 0.0;
    s.ls = ok ? A.lstart[(int64_t)m * A.npairs + p] : A.lmax + 1;
    s.l0 = s.l1 = s.w0 = s.w1 = s.q0 = s.q1 = 0.0;
    const int64_t o = (int64_t)m * A.npairs + s.pr;
#pragma unroll
    for (int i = 0; i < 6; ++i) s.sd[i] = A.seed[i * A.sstride + o];
    // degrees of the seeds, clamped into [m, lmax] (a seed below m is 0; an
    // inactive lane's seeds are never taken)
    const double* sc = A.scale + mbase(m, A.lmax) * 2;
    auto at = [&](int l) { return (int64_t)min(max(l, m), A.lmax) * 2; };
    const int l2 = m < 2 ? 2 : s.ls;             // spin 2 of m < 2 starts at l = 2
    s.sd[0] /= sc[at(s.ls - 1)];
    s.sd[1] /= sc[at(s.ls)];
    const double s2a = sc[at(l2 - 1) + 1], s2b = sc[at(l2) + 1];
    s.sd[2] /= s2a;
    s.sd[3] /= s2b;
    s.sd[4] /= s2a;
    s.sd[5] /= s2b;
}

// one recursion step to degree l (zero beyond the launch's band limit)
__device__ __forceinline__ void rec_step(const BatchArgs& A, const double* __restrict__ cf, int m, int l, int lo,
                                         int hi, Rec& s, double& lam, double& pp, double& qq) {
    if (l <= A.lend) {
        if (l > lo) rec_advance(cf + (int64_t)l * kCoefSStride, s);
        if (l <= hi) rec_activate(A, m, l, s);
        lam = s.l1;
        pp = s.w1;
        qq = s.q1;
    } else {
        lam = pp = qq = 0.0;
    }
}

// recursion values of the next degree for the steady state (every lane
// past its start degree, degree <= lmax): no branch, so the compiler can
// interleave it with the matrix instructions of the current round
__device__ __forceinline__ void rec_next(const double* __restrict__ cf, int l, Rec& s) {
    rec_advance(cf + (int64_t)l * kCoefSStride, s);
}

// ---------------------------------------------------------------------------
// synthesis: W waves x PW ring pairs per block (PW = 64 FP32, 32 FP64; W =
// 1, 2, 4 or 8, picked by the autotuner, 4 by default),
// rounds of 4 degrees (one K step), one column tile of 8 RHS per block.
// The rows of one matrix instruction are 16 ring pairs of one side: the
// north rows take (lam, +2lam, -2lam) times D_f, the mirror rows
// (lam, -2lam, +2lam) times eps_l D_f, with the sign on the B operand (per
// lane, fixed for the kernel since rounds advance by 4 degrees).
// ---------------------------------------------------------------------------

// [f = lam, +2, -2][degree in round][pair]; FP32 operand reads of one
// instruction (16 pairs x 4 degrees, 32 lanes at a time) are conflict-free
// with rows 16 words apart modulo 32; FP64 reads go 16 lanes (one degree)
// at a time and need no padding
template <typename T, int PW>
struct SynTile {
    static constexpr int K = sizeof(T) == 4 ? PW + 16 : PW;
    static constexpr int F = 4 * K;
    T v[3 * F];
    __device__ T& at(int f, int j, int pair) { return v[f * F + j * K + pair]; }
    __device__ const T& at(int f, int j, int pair) const { return v[f * F + j * K + pair]; }
};

// per-wave LDS: two tiles, reused by the epilogue as staging for one row
// tile of outputs, [f][16 pairs][8 RHS][side][re/im]
template <typename T, int PW>
constexpr int syn_wave_bytes() {
    return 2 * (int)sizeof(SynTile<T, PW>) > 1536 * (int)sizeof(T) ? 2 * (int)sizeof(SynTile<T, PW>)
                                                                    : 1536 * (int)sizeof(T);
}

template <typename T, int PW>
__device__ __forceinline__ void syn_store(SynTile<T, PW>& tl, int j, int pair, double lam, double pp, double qq) {
    tl.at(0, j, pair) = (T)lam;
    tl.at(1, j, pair) = (T)pp;
    tl.at(2, j, pair) = (T)qq;
}

template <typename T, int PW>
__device__ __forceinline__ void bsyn_mfma(const SynTile<T, PW>& tl, int k, int row, const T (&b)[3], const T (&bs)[3],
                                          typename Mfma<T>::v4 (&acc)[PW / 16][2][3]) {
#pragma unroll
    for (int t = 0; t < PW / 16; ++t) {
        const int pi = t * 16 + row;
        const T l = tl.at(0, k, pi), pp = tl.at(1, k, pi), qq = tl.at(2, k, pi);
        acc[t][0][0] = Mfma<T>::run(l, b[0], acc[t][0][0]);
        acc[t][0][1] = Mfma<T>::run(pp, b[1], acc[t][0][1]);
        acc[t][0][2] = Mfma<T>::run(qq, b[2], acc[t][0][2]);
        acc[t][1][0] = Mfma<T>::run(l, bs[0], acc[t][1][0]);
        acc[t][1][1] = Mfma<T>::run(qq, bs[1], acc[t][1][1]);
        acc[t][1][2] = Mfma<T>::run(pp, bs[2], acc[t][1][2]);
    }
}

// OffT: the lanes' byte offsets from uniform bases (unsigned where they
// stay below 2^32, see offsets_fit; 64-bit otherwise)
template <typename T, int PW, int kSynWaves, typename OffT>
__global__ __launch_bounds__(64 * kSynWaves) void bsyn_kernel(BatchArgs A, const double2* __restrict__ spin,
                                                              T* __restrict__ phase) {
    typedef typename Mfma<T>::v4 v4;
    constexpr int NT = PW / 16;                       // row tiles per side
    constexpr int WB = syn_wave_bytes<T, PW>();
    __shared__ __align__(16) unsigned char lds[kSynWaves][WB];
    __shared__ double cofw[kSynWaves][2][64];
    const BlockPos bp = block_pos(A.nx, A.mchunk);
    const int m = bp.m;
    if (m > A.mmax) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int pbase = (bp.x * kSynWaves + wv) * PW;
    const int rb = blockIdx.y * 8;
    const int lmax = A.lmax;
    const int lend = A.lend;          // degrees above it contribute nothing (zero coefficients)
    const int64_t base = mbase(m, lmax);
    const double* __restrict__ cf = A.coef + base * kCoefSStride;
    SynTile<T, PW>* tile = reinterpret_cast<SynTile<T, PW>*>(&lds[wv][0]);
    // the ring pair this lane recurses; with PW < 64 the upper lanes repeat
    // the lower ones and store the same values to the same addresses
    const int me = lane % PW;

    Rec s;
    rec_init(s, A, m, pbase + me);
    int lo = __builtin_amdgcn_readfirstlane(wave_min(s.ls));
    int hi = __builtin_amdgcn_readfirstlane(wave_max(s.ls <= lmax ? s.ls : 0));
    if (m < 2) hi = max(hi, 2);

    v4 acc[NT][2][3];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int f = 0; f < 3; ++f) acc[t][sd][f] = v4{0, 0, 0, 0};

    const int row = lane & 15, k = lane >> 4;
    const int col = lane & 15, ri = col & 1;
    const int rhs = rb + (col >> 1);
    const bool rhs_ok = rhs < A.nrhs;
    // eps of this lane's degree l0 + k (rounds start at lo + 4n)
    const T eps = ((lo + k + m) & 1) ? (T)-1 : (T)1;
    // padding columns read RHS 0 and are never stored
    const double* __restrict__ sbase = reinterpret_cast<const double*>(spin) +
                                       (((int64_t)(rhs_ok ? rhs : 0) * 3) * A.nalm + base) * 2 + ri;
    auto load_b = [&](int l, double (&b)[3]) {
        const int lc = min(l, lend);              // beyond lend the A operand is zero
        b[0] = sbase[(int64_t)lc * 2];
        b[1] = sbase[(A.nalm + lc) * 2];
        b[2] = sbase[(2 * A.nalm + lc) * 2];
    };
    auto produce_any = [&](int l0, int q) {
        for (int j = 0; j < 4; ++j) {
            double lam, pp, qq;
            rec_step(A, cf, m, l0 + j, lo, hi, s, lam, pp, qq);
            syn_store<T, PW>(tile[q], j, me, lam, pp, qq);
        }
    };
    auto operands = [&](const double (&braw)[3], T (&b)[3], T (&bs)[3]) {
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            b[f] = (T)braw[f];
            bs[f] = eps * b[f];
        }
    };

    if (lo <= lend) {
        produce_any(lo, 0);
        double braw[3];
        load_b(lo + k, braw);
        wave_sync();
        int q = 0, l0 = lo;
        // rounds whose successor still needs activation or runs past lmax
        for (; l0 <= lend; l0 += 4, q ^= 1) {
            const int ln = l0 + 4;
            if (ln > hi && ln + 3 <= lend) break;
            T b[3], bs[3];
            operands(braw, b, bs);
            load_b(ln + k, braw);
            bsyn_mfma<T, PW>(tile[q], k, row, b, bs, acc);
            if (ln <= lend) produce_any(ln, q ^ 1);
            wave_sync();
        }
        // steady state: matrix products of this round, recursion of the next
        if (l0 + 7 <= lend) {
            // coefficients of the first steady recursion (degrees l0 + 4 ..
            // l0 + 7) to LDS slot q (the slot index follows the tile index),
            // the next group in flight
            cofw[wv][q][lane] = coef_fetch(cf, l0 + 4, lmax, lane, 4);
            double creg = coef_fetch(cf, l0 + 8, lmax, lane, 4);
            // B operands of the next round (degree l0 + 4 + k <= lend: no
            // clamp): three uniform field bases at this column tile's first
            // RHS and one byte offset per lane (at most 7 RHS x 3 fields + 1
            // of nalm complex past the base), advanced by 4 degrees per round
            const char* __restrict__ sb0 = reinterpret_cast<const char*>(spin + (int64_t)rb * 3 * A.nalm);
            const int64_t fbytes = A.nalm * 16;
            OffT boff = (OffT)(((((int64_t)(rhs_ok ? rhs - rb : 0) * 3) * A.nalm + base + l0 + 4 + k) * 2 + ri) * 8);
            wave_sync();
            // one round with tile Q (products) and Q ^ 1 (the next degrees);
            // two rounds per loop trip, so that the tile and slot addresses
            // are fixed
            auto steady = [&](auto qc) {
                constexpr int Q = decltype(qc)::value;
                T b[3], bs[3];
                operands(braw, b, bs);
                // the in-flight group (degrees l0 + 8 ..) to the other slot,
                // then the group after it, then the next B operands
                cofw[wv][Q ^ 1][lane] = creg;
                creg = coef_fetch(cf, l0 + 12, lmax, lane, 4);
                braw[0] = *reinterpret_cast<const double*>(sb0 + boff);
                braw[1] = *reinterpret_cast<const double*>(sb0 + fbytes + boff);
                braw[2] = *reinterpret_cast<const double*>(sb0 + 2 * fbytes + boff);
                bsyn_mfma<T, PW>(tile[Q], k, row, b, bs, acc);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    rec_advance(coef_lds(&cofw[wv][Q][j * kCoefN]), s);
                    syn_store<T, PW>(tile[Q ^ 1], j, me, s.l1, s.w1, s.q1);
                }
                wave_sync();
                l0 += 4;
                boff += 64;
            };
            if (q == 1) {
                steady(std::integral_constant<int, 1>());
                q = 0;
            }
            for (; l0 + 11 <= lend;) {
                steady(std::integral_constant<int, 0>());
                steady(std::integral_constant<int, 1>());
            }
            if (l0 + 7 <= lend) {
                steady(std::integral_constant<int, 0>());
                q = 1;
            }
        }
        // tail
        for (; l0 <= lend; l0 += 4, q ^= 1) {
            const int ln = l0 + 4;
            T b[3], bs[3];
            operands(braw, b, bs);
            load_b(ln + k, braw);
            bsyn_mfma<T, PW>(tile[q], k, row, b, bs, acc);
            if (ln <= lend) produce_any(ln, q ^ 1);
            wave_sync();
        }
    }

    // epilogue, through the wave's (now free) LDS: per row tile (16 ring
    // pairs) the raw products go to LDS as [f][pair][rhs][side][re/im]; then
    // each lane takes two (pair, rhs), forms T, Q = (P + M)/2,
    // U = (P - M)/(2i) and writes 32 contiguous bytes (both sides, re/im)
    // per field
    T* stg = reinterpret_cast<T*>(&lds[wv][0]);
    const int64_t fstride = (int64_t)A.npairs * (A.mmax + 1) * 4;     // values per field
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        wave_sync();
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = Mfma<T>::row(lane, v);
                    stg[(((f * 16 + r) * 8 + (col >> 1)) * 2 + sd) * 2 + ri] = acc[t][sd][f][v];
                }
        wave_sync();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int u = lane + 64 * h;
            const int r = u >> 3, rc = u & 7;
            const int pair = pbase + t * 16 + r, rw = rb + rc;
            if (pair < A.npairs && rw < A.nrhs) {
                const T* g = stg + (r * 8 + rc) * 4;
                const T* gp = g + 16 * 8 * 4;
                const T* gm = g + 2 * 16 * 8 * 4;
                double qv[4], uv[4];
#pragma unroll
                for (int sd = 0; sd < 2; ++sd) {
                    const double pr = gp[2 * sd], pi = gp[2 * sd + 1], mr = gm[2 * sd], mi = gm[2 * sd + 1];
                    qv[2 * sd] = 0.5 * (pr + mr);
                    qv[2 * sd + 1] = 0.5 * (pi + mi);
                    uv[2 * sd] = 0.5 * (pi - mi);
                    uv[2 * sd + 1] = -0.5 * (pr - mr);
                }
                typedef typename Vec2<T>::t T2;
                T* ob = phase + ((((int64_t)rw * 3) * A.npairs + pair) * (A.mmax + 1) + m) * 4;
                T2* o = reinterpret_cast<T2*>(ob);
                o[0] = vec2<T>(g[0], g[1]);
                o[1] = vec2<T>(g[2], g[3]);
                T2* oq = reinterpret_cast<T2*>(ob + fstride);
                oq[0] = vec2<T>(qv[0], qv[1]);
                oq[1] = vec2<T>(qv[2], qv[3]);
                T2* ou = reinterpret_cast<T2*>(ob + 2 * fstride);
                ou[0] = vec2<T>(uv[0], uv[1]);
                ou[1] = vec2<T>(uv[2], uv[3]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// analysis: W waves x 64 ring pairs per block (one pair per lane), rounds of
// 16 degrees, one column tile of 8 RHS per block.  The K dimension is split
// by side: the north rings give C_N = sum A_N G_N, the mirror rings
// C_S = sum A_S G_S with A_S = (lam, q, p) unsigned, and a round's output
// row l is C_N + eps_l C_S.  Each wave's tile holds one round: the matrix
// products read it, then the recursion overwrites it with the next round.
// The waves' outputs are summed in LDS one round late, and one
// partial-sum slot per block goes to the combine kernel.
// ---------------------------------------------------------------------------
constexpr int kAnaPW = 64;                              // ring pairs per wave
constexpr int kAnaKH = kAnaPW / 4;                      // K steps per side
constexpr int kAnaKS = 2 * kAnaKH;                      // K steps per round
// tile row length: the operand reads of one matrix instruction (16 degrees
// x 4 pairs) are conflict-free with rows 2 words apart modulo 32 (FP32,
// 32 lanes at a time) or 1 double apart modulo 16 (FP64, 16 lanes at a time)
template <typename T>
constexpr int ana_rl() { return sizeof(T) == 4 ? kAnaPW + 2 : kAnaPW + 1; }
template <typename T>
constexpr int ana_tile() { return 3 * 16 * ana_rl<T>(); }       // [f][degree][pair]
constexpr int kRedCol = 17;                             // [f][col][row] with padded columns
constexpr int kRedF = 16 * kRedCol;

// recursion of an activation round: every lane advances (lanes before
// their start degree hold zeros), lanes whose start degree is l take seeds
__device__ __forceinline__ void rec_act(const BatchArgs& A, const double* __restrict__ cf, int m, int l, Rec& s) {
    rec_advance(cf + (int64_t)l * kCoefSStride, s);
    rec_activate(A, m, l, s);
}

// PT: the partial-sum slots' type (FP32 on the mixed path, where the
// products are FP32 already; the combine kernel sums the slots in FP64)
template <typename T, int W, typename PT, typename OffT>
__global__ __launch_bounds__(64 * W, sizeof(T) == 4 ? 2 : 1) void bana_kernel(BatchArgs A, const typename Vec2<T>::t* __restrict__ phase,
                                                      const double* __restrict__ pair_w,
                                                      PT* __restrict__ partial) {
    typedef typename Mfma<T>::v4 v4;
    constexpr int RL = ana_rl<T>();
    __shared__ T tile[W][ana_tile<T>()];
    __shared__ T red[2][W][3 * kRedF];
    __shared__ double cofb[2][64];                      // recursion coefficients of 16 degrees
    __shared__ int s_lo[W], s_hi[W];
    const BlockPos bp = block_pos(A.nx, A.mchunk);
    const int m = bp.m;
    // orders above the band limit: nothing to sum (the combine writes zeros)
    if (m > A.mmax || m > A.lend) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int pbase = (bp.x * W + wv) * kAnaPW;
    const int rb = blockIdx.y * 8;
    const int lmax = A.lmax;
    const int lend = A.lend;
    const int64_t base = mbase(m, lmax);
    const double* __restrict__ cf = A.coef + base * kCoefSStride;
    const int64_t fstride = (int64_t)A.npairs * (A.mmax + 1) * 2;

    Rec s;
    rec_init(s, A, m, pbase + lane);
    int lo = wave_min(s.ls);
    int hi = wave_max(s.ls <= lmax ? s.ls : 0);
    if (lane == 0) { s_lo[wv] = lo; s_hi[wv] = hi; }
    // the wave's own last start degree: past it, its rounds need no
    // activation even while other waves of the block still start
    int hi_w = __builtin_amdgcn_readfirstlane(hi);
    if (m < 2) hi_w = max(hi_w, 2);

    // B operands: K step st < KH takes the north ring of pair 4 st + k,
    // st >= KH the mirror ring of pair 4 (st - KH) + k; col = (rhs, re/im);
    // weighted G^T, G^Q + i G^U, G^Q - i G^U
    const int k = lane >> 4, col = lane & 15, ri = col & 1;
    const int rhs = rb + (col >> 1);
    const bool rhs_ok = rhs < A.nrhs;
    T bop[kAnaKS][3];
#pragma unroll
    for (int st = 0; st < kAnaKS; ++st) {
        const int sd = st / kAnaKH;
        const int pair = pbase + 4 * (st % kAnaKH) + k;
        const bool ok = pair < A.npairs && rhs_ok;
        const int pc = ok ? pair : 0;
        const double w = pair_w[pc];
        const typename Vec2<T>::t* in =
            phase + ((((int64_t)(rhs_ok ? rhs : 0) * 3) * A.npairs + pc) * (A.mmax + 1) + m) * 2 + sd;
        const typename Vec2<T>::t t0 = in[0], q0 = in[fstride], u0 = in[2 * fstride];
        const double gt = ri ? t0.y : t0.x;
        const double gp = ri ? (q0.y + u0.x) : (q0.x - u0.y);
        const double gm = ri ? (q0.y - u0.x) : (q0.x + u0.y);
        bop[st][0] = ok ? (T)(w * gt) : (T)0;
        bop[st][1] = ok ? (T)(w * gp) : (T)0;
        bop[st][2] = ok ? (T)(w * gm) : (T)0;
    }
    __syncthreads();
    lo = s_lo[0];
    hi = s_hi[0];
    for (int q = 1; q < W; ++q) { lo = min(lo, s_lo[q]); hi = max(hi, s_hi[q]); }
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    if (m < 2) hi = max(hi, 2);

    const int nrhs = A.nrhs;
    PT* out = partial + ((int64_t)bp.x * nrhs * 3) * A.nalm * 2;
    // this column tile's part of the slot (a uniform base; lanes add byte
    // offsets within 8 RHS x 3 fields of nalm complex)
    char* const outb = reinterpret_cast<char*>(out + (int64_t)rb * 3 * A.nalm * 2);
    const OffT nal = (OffT)A.nalm;
    // degrees below the block's first start degree lo are not written: the
    // combine kernel reads this slot from lo on (the slot start table)
    if (lo > lend) return;

    T* tl = tile[wv];
    auto store = [&](int j, double lam, double pp, double qq) {
        tl[(0 * 16 + j) * RL + lane] = (T)lam;
        tl[(1 * 16 + j) * RL + lane] = (T)pp;
        tl[(2 * 16 + j) * RL + lane] = (T)qq;
    };
    // recursion of the round starting at degree l0 into the tile; modes 0
    // (steady) and 1 (activation) take the coefficients from cofb[cq]
    auto produce = [&](int l0, int cq, auto mode) {
        constexpr int kMode = decltype(mode)::value;            // 0 steady, 1 activation, 2 past lmax
        if constexpr (kMode == 2) {
            for (int j = 0; j < 16; ++j) {
                double lam, pp, qq;
                rec_step(A, cf, m, l0 + j, lo, hi, s, lam, pp, qq);
                store(j, lam, pp, qq);
            }
        } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                rec_advance(coef_lds(&cofb[cq][j * kCoefN]), s);
                if constexpr (kMode == 1) rec_activate(A, m, l0 + j, s);
                store(j, s.l1, s.w1, s.q1);
            }
        }
    };
    // coefficient pipeline (wave 0): cofb[cq] holds the degrees the current
    // round's recursion needs, creg the 16 degrees after them
    auto coef_group = [&](int l, int slot) { cofb[slot][lane] = coef_fetch(cf, l, lmax, lane, 16); };
    double creg0 = 0.0;

    // A operand of this lane: degree row, pair 4 st + k (the north K step
    // st and the mirror one st + KH share it)
    const int row = lane & 15;
    const int pofs = row * RL + k;
    const int oN[3] = {pofs, 16 * RL + pofs, 32 * RL + pofs};
    // eps of each output element: rounds advance by 16 degrees, so the
    // parity of a row is the same in every round
    T sg[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) sg[v] = ((lo + Mfma<T>::row(lane, v) + m) & 1) ? (T)-1 : (T)1;

    // sum over the waves of the round that started at degree l0,
    // held in red[qb], into the block's slot; element e of the round's
    // 3 x 8 x 16 x 2 outputs is re/im e & 1, degree (e >> 1) & 15, rhs
    // (e >> 5) & 7 and field e >> 8, so that each run of 32 threads writes
    // 128 contiguous bytes and a thread's fields are compile-time constants
    static_assert(768 % (64 * W) == 0, "the round's outputs split evenly over the block");
    auto reduce = [&](int l0, int qb) {
#pragma unroll
        for (int k = 0; k < 768 / (64 * W); ++k) {
            const int e = threadIdx.x + k * 64 * W;
            const int ri2 = e & 1, r = (e >> 1) & 15, rr = (e >> 5) & 7, f = e >> 8;
            const int ofs = f * kRedF + (2 * rr + ri2) * kRedCol + r;
            // in the products' own precision: FP32 on the mixed path, whose
            // slots hold FP32 anyway (the combine sums the slots in FP64)
            T sum = red[qb][0][ofs];
#pragma unroll
            for (int w2 = 1; w2 < W; ++w2) sum += red[qb][w2][ofs];
            const int l = l0 + r;
            if (l <= lend && rb + rr < nrhs)
                *reinterpret_cast<PT*>(outb + (((OffT)(rr * 3 + f) * nal + (OffT)(base + l)) * 2u + (OffT)ri2) *
                                                  (OffT)sizeof(PT)) = (PT)sum;
        }
    };

    if (lo + 15 <= lend) {
        for (int j = 0; j < 16; ++j) {
            rec_act(A, cf, m, lo + j, s);
            store(j, s.l1, s.w1, s.q1);
        }
    } else {
        produce(lo, 0, std::integral_constant<int, 2>());
    }
    if (wv == 0) {
        coef_group(lo + 16, 0);
        creg0 = coef_fetch(cf, lo + 32, lmax, lane, 16);
    }
    __syncthreads();
    int q = 0, l0 = lo;
    // one round; QC >= 0 fixes the slot parity q at compile time (the
    // steady loop's rounds, two per trip), QC = -1 takes it from q
    auto round = [&](auto mode, auto qc) {
        constexpr int QC = decltype(qc)::value;
        const int qr = QC >= 0 ? QC : q;
        v4 CN[3] = {v4{0, 0, 0, 0}, v4{0, 0, 0, 0}, v4{0, 0, 0, 0}};
        v4 CS[3] = {v4{0, 0, 0, 0}, v4{0, 0, 0, 0}, v4{0, 0, 0, 0}};
        // the north K step st and the mirror one st + KH read the same tile
        // values (lam, p, q) of pair 4 st + k: one read each serves both,
        // the mirror rows taking (lam, q, p)
#pragma unroll
        for (int st = 0; st < kAnaKH; ++st) {
            const int po = 4 * st;
            const T a0 = tl[oN[0] + po], a1 = tl[oN[1] + po], a2 = tl[oN[2] + po];
            CN[0] = Mfma<T>::run(a0, bop[st][0], CN[0]);
            CN[1] = Mfma<T>::run(a1, bop[st][1], CN[1]);
            CN[2] = Mfma<T>::run(a2, bop[st][2], CN[2]);
            CS[0] = Mfma<T>::run(a0, bop[st + kAnaKH][0], CS[0]);
            CS[1] = Mfma<T>::run(a2, bop[st + kAnaKH][1], CS[1]);
            CS[2] = Mfma<T>::run(a1, bop[st + kAnaKH][2], CS[2]);
            // keep the operand loads within a few K steps of their use
            if (st % 2 == 1) __builtin_amdgcn_sched_barrier(0);
        }
        constexpr int kMode = decltype(mode)::value;
        if (kMode != 2 && wv == 0) {
            // publish the next round's coefficients (visible after this
            // round's barrier), fetch the ones after them
            cofb[qr ^ 1][lane] = creg0;
            creg0 = coef_fetch(cf, l0 + 48, lmax, lane, 16);
        }
        // the products have read the tile (LDS operations of a wave
        // complete in order): the next round's recursion overwrites it
        if constexpr (kMode == 1) {
            if (l0 + 16 <= lend) {
                if (l0 + 16 <= hi_w) produce(l0 + 16, qr, mode);
                else produce(l0 + 16, qr, std::integral_constant<int, 0>());
            }
        } else {
            if (l0 + 16 <= lend) produce(l0 + 16, qr, mode);
        }
        if (l0 > lo) reduce(l0 - 16, qr ^ 1);
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                red[qr][wv][f * kRedF + col * kRedCol + Mfma<T>::row(lane, v)] = CN[f][v] + sg[v] * CS[f][v];
        __syncthreads();
    };
    using Qrt = std::integral_constant<int, -1>;
    using Q0 = std::integral_constant<int, 0>;
    using Q1 = std::integral_constant<int, 1>;
    // rounds whose successor has lanes starting in it
    for (; l0 + 16 <= hi && l0 + 31 <= lend; l0 += 16, q ^= 1) round(std::integral_constant<int, 1>(), Qrt());
    // steady rounds, two per trip (slot parity 0 then 1)
    if (q == 1 && l0 + 31 <= lend) {
        round(std::integral_constant<int, 0>(), Q1());
        l0 += 16;
        q = 0;
    }
    for (; l0 + 47 <= lend; l0 += 16) {
        round(std::integral_constant<int, 0>(), Q0());
        l0 += 16;
        round(std::integral_constant<int, 0>(), Q1());
    }
    if (l0 + 31 <= lend) {
        round(std::integral_constant<int, 0>(), Q0());
        l0 += 16;
        q = 1;
    }
    for (; l0 <= lend; l0 += 16, q ^= 1) round(std::integral_constant<int, 2>(), Qrt());
    // the last round's sum
    reduce(l0 - 16, q ^ 1);
}

BatchArgs batch_args(dm_plan* p, int nrhs) {
    BatchArgs a;
    a.lmax = p->lmax;
    a.mmax = p->mmax;
    a.npairs = p->npairs;
    a.nrhs = nrhs;
    a.nalm = p->nalm;
    a.pair_x = p->d_pair_x;
    a.coef = p->d_coef_s;
    a.scale = p->d_scale;
    a.lstart = p->d_lstart;
    a.seed = p->d_seed;
    a.sstride = (int64_t)(p->mmax + 1) * p->npairs;
    a.lend = (p->lcut > 0 && p->lcut < p->lmax) ? p->lcut : p->lmax;
    a.nx = 1;
    a.mchunk = 0;
    return a;
}

// waves per analysis block, both precisions: FP32 blocks take 77 KB of LDS
// and at most 256 registers per lane, so two blocks share a CU and one
// block's barriers do not stall the other (at Nside 1024, lmax 2048, 8 RHS:
// 8.8 against 9.7 ms for one block of 8 waves per CU); FP64 blocks take
// 152 KB, one per CU.  Both group 256 ring pairs per partial-sum slot.
constexpr int kAnaWaves = 4;

}  // namespace

int batched_analysis_slots(dm_plan* p) {
    const int per = kAnaPW * kAnaWaves;
    return (p->npairs + per - 1) / per;
}

namespace {

// first start degree of each (m, partial-sum slot): the smallest start
// degree of the slot's ring pairs (lmax + 1 if none starts)
__global__ void slot_start_kernel(int npairs, int per, int nslots, int lmax, const int* __restrict__ lstart,
                                  int* __restrict__ slot_lo) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (x >= nslots) return;
    int lo = lmax + 1;
    const int p1 = min(npairs, (x + 1) * per);
    for (int p = x * per; p < p1; ++p) lo = min(lo, lstart[(int64_t)m * npairs + p]);
    slot_lo[(int64_t)m * nslots + x] = lo;
}

}  // namespace

hipError_t launch_slot_starts(dm_plan* p, int* slot_lo, hipStream_t s) {
    const int nslots = batched_analysis_slots(p);
    dim3 grid((nslots + 63) / 64, p->mmax + 1);
    hipLaunchKernelGGL(slot_start_kernel, grid, dim3(64), 0, s, p->npairs, kAnaPW * kAnaWaves, nslots, p->lmax,
                       p->d_lstart, slot_lo);
    return hipGetLastError();
}

// 32-bit lane offsets hold when a column tile's 8 RHS x 3 fields of nalm
// complex FP64 values (the largest span a lane addresses from its uniform
// base) stay below 2^32 bytes: lmax <= 4727
static bool offsets_fit(dm_plan* p) { return (uint64_t)24 * (uint64_t)p->nalm * 16 < ((uint64_t)1 << 32); }

template <int W, typename OffT>
void launch_bsyn_wo(dm_plan* p, BatchArgs A, int nrhs, const double2* sp, void* phase, hipStream_t s) {
    const int pw = p->precision == DM_MIXED ? 64 : 32;
    A.nx = (p->npairs + pw * W - 1) / (pw * W);
    dim3 grid(grid_blocks(A.nx, p->mmax, A.mchunk), (nrhs + 7) / 8);
    dim3 block(64 * W);
    if (p->precision == DM_MIXED)
        hipLaunchKernelGGL((bsyn_kernel<float, 64, W, OffT>), grid, block, 0, s, A, sp, static_cast<float*>(phase));
    else
        hipLaunchKernelGGL((bsyn_kernel<double, 32, W, OffT>), grid, block, 0, s, A, sp, static_cast<double*>(phase));
}

template <int W>
void launch_bsyn_w(dm_plan* p, BatchArgs A, int nrhs, const double2* sp, void* phase, hipStream_t s) {
    if (offsets_fit(p)) launch_bsyn_wo<W, unsigned>(p, A, nrhs, sp, phase, s);
    else launch_bsyn_wo<W, uint64_t>(p, A, nrhs, sp, phase, s);
}

hipError_t launch_bsyn(dm_plan* p, int nrhs, const double* spin, void* phase, hipStream_t s) {
    BatchArgs A = batch_args(p, nrhs);
    A.mchunk = p->syn_mchunk;
    const double2* sp = reinterpret_cast<const double2*>(spin);
    if (p->syn_waves == 1) launch_bsyn_w<1>(p, A, nrhs, sp, phase, s);
    else if (p->syn_waves == 2) launch_bsyn_w<2>(p, A, nrhs, sp, phase, s);
    else if (p->syn_waves == 8) launch_bsyn_w<8>(p, A, nrhs, sp, phase, s);
    else launch_bsyn_w<4>(p, A, nrhs, sp, phase, s);
    return hipGetLastError();
}

hipError_t launch_bana(dm_plan* p, int nrhs, const void* phase, const double* pair_w, double* partial,
                       hipStream_t s) {
    BatchArgs A = batch_args(p, nrhs);
    A.nx = batched_analysis_slots(p);
    A.mchunk = p->ana_mchunk;
    dim3 grid(grid_blocks(A.nx, p->mmax, A.mchunk), (nrhs + 7) / 8);
    const bool fit = offsets_fit(p);
    if (p->precision == DM_MIXED && fit)
        hipLaunchKernelGGL((bana_kernel<float, kAnaWaves, float, unsigned>), grid, dim3(64 * kAnaWaves), 0, s, A,
                           static_cast<const float2*>(phase), pair_w, reinterpret_cast<float*>(partial));
    else if (p->precision == DM_MIXED)
        hipLaunchKernelGGL((bana_kernel<float, kAnaWaves, float, uint64_t>), grid, dim3(64 * kAnaWaves), 0, s, A,
                           static_cast<const float2*>(phase), pair_w, reinterpret_cast<float*>(partial));
    else if (fit)
        hipLaunchKernelGGL((bana_kernel<double, kAnaWaves, double, unsigned>), grid, dim3(64 * kAnaWaves), 0, s, A,
                           static_cast<const double2*>(phase), pair_w, partial);
    else
        hipLaunchKernelGGL((bana_kernel<double, kAnaWaves, double, uint64_t>), grid, dim3(64 * kAnaWaves), 0, s, A,
                           static_cast<const double2*>(phase), pair_w, partial);
    return hipGetLastError();
}

}  // namespace dmwf
