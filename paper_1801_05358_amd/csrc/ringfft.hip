// Ring step of the spherical harmonic transforms and the per-pixel
// messenger update of eq 9 (Algorithm 1's pixel-space half), one workgroup
// per ring pair (the north ring and its mirror, which share length and
// first-pixel longitude).
//
// Per field, the two real rings are packed as z = x_N + i x_S and
// transformed together:
//   synthesis   x_j = sum_{|m|<=mmax} F_m e^{i m (phi0 + 2 pi j / n)}:
//               fold F_m e^{i m phi0} into n bins (m mod n, with
//               F_{-m} = conj F_m), then an inverse DFT of length n;
//   update      t = K x + b  (eq 9 as t = u + T N^-1 (d - u));
//   analysis    G_m = e^{-i m phi0} DFT(t)[m mod n], m = 0..mmax, split
//               back into the two rings by Hermitian symmetry.
// Lengths 2^k use a radix-2 FFT in LDS and lengths 3 2^k a radix-3 pass
// joined to three radix-2 blocks (mixed radix); other lengths (most HEALPix
// polar rings, 4i) use Bluestein's chirp-z convolution with an FFT of size
// M >= 2n - 1, the smaller of 2^a and 3 2^b, also in LDS.  Where that M would be
// the largest buffer of the plan, a length n = 4i is split by decimation
// (four length-i Bluestein transforms and a radix-4 step), which needs
// max(n, M_i) elements instead.  Inverse transforms are conj(DFT(conj(.))).
#include "dmwf_internal.h"

namespace dmwf {

namespace {

// complex values of the transform's real type R (FP64, or FP32 for mixed
// plans that ask for it: the FFTs in LDS and the fold/unfold run in R, the
// ring data in HBM and the pixel update t = K x + b stay FP64)
template <typename R>
struct V2;
template <>
struct V2<double> {
    typedef double2 t;
};
template <>
struct V2<float> {
    typedef float2 t;
};
template <typename R>
using C2 = typename V2<R>::t;

template <typename R>
__device__ __forceinline__ C2<R> mk(R x, R y) {
    C2<R> c;
    c.x = x;
    c.y = y;
    return c;
}

template <typename R>
struct RingArgs {
    int npairs, mmax, logMmax, nrhs;
    const int* __restrict__ plist;   // the launch's ring pairs (null: all, in order)
    int nlist;
    int64_t npix;
    const RingPairDev* __restrict__ pairs;
    const FftLenDev* __restrict__ lens;
    const C2<R>* __restrict__ chirp;
    const C2<R>* __restrict__ bhat;
    const C2<R>* __restrict__ tw;
    const C2<R>* __restrict__ tw3;   // exp(-2 pi i e / (3 P3max)), e < 3 P3max
    int P3max;
};

// LDS layout of a transform buffer of size M = 2^logM: element i at
// i + i/8 + i/(M/8), with sh = logM - 3.  Eight consecutive lanes then hit
// eight distinct 16-byte bank groups both for the strided groups of the
// radix-8 passes (the i/8 term) and for bit-reversed positions, which differ
// by multiples of M/8 (the last term): the pixel loop and the Bluestein
// unfold address the buffer that way.
__device__ __forceinline__ int pad_shift(int logM) { return logM > 6 ? logM - 3 : 3; }
__device__ __forceinline__ int pidx(int i, int sh) { return i + (i >> 3) + (i >> sh); }

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    C c;
    c.x = a.x * b.x - a.y * b.y;
    c.y = a.x * b.y + a.y * b.x;
    return c;
}
template <typename C>
__device__ __forceinline__ C conjc(C a) {
    a.y = -a.y;
    return a;
}
__device__ __forceinline__ unsigned brev(unsigned j, int logM) {
    return logM == 0 ? 0u : (__brev(j) >> (32 - logM));
}

// Slot of logical index j in a transform buffer of size M: bit reversal for
// M = 2^logM; for M = 3 P (P = 2^logM) the mixed-radix digit reversal
// (j mod 3) P + brev(j div 3), which is both the input order of the
// decimation-in-time transform and the output order of the
// decimation-in-frequency one below.
__device__ __forceinline__ int perm(int j, const FftLenDev& L) {
    if (L.r3) {
        const int q = j / 3;
        return (j - 3 * q) * (L.M / 3) + (int)brev((unsigned)q, L.logM);
    }
    return (int)brev((unsigned)j, L.logM);
}

// logical index held by slot k (the inverse of perm): brev(k), or for
// M = 3 P, k = d P + e, the index 3 brev(e) + d
__device__ __forceinline__ int perm_inv(int k, const FftLenDev& L) {
    if (L.r3) return 3 * (int)brev((unsigned)(k & ((L.M / 3) - 1)), L.logM) + (k >> L.logM);
    return (int)brev((unsigned)k, L.logM);
}

// e^{i m phi0} with phi0 = pi / den (den = 0: phi0 = 0), reduced exactly
template <typename R>
__device__ __forceinline__ C2<R> phase_rot(int m, int den) {
    if (den == 0) return mk<R>(1, 0);
    const int per = 2 * den;
    int r = m % per;
    if (r < 0) r += per;
    R sn, cs;
    if constexpr (sizeof(R) == 8) sincospi((double)r / (double)den, &sn, &cs);
    else sincospif((float)r / (float)den, &sn, &cs);
    return mk<R>(cs, sn);
}

// Radix-2 stages in passes of up to three: one pass loads the 2^G elements
// base + c h (h = 2^s, c < 2^G) that stages s .. s+G-1 combine, applies the
// G stages in registers and stores them back, so that the LDS round trips
// and barriers drop threefold.  The stage-(s+t) twiddle of element c is
// W(j, s+t+1) w_t(c mod 2^t), with W(x, S) = exp(-2 pi i x / 2^S),
// j = base mod h and w_t(r) = exp(-2 pi i r / 2^(t+1)) a root of unity of
// order <= 8, so each group loads only G twiddles.
template <typename R>
__device__ __forceinline__ C2<R> root_mul(C2<R> w, int r, int t, bool inv) {
    // w * exp(-+ 2 pi i r / 2^(t+1)), r < 2^t, t <= 2
    if (r == 0) return w;
    const R sg = inv ? R(-1) : R(1);
    if (t == 1 || r == 2) return mk<R>(sg * w.y, -sg * w.x);                // * (-+i)
    const R c = R(0.70710678118654752440);                                    // r = 1 or 3, t = 2
    const C2<R> z = r == 1 ? mk<R>(c, -sg * c) : mk<R>(-c, -sg * c);
    return cmul(w, z);
}

// one group of a pass: the 2^G elements at slots at[c], stages s .. s+G-1
template <typename R, int G, bool DIT>
__device__ __forceinline__ void fft_group(C2<R>* buf, const int (&at)[1 << G], int j, int s, int logMmax,
                                          const C2<R>* __restrict__ tw, bool inv) {
    constexpr int NG = 1 << G;
    C2<R> x[NG];
#pragma unroll
    for (int c = 0; c < NG; ++c) x[c] = buf[at[c]];
    C2<R> wb[G];
#pragma unroll
    for (int t = 0; t < G; ++t) {
        wb[t] = tw[j << (logMmax - s - t - 1)];
        if (inv) wb[t].y = -wb[t].y;
    }
#pragma unroll
    for (int tt = 0; tt < G; ++tt) {
        const int t = DIT ? tt : G - 1 - tt;
        const int half = 1 << t;
#pragma unroll
        for (int c = 0; c < NG; ++c) {
            if (c & half) continue;
            const C2<R> a = x[c], b = x[c + half];
            const C2<R> w = root_mul<R>(wb[t], c & (half - 1), t, inv);
            if (DIT) {
                const C2<R> bw = cmul(b, w);
                x[c] = mk<R>(a.x + bw.x, a.y + bw.y);
                x[c + half] = mk<R>(a.x - bw.x, a.y - bw.y);
            } else {
                x[c] = mk<R>(a.x + b.x, a.y + b.y);
                x[c + half] = cmul(mk<R>(a.x - b.x, a.y - b.y), w);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NG; ++c) buf[at[c]] = x[c];
}

// The slots of a group's elements base + c h are pidx(base) + c step, with
// step = h + h/8 + h/2^sh, whenever neither shift of pidx carries across the
// group: s >= 3 or s + G <= 3 for i/8, and s >= sh or s + G <= sh for
// i/2^sh.  That holds for every pass of the transforms below but at most
// one per transform (the pass that straddles bit sh); those passes take
// pidx per element, the others one add per element.
template <typename R, int G, bool DIT>
__device__ __forceinline__ void fft_pass(C2<R>* buf, int M, int sh, int s, int logMmax,
                                         const C2<R>* __restrict__ tw, bool inv) {
    constexpr int NG = 1 << G;
    const int h = 1 << s;
    const int ngroups = M >> G;
    const bool lin = (s >= 3 || s + G <= 3) && (s >= sh || s + G <= sh);
    const int step = h + (h >> 3) + (h >> sh);
    if (lin) {
        for (int q = threadIdx.x; q < ngroups; q += blockDim.x) {
            const int j = q & (h - 1);
            const int base = ((q >> s) << (s + G)) + j;
            int at[NG];
            at[0] = pidx(base, sh);
#pragma unroll
            for (int c = 1; c < NG; ++c) at[c] = at[c - 1] + step;
            fft_group<R, G, DIT>(buf, at, j, s, logMmax, tw, inv);
        }
    } else {
        for (int q = threadIdx.x; q < ngroups; q += blockDim.x) {
            const int j = q & (h - 1);
            const int base = ((q >> s) << (s + G)) + j;
            int at[NG];
#pragma unroll
            for (int c = 0; c < NG; ++c) at[c] = pidx(base + c * h, sh);
            fft_group<R, G, DIT>(buf, at, j, s, logMmax, tw, inv);
        }
    }
    __syncthreads();
}

// decimation in time: bit-reversed input, natural output
template <typename R>
__device__ void fft_dit(C2<R>* buf, int M, int logM, int logMmax, const C2<R>* __restrict__ tw, bool inv) {
    const int sh = pad_shift(logM);
    int s = 0;
    for (; s + 3 <= logM; s += 3) fft_pass<R, 3, true>(buf, M, sh, s, logMmax, tw, inv);
    if (logM - s == 2) fft_pass<R, 2, true>(buf, M, sh, s, logMmax, tw, inv);
    else if (logM - s == 1) fft_pass<R, 1, true>(buf, M, sh, s, logMmax, tw, inv);
}

// decimation in frequency: natural input, bit-reversed output
template <typename R>
__device__ void fft_dif(C2<R>* buf, int M, int logM, int logMmax, const C2<R>* __restrict__ tw, bool inv) {
    const int sh = pad_shift(logM);
    // the stages that do not fill a radix-8 pass first, so that the radix-8
    // passes sit at s = 0, 3, 6, ... (as in the DIT transform)
    int top = logM;
    if (logM % 3 == 2) fft_pass<R, 2, false>(buf, M, sh, top - 2, logMmax, tw, inv), top -= 2;
    else if (logM % 3 == 1) fft_pass<R, 1, false>(buf, M, sh, top - 1, logMmax, tw, inv), top -= 1;
    for (; top >= 3; top -= 3) fft_pass<R, 3, false>(buf, M, sh, top - 3, logMmax, tw, inv);
}

// The radix-3 pass of a size M = 3 P: elements k, P + k, 2P + k for
// k < P.  Decimation in time (after three DIT transforms of length P, which
// leave Y_r[k] at r P + k):  X[k + P q] = sum_r W_3^{r q} W_M^{r k} Y_r[k],
// stored at q P + k, natural order.  Decimation in frequency (before three
// DIF transforms of length P):  y_q[k] = W_M^{q k} sum_r W_3^{r q} x[k + P r],
// stored at q P + k.  Twiddles W_M^e = tw3[e P3max / P]; inv conjugates every
// root (the inverse transform).
template <typename R, bool DIT>
__device__ void r3_pass(C2<R>* buf, int P, int sh, const C2<R>* __restrict__ tw3, int P3max, bool inv) {
    const int st = P3max / P;
    const int Ps = P + (P >> 3) + (P >> sh);
    const R h = R(0.86602540378443864676);          // sin(2 pi / 3)
    const R sg = inv ? R(-1) : R(1);
    for (int k = threadIdx.x; k < P; k += blockDim.x) {
        C2<R> w1 = tw3[k * st], w2 = tw3[2 * k * st];
        if (inv) { w1.y = -w1.y; w2.y = -w2.y; }
        // P = 2^k with k >= 3 is a multiple of 8 and of 2^sh: the slots of k, P + k, 2P + k
        // are pidx(k) + {0, 1, 2} (P + P/8 + P/2^sh)
        const int a0 = pidx(k, sh), a1 = a0 + Ps, a2 = a1 + Ps;
        C2<R> x0 = buf[a0], x1 = buf[a1], x2 = buf[a2];
        if (DIT) { x1 = cmul(x1, w1); x2 = cmul(x2, w2); }
        const C2<R> t1 = mk<R>(x1.x + x2.x, x1.y + x2.y), t2 = mk<R>(x1.x - x2.x, x1.y - x2.y);
        const C2<R> mid = mk<R>(x0.x - R(0.5) * t1.x, x0.y - R(0.5) * t1.y);
        // -+ i sin(2 pi / 3) t2
        const C2<R> it = mk<R>(sg * h * t2.y, -sg * h * t2.x);
        C2<R> y1 = mk<R>(mid.x + it.x, mid.y + it.y), y2 = mk<R>(mid.x - it.x, mid.y - it.y);
        if (!DIT) { y1 = cmul(y1, w1); y2 = cmul(y2, w2); }
        buf[a0] = mk<R>(x0.x + t1.x, x0.y + t1.y);
        buf[a1] = y1;
        buf[a2] = y2;
    }
    __syncthreads();
}

// transforms of a buffer of size M (2^logM, or 3 2^logM as three aligned
// blocks of 2^logM: the radix-2 passes never cross a block)
template <typename R>
__device__ void fft_dit_any(C2<R>* buf, const FftLenDev& L, const RingArgs<R>& A, bool inv) {
    fft_dit<R>(buf, L.M, L.logM, A.logMmax, A.tw, inv);
    if (L.r3) r3_pass<R, true>(buf, L.M / 3, pad_shift(L.logM), A.tw3, A.P3max, inv);
}
template <typename R>
__device__ void fft_dif_any(C2<R>* buf, const FftLenDev& L, const RingArgs<R>& A, bool inv) {
    if (L.r3) r3_pass<R, false>(buf, L.M / 3, pad_shift(L.logM), A.tw3, A.P3max, inv);
    fft_dif<R>(buf, L.M, L.logM, A.logMmax, A.tw, inv);
}

// Forward DFT core.  On entry buf[perm(j)] holds a_j (times chirp_j for
// Bluestein, zeros at perm(j) for j >= n).  On exit the transform value X_k
// is at buf[k] (direct lengths) or buf[perm(k)] times chirp_k (Bluestein).
template <typename R>
__device__ void dft_core(C2<R>* buf, const FftLenDev& L, const RingArgs<R>& A) {
    if (!L.bluestein) {
        fft_dit_any<R>(buf, L, A, false);
    } else {
        fft_dit_any<R>(buf, L, A, false);
        const C2<R>* bh = A.bhat + L.bhat_off;
        const int sh = pad_shift(L.logM);
        for (int q = threadIdx.x; q < L.M; q += blockDim.x) buf[pidx(q, sh)] = cmul(buf[pidx(q, sh)], bh[q]);
        __syncthreads();
        fft_dif_any<R>(buf, L, A, true);
    }
}

// Inverse-direction core for the synthesis: on entry buf holds conj(c)
// placed for the transform; on exit x_j = conj(value at perm(j)) (times
// chirp for Bluestein).  For direct lengths the input is in natural order.
template <typename R>
__device__ void idft_core(C2<R>* buf, const FftLenDev& L, const RingArgs<R>& A) {
    if (!L.bluestein) {
        fft_dif_any<R>(buf, L, A, false);
    } else {
        dft_core<R>(buf, L, A);
    }
}


// out[r] = sum_q (-i)^{r q} v_q (a length-4 DFT)
template <typename R>
__device__ __forceinline__ void dft4(C2<R> v0, C2<R> v1, C2<R> v2, C2<R> v3, C2<R> (&out)[4]) {
    const C2<R> a = mk<R>(v0.x + v2.x, v0.y + v2.y), b = mk<R>(v0.x - v2.x, v0.y - v2.y);
    const C2<R> c = mk<R>(v1.x + v3.x, v1.y + v3.y), d = mk<R>(v1.x - v3.x, v1.y - v3.y);
    out[0] = mk<R>(a.x + c.x, a.y + c.y);
    out[2] = mk<R>(a.x - c.x, a.y - c.y);
    out[1] = mk<R>(b.x + d.y, b.y - d.x);   // b - i d
    out[3] = mk<R>(b.x - d.y, b.y + d.x);   // b + i d
}

// exp(-2 pi i e / n) for 0 <= e < n
template <typename R>
__device__ __forceinline__ C2<R> unit_root(int e, int n) {
    R sn, cs;
    if constexpr (sizeof(R) == 8) sincospi(2.0 * (double)e / (double)n, &sn, &cs);
    else sincospif(2.0f * (float)e / (float)n, &sn, &cs);
    return mk<R>(cs, -sn);
}

// SPLITK > 0: the launch over the split rings (n = 4 i, see split_ring
// below), each lane holding SPLITK values of kappa (i <= SPLITK blockDim.x,
// checked when the plan is made); the other rings run in a launch of their
// own, so that neither carries the other's registers or buffer size.
template <int MODE, int SPLITK, typename R, typename P>
__global__ __launch_bounds__(SPLITK > 0 ? 512 : 1024) void ring_kernel(RingArgs<R> A, const double* __restrict__ map_in,
                                                   double* __restrict__ map_out, const double* __restrict__ Kp,
                                                   const double* __restrict__ bp, C2<P>* __restrict__ phase) {
    typedef C2<R> CR;
    typedef C2<P> CP;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    CR* buf = reinterpret_cast<CR*>(lds_raw);
    // workgroups go to the 8 XCDs in turn: the RHS of one ring pair are
    // placed consecutively on one XCD, so that they share that ring's
    // tables (chirp, Bluestein kernel, K) in its L2
    const int c = blockIdx.x % 8, k = blockIdx.x / 8;
    const int rhs = k % A.nrhs;
    const int idx = 8 * (k / A.nrhs) + c;
    if (idx >= A.nlist) return;
    const int p = A.plist ? A.plist[idx] : idx;
    const RingPairDev P_ = A.pairs[p];
    const FftLenDev L = A.lens[P_.len_idx];
    const int n = P_.nphi, M = L.M, logM = L.logM, sh = pad_shift(logM);
    const int nt = blockDim.x, tid = threadIdx.x;
    const int mmax = A.mmax;
    const bool synth = (MODE == RING_SYNTH || MODE == RING_ITERATE);
    const bool anal = (MODE == RING_ANALYSIS || MODE == RING_ITERATE || MODE == RING_ANALYSIS6);
    // the analysis input of field f at pixel pix: the map, or (3x3 noise)
    // the messenger t_f = u_x,f - (T_p P_p u_x)_f + b_f from the three fields
    // of u_x, with the arithmetic of the separate 3x3 update pass
    auto in_val = [&](int f, int64_t moff, int64_t pix) -> double {
        if constexpr (MODE == RING_ANALYSIS6) {
            const int64_t np = A.npix;
            const int64_t base = moff - (int64_t)f * np + pix;
            const double x0 = map_in[base], x1 = map_in[base + np], x2 = map_in[base + 2 * np];
            double y, xf;
            if (f == 0) {
                y = Kp[pix] * x0 + Kp[np + pix] * x1 + Kp[2 * np + pix] * x2;
                xf = x0;
            } else if (f == 1) {
                y = Kp[np + pix] * x0 + Kp[3 * np + pix] * x1 + Kp[4 * np + pix] * x2;
                xf = x1;
            } else {
                y = Kp[2 * np + pix] * x0 + Kp[4 * np + pix] * x1 + Kp[5 * np + pix] * x2;
                xf = x2;
            }
            return (xf - y) + bp[moff + pix];
        } else {
            return map_in[moff + pix];
        }
    };
    const CR* chirp = L.bluestein ? A.chirp + L.chirp_off : nullptr;
    const CR zero = mk<R>(0, 0);
    // split ring (n = 4 i): the buffer holds the length-n spectrum or ring in
    // natural order (padding i/8 only) and, in turn, the four length-i
    // Bluestein transforms of size M; blu: whole-ring Bluestein (bit-reversed
    // slots, chirp factors)
    constexpr bool split = SPLITK > 0;
    constexpr int kSplitK = SPLITK > 0 ? SPLITK : 1;
    const bool blu = L.bluestein && !split;
    const int shn = split ? 31 : sh;
    const int i4 = n >> 2;
    // W^kappa = exp(-2 pi i kappa / n) of this lane's kappa = tid + nt u
    CR w1[kSplitK];
    if constexpr (split) {
#pragma unroll
        for (int u = 0; u < kSplitK; ++u) {
            const int kap = tid + nt * u;
            w1[u] = kap < i4 ? unit_root<R>(kap, n) : mk<R>(1, 0);
        }
    }
    // the factor e^{i n phi0} between aliased m of the synthesis fold (-1 on
    // HEALPix rings, whose phi0 = pi / n, 1 for phi0 = 0)
    const CR alias_step = phase_rot<R>(n, P_.phi0_den);

    // A split ring's transform between the folded spectrum (natural order,
    // synthesis) or the ring (analysis) and the spectrum X (natural order):
    //   DFT(v)_{4 j' + r} = DFT_i(G_r)[j'],  G_r[kap] = W^{r kap} sum_q (-i)^{r q} v_{kap + q i},
    //   X_{kap + q i} = sum_r (-i)^{r q} W^{r kap} Y_r[kap],  Y_r = DFT_i(t_{4 j' + r}),
    // with W = exp(-2 pi i / n).  Per r the inverse sub-transform, the pixel
    // update of pixels 4 j' + r and the forward sub-transform run back to
    // back; G_r and then W^{r kap} Y_r stay in registers.
    auto split_ring = [&](int f, int64_t moff) {
        CR Z[kSplitK][4];
        auto wpow = [&](int u, int r) {
            CR w = mk<R>(1, 0);
            for (int e = 0; e < r; ++e) w = cmul(w, w1[u]);
            return w;
        };
        if (synth) {
#pragma unroll
            for (int u = 0; u < kSplitK; ++u) {
                const int kap = tid + nt * u;
                if (kap < i4) {
                    dft4<R>(buf[pidx(kap, shn)], buf[pidx(kap + i4, shn)], buf[pidx(kap + 2 * i4, shn)],
                         buf[pidx(kap + 3 * i4, shn)], Z[u]);
#pragma unroll
                    for (int r = 1; r < 4; ++r) Z[u][r] = cmul(Z[u][r], wpow(u, r));
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (synth) {
#pragma unroll
                for (int u = 0; u < kSplitK; ++u) {
                    const int kap = tid + nt * u;
                    if (kap < i4) buf[pidx((int)brev(kap, logM), sh)] = cmul(Z[u][r], chirp[kap]);
                }
                for (int jj = i4 + tid; jj < M; jj += nt) buf[pidx((int)brev(jj, logM), sh)] = zero;
                __syncthreads();
                dft_core<R>(buf, L, A);
                // x_{4 j' + r} = conj(buf[brev(j')] chirp_j')
                for (int jp = tid; jp < i4; jp += nt) {
                    const int q = (int)brev(jp, logM);
                    const CR y = cmul(buf[pidx(q, sh)], chirp[jp]);
                    const int j = 4 * jp + r;
                    const double xn = (double)y.x, xs = -(double)y.y;
                    if (MODE == RING_SYNTH) {
                        map_out[moff + P_.off_n + j] = xn;
                        if (P_.has_s) map_out[moff + P_.off_s + j] = xs;
                    } else {
                        const int64_t kn = (int64_t)f * A.npix + P_.off_n + j;
                        const double tn = Kp[kn] * xn + bp[moff + P_.off_n + j];
                        double ts = 0.0;
                        if (P_.has_s) {
                            const int64_t ks = (int64_t)f * A.npix + P_.off_s + j;
                            ts = Kp[ks] * xs + bp[moff + P_.off_s + j];
                        }
                        if (map_out) {
                            map_out[moff + P_.off_n + j] = tn;
                            if (P_.has_s) map_out[moff + P_.off_s + j] = ts;
                        }
                        buf[pidx(q, sh)] = cmul(mk<R>((R)tn, (R)ts), chirp[jp]);
                    }
                }
                if (MODE == RING_ITERATE)
                    for (int jj = i4 + tid; jj < M; jj += nt) buf[pidx((int)brev(jj, logM), sh)] = zero;
                __syncthreads();
            } else {
                for (int jp = tid; jp < M; jp += nt) {
                    CR a = zero;
                    if (jp < i4) {
                        const int j = 4 * jp + r;
                        a.x = (R)in_val(f, moff, P_.off_n + j);
                        a.y = P_.has_s ? (R)in_val(f, moff, P_.off_s + j) : R(0);
                        a = cmul(a, chirp[jp]);
                    }
                    buf[pidx((int)brev(jp, logM), sh)] = a;
                }
                __syncthreads();
            }
            if (anal) {
                dft_core<R>(buf, L, A);
#pragma unroll
                for (int u = 0; u < kSplitK; ++u) {
                    const int kap = tid + nt * u;
                    if (kap < i4) {
                        const CR y = cmul(buf[pidx((int)brev(kap, logM), sh)], chirp[kap]);
                        Z[u][r] = r == 0 ? y : cmul(y, wpow(u, r));
                    }
                }
                __syncthreads();
            }
        }
        if (anal) {
#pragma unroll
            for (int u = 0; u < kSplitK; ++u) {
                const int kap = tid + nt * u;
                if (kap < i4) {
                    CR X[4];
                    dft4<R>(Z[u][0], Z[u][1], Z[u][2], Z[u][3], X);
#pragma unroll
                    for (int q = 0; q < 4; ++q) buf[pidx(kap + q * i4, shn)] = X[q];
                }
            }
            __syncthreads();
        }
    };

    for (int f = 0; f < 3; ++f) {
        CP* ph = phase + (((int64_t)rhs * 3 + f) * A.npairs + p) * (mmax + 1) * 2;
        const int64_t moff = ((int64_t)rhs * 3 + f) * A.npix;
        if (synth) {
            // fold into n bins, place conj(C_N + i C_S) for the inverse
            // transform.  Lanes take consecutive logical indices j (coalesced
            // ring-data reads; the slot is perm(j) for Bluestein lengths).
            // e^{i mstart phi0} = e^{i j phi0} e^{-i w n phi0} with
            // mstart = j - w n: the first factor advances by e^{i nt phi0}
            // from one j of a lane to the next, and the second is (-1)^w on
            // rings with n phi0 = pi (HEALPix) and 1 for phi0 = 0.
            const bool half_turn = P_.phi0_den == n;
            CR rotj = phase_rot<R>(tid, P_.phi0_den);
            const CR rstep = phase_rot<R>(nt, P_.phi0_den);
            for (int j = tid; j < n; j += nt, rotj = cmul(rotj, rstep)) {
                CR v = zero;
                const int k = blu ? perm(j, L) : j;           // slot of logical index j
                {
                    CR cn = zero, cs = zero;
                    const int w = (j + mmax) / n;
                    const int mstart = j - n * w;
                    CR rot;
                    if (P_.phi0_den == 0) rot = mk<R>(1, 0);
                    else if (half_turn) rot = (w & 1) ? mk<R>(-rotj.x, -rotj.y) : rotj;
                    else rot = phase_rot<R>(mstart, P_.phi0_den);
                    for (int m = mstart; m <= mmax; m += n) {
                        const int a = m < 0 ? -m : m;
                        const CP fnd = ph[2 * a], fsd = ph[2 * a + 1];
                        CR fn = mk<R>((R)fnd.x, (R)fnd.y), fs = mk<R>((R)fsd.x, (R)fsd.y);
                        if (m < 0) { fn.y = -fn.y; fs.y = -fs.y; }
                        const CR tn = cmul(fn, rot), ts = cmul(fs, rot);
                        cn.x += tn.x; cn.y += tn.y;
                        cs.x += ts.x; cs.y += ts.y;
                        rot = cmul(rot, alias_step);
                    }
                    // z = C_N + i C_S ; store conj(z)
                    v = mk<R>(cn.x - cs.y, -(cn.y + cs.x));
                    if (blu) v = cmul(v, chirp[j]);
                }
                buf[pidx(k, shn)] = v;
            }
            // Bluestein: zeros in the slots of the indices n .. M-1
            if (blu)
                for (int k = tid; k < M; k += nt)
                    if (perm_inv(k, L) >= n) buf[pidx(k, sh)] = zero;
            __syncthreads();
        }
        if constexpr (split) {
            split_ring(f, moff);
        } else if (synth) {
            idft_core<R>(buf, L, A);
            // now x_j (packed N + i S) = conj(buf[perm(j)] * chirp_j)
            for (int j = tid; j < n; j += nt) {
                const int q = perm(j, L);
                CR y = buf[pidx(q, sh)];
                if (L.bluestein) y = cmul(y, chirp[j]);
                const double xn = (double)y.x, xs = -(double)y.y;
                if (MODE == RING_SYNTH) {
                    map_out[moff + P_.off_n + j] = xn;
                    if (P_.has_s) map_out[moff + P_.off_s + j] = xs;
                } else {
                    const int64_t kn = (int64_t)f * A.npix + P_.off_n + j;
                    double tn = Kp[kn] * xn + bp[moff + P_.off_n + j];
                    double ts = 0.0;
                    if (P_.has_s) {
                        const int64_t ks = (int64_t)f * A.npix + P_.off_s + j;
                        ts = Kp[ks] * xs + bp[moff + P_.off_s + j];
                    }
                    if (map_out) {
                        map_out[moff + P_.off_n + j] = tn;
                        if (P_.has_s) map_out[moff + P_.off_s + j] = ts;
                    }
                    CR a = mk<R>((R)tn, (R)ts);
                    if (L.bluestein) a = cmul(a, chirp[j]);
                    buf[pidx(q, sh)] = a;
                }
            }
            if (MODE == RING_ITERATE && L.bluestein) {
                for (int k = tid; k < M; k += nt)
                    if (perm_inv(k, L) >= n) buf[pidx(k, sh)] = zero;
            }
            __syncthreads();
        }
        if ((MODE == RING_ANALYSIS || MODE == RING_ANALYSIS6) && !split) {
            // lanes take consecutive pixels j (coalesced reads); a_j goes to
            // the digit-reversed slot perm(j)
            for (int j = tid; j < n; j += nt) {
                CR a;
                a.x = (R)in_val(f, moff, P_.off_n + j);
                a.y = P_.has_s ? (R)in_val(f, moff, P_.off_s + j) : R(0);
                if (L.bluestein) a = cmul(a, chirp[j]);
                buf[pidx(perm(j, L), sh)] = a;
            }
            if (L.bluestein)
                for (int k = tid; k < M; k += nt)
                    if (perm_inv(k, L) >= n) buf[pidx(k, sh)] = zero;
            __syncthreads();
        }
        if (anal) {
            if (!split) dft_core<R>(buf, L, A);
            // unfold: X_N = (Z_k + conj Z_{-k}) / 2,  X_S = (Z_k - conj Z_{-k}) / (2i)
            auto unfold = [&](int m, CR rot) {
                const int k = m % n;
                const int k2 = (n - k) % n;
                const int q1 = blu ? perm(k, L) : k;
                const int q2 = blu ? perm(k2, L) : k2;
                CR z1 = buf[pidx(q1, shn)], z2 = buf[pidx(q2, shn)];
                if (blu) { z1 = cmul(z1, chirp[k]); z2 = cmul(z2, chirp[k2]); }
                const CR xn = mk<R>(R(0.5) * (z1.x + z2.x), R(0.5) * (z1.y - z2.y));
                const CR xs = mk<R>(R(0.5) * (z1.y + z2.y), R(-0.5) * (z1.x - z2.x));
                const CR on = cmul(xn, rot), os = cmul(xs, rot);
                ph[2 * m] = mk<P>((P)on.x, (P)on.y);
                ph[2 * m + 1] = P_.has_s ? mk<P>((P)os.x, (P)os.y) : mk<P>(0, 0);
            };
            // e^{-i m phi0} for m = tid, tid + nt, ...: one rotation per step
            CR rot = conjc(phase_rot<R>(tid, P_.phi0_den));
            const CR ustep = conjc(phase_rot<R>(nt, P_.phi0_den));
            for (int m = tid; m <= mmax; m += nt, rot = cmul(rot, ustep)) unfold(m, rot);
            __syncthreads();
        }
    }
}

template <typename R>
RingArgs<R> ring_args(dm_plan* p, const void* chirp, const void* bhat, const void* tw, const void* tw3) {
    RingArgs<R> A;
    A.npairs = p->npairs;
    A.plist = nullptr;
    A.nlist = p->npairs;
    A.mmax = p->mmax;
    int lm = 0;
    while ((1 << lm) < p->fft.Mmax) ++lm;
    A.logMmax = lm;
    A.npix = p->npix;
    A.pairs = p->d_pairs;
    A.lens = p->d_fftlen;
    A.chirp = reinterpret_cast<const C2<R>*>(chirp);
    A.bhat = reinterpret_cast<const C2<R>*>(bhat);
    A.tw = reinterpret_cast<const C2<R>*>(tw);
    A.tw3 = reinterpret_cast<const C2<R>*>(tw3);
    A.P3max = p->fft.P3max;
    return A;
}

template <int MODE, int SPLITK, typename R, typename P>
void launch_mode(const RingArgs<R>& A, int nlist, const int* plist, int lds_elems, int threads,
                 const double* map_in, double* map_out, const double* K, const double* b, C2<P>* ph, hipStream_t s) {
    if (nlist <= 0) return;
    RingArgs<R> Ar = A;
    Ar.plist = plist;
    Ar.nlist = nlist;
    const dim3 grid((unsigned)(((nlist + 7) / 8) * 8 * A.nrhs));
    // padded layout: up to M + M/8 + 24 elements for M = 3 2^k (pidx)
    const size_t lds = (size_t)(lds_elems + lds_elems / 8 + 32) * sizeof(C2<R>);
    hipLaunchKernelGGL((ring_kernel<MODE, SPLITK, R, P>), grid, dim3(threads), lds, s, Ar, map_in, map_out, K, b, ph);
}

// One launch over every ring pair, or (with split rings) one over the
// others and one over the split rings.  Where the unsplit pairs have both
// transform buffers above 80 KB and below, and the launch has at least
// kRingClassMinRhs right-hand sides, they run in two launches, each with its
// own buffer size: at Nside 1024 with 8 RHS the ring step takes 4.4 instead
// of 5.0 ms; with 1 RHS the second launch's tail makes it slower (1.31
// against 0.96 ms).
constexpr int kRingClassMinRhs = 4;
template <int MODE, typename R, typename P>
void launch_both(dm_plan* p, const RingArgs<R>& A, const double* map_in, double* map_out, const double* K,
                 const double* b, C2<P>* ph, hipStream_t s) {
    if (p->ring_classes && A.nrhs >= kRingClassMinRhs) {
        // the large transforms first, one workgroup per CU (1024 threads by
        // default); then the others with a smaller buffer, two workgroups per
        // CU (512 threads by default); the autotuner may pick other widths
        launch_mode<MODE, 0, R, P>(A, p->n_big, p->d_plist_big, p->lds_big, p->ring_big_threads, map_in, map_out, K,
                                   b, ph, s);
        launch_mode<MODE, 0, R, P>(A, p->n_small, p->d_plist_small, p->lds_small, p->ring_small_threads, map_in,
                                   map_out, K, b, ph, s);
    } else if (p->n_split == 0) {
        launch_mode<MODE, 0, R, P>(A, p->npairs, nullptr, p->fft.lds_elems, p->ring_threads, map_in, map_out, K, b,
                                   ph, s);
        return;
    } else {
        launch_mode<MODE, 0, R, P>(A, p->n_whole, p->d_plist_whole, p->fft.lds_elems, p->ring_threads, map_in,
                                   map_out, K, b, ph, s);
    }
    if (p->n_split == 0) return;
    if (p->split_k <= 2)
        launch_mode<MODE, 2, R, P>(A, p->n_split, p->d_plist_split, p->fft.lds_split, p->fft_threads, map_in,
                                   map_out, K, b, ph, s);
    else
        launch_mode<MODE, 4, R, P>(A, p->n_split, p->d_plist_split, p->fft.lds_split, p->fft_threads, map_in,
                                   map_out, K, b, ph, s);
}

template <typename R, typename P>
void launch_ring_t(dm_plan* p, int mode, int nrhs, const double* map_in, double* map_out, const double* K,
                   const double* b, void* phase, const RingArgs<R>& A, hipStream_t s) {
    C2<P>* ph = static_cast<C2<P>*>(phase);
    RingArgs<R> Ar = A;
    Ar.nrhs = nrhs;
    switch (mode) {
        case RING_ANALYSIS: launch_both<RING_ANALYSIS, R, P>(p, Ar, map_in, map_out, K, b, ph, s); break;
        case RING_SYNTH: launch_both<RING_SYNTH, R, P>(p, Ar, map_in, map_out, K, b, ph, s); break;
        case RING_ANALYSIS6: launch_both<RING_ANALYSIS6, R, P>(p, Ar, map_in, map_out, K, b, ph, s); break;
        default: launch_both<RING_ITERATE, R, P>(p, Ar, map_in, map_out, K, b, ph, s); break;
    }
}

template <int MODE, int SPLITK, typename R, typename P>
hipError_t set_lds_one(size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&ring_kernel<MODE, SPLITK, R, P>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int SPLITK, typename R, typename P>
hipError_t set_lds_modes(size_t bytes) {
    hipError_t e = set_lds_one<RING_ANALYSIS, SPLITK, R, P>(bytes);
    if (e == hipSuccess) e = set_lds_one<RING_SYNTH, SPLITK, R, P>(bytes);
    if (e == hipSuccess) e = set_lds_one<RING_ITERATE, SPLITK, R, P>(bytes);
    if (e == hipSuccess) e = set_lds_one<RING_ANALYSIS6, SPLITK, R, P>(bytes);
    return e;
}

template <typename R, typename P>
hipError_t set_lds_t(size_t bytes) {
    hipError_t e = set_lds_modes<0, R, P>(bytes);
    if (e == hipSuccess) e = set_lds_modes<2, R, P>(bytes);
    if (e == hipSuccess) e = set_lds_modes<4, R, P>(bytes);
    return e;
}

}  // namespace

// FP64 transforms on FP64 ring data; on FP32 ring data (mixed plans) FP32
// transforms if the plan carries the FP32 tables (opt-in), else FP64
hipError_t launch_ring(dm_plan* p, int mode, int nrhs, const double* map_in, double* map_out, const double* K,
                       const double* b, void* phase, bool phase32, hipStream_t s) {
    if (!phase32) {
        const RingArgs<double> A = ring_args<double>(p, p->d_chirp, p->d_bhat, p->d_tw, p->d_tw3);
        launch_ring_t<double, double>(p, mode, nrhs, map_in, map_out, K, b, phase, A, s);
    } else if (p->d_tw32) {
        const RingArgs<float> A = ring_args<float>(p, p->d_chirp32, p->d_bhat32, p->d_tw32, p->d_tw332);
        launch_ring_t<float, float>(p, mode, nrhs, map_in, map_out, K, b, phase, A, s);
    } else {
        const RingArgs<double> A = ring_args<double>(p, p->d_chirp, p->d_bhat, p->d_tw, p->d_tw3);
        launch_ring_t<double, float>(p, mode, nrhs, map_in, map_out, K, b, phase, A, s);
    }
    return hipGetLastError();
}

hipError_t ring_set_lds_limit(size_t bytes) {
    hipError_t e = set_lds_t<double, double>(bytes);
    if (e != hipSuccess) return e;
    e = set_lds_t<double, float>(bytes);
    if (e != hipSuccess) return e;
    return set_lds_t<float, float>(bytes / 2);
}

}  // namespace dmwf
