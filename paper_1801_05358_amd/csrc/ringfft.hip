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
// Lengths that are powers of two use a radix-2 FFT in LDS; other lengths
// (most HEALPix polar rings, 4i) use Bluestein's chirp-z convolution with a
// power-of-two FFT of size M >= 2n - 1, also in LDS.  Inverse transforms
// are conj(DFT(conj(.))).
#include "dmwf_internal.h"

namespace dmwf {

namespace {

struct RingArgs {
    int npairs, mmax, logMmax;
    int64_t npix;
    const RingPairDev* __restrict__ pairs;
    const FftLenDev* __restrict__ lens;
    const double2* __restrict__ chirp;
    const double2* __restrict__ bhat;
    const double2* __restrict__ tw;
};

// LDS layout of a transform buffer: element i at i + i/8, so that the
// stride-8 and stride-64 element groups of the first radix-8 passes fall in
// distinct banks (one 16-byte pad per 128 bytes)
__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ unsigned brev(unsigned j, int logM) {
    return logM == 0 ? 0u : (__brev(j) >> (32 - logM));
}

// e^{i m phi0} with phi0 = pi / den (den = 0: phi0 = 0), reduced exactly
__device__ __forceinline__ double2 phase_rot(int m, int den) {
    if (den == 0) return make_double2(1.0, 0.0);
    const int per = 2 * den;
    int r = m % per;
    if (r < 0) r += per;
    double s, c;
    sincospi((double)r / (double)den, &s, &c);
    return make_double2(c, s);
}

// Radix-2 stages in passes of up to three: one pass loads the 2^R elements
// base + c h (h = 2^s, c < 2^R) that stages s .. s+R-1 combine, applies the
// R stages in registers and stores them back, so that the LDS round trips
// and barriers drop threefold.  The stage-(s+t) twiddle of element c is
// W(j, s+t+1) w_t(c mod 2^t), with W(x, S) = exp(-2 pi i x / 2^S),
// j = base mod h and w_t(r) = exp(-2 pi i r / 2^(t+1)) a root of unity of
// order <= 8, so each group loads only R twiddles.
__device__ __forceinline__ double2 root_mul(double2 w, int r, int t, bool inv) {
    // w * exp(-+ 2 pi i r / 2^(t+1)), r < 2^t, t <= 2
    if (r == 0) return w;
    const double sg = inv ? -1.0 : 1.0;
    if (t == 1 || r == 2) return make_double2(sg * w.y, -sg * w.x);            // * (-+i)
    const double c = 0.70710678118654752440;                                  // r = 1 or 3, t = 2
    const double2 z = r == 1 ? make_double2(c, -sg * c) : make_double2(-c, -sg * c);
    return cmul(w, z);
}

template <int R, bool DIT>
__device__ __forceinline__ void fft_pass(double2* buf, int M, int s, int logMmax, const double2* __restrict__ tw,
                                         bool inv) {
    constexpr int G = 1 << R;
    const int h = 1 << s;
    const int ngroups = M >> R;
    for (int q = threadIdx.x; q < ngroups; q += blockDim.x) {
        const int j = q & (h - 1);
        const int base = ((q >> s) << (s + R)) + j;
        double2 x[G];
#pragma unroll
        for (int c = 0; c < G; ++c) x[c] = buf[pidx(base + c * h)];
        double2 wb[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            wb[t] = tw[j << (logMmax - s - t - 1)];
            if (inv) wb[t].y = -wb[t].y;
        }
#pragma unroll
        for (int tt = 0; tt < R; ++tt) {
            const int t = DIT ? tt : R - 1 - tt;
            const int half = 1 << t;
#pragma unroll
            for (int c = 0; c < G; ++c) {
                if (c & half) continue;
                const double2 w = root_mul(wb[t], c & (half - 1), t, inv);
                const double2 a = x[c], b = x[c + half];
                if (DIT) {
                    const double2 bw = cmul(b, w);
                    x[c] = make_double2(a.x + bw.x, a.y + bw.y);
                    x[c + half] = make_double2(a.x - bw.x, a.y - bw.y);
                } else {
                    x[c] = make_double2(a.x + b.x, a.y + b.y);
                    x[c + half] = cmul(make_double2(a.x - b.x, a.y - b.y), w);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < G; ++c) buf[pidx(base + c * h)] = x[c];
    }
    __syncthreads();
}

// decimation in time: bit-reversed input, natural output
__device__ void fft_dit(double2* buf, int M, int logM, int logMmax, const double2* __restrict__ tw, bool inv) {
    int s = 0;
    for (; s + 3 <= logM; s += 3) fft_pass<3, true>(buf, M, s, logMmax, tw, inv);
    if (logM - s == 2) fft_pass<2, true>(buf, M, s, logMmax, tw, inv);
    else if (logM - s == 1) fft_pass<1, true>(buf, M, s, logMmax, tw, inv);
}

// decimation in frequency: natural input, bit-reversed output
__device__ void fft_dif(double2* buf, int M, int logM, int logMmax, const double2* __restrict__ tw, bool inv) {
    int top = logM;
    for (; top >= 3; top -= 3) fft_pass<3, false>(buf, M, top - 3, logMmax, tw, inv);
    if (top == 2) fft_pass<2, false>(buf, M, 0, logMmax, tw, inv);
    else if (top == 1) fft_pass<1, false>(buf, M, 0, logMmax, tw, inv);
}

// Forward DFT core.  On entry buf[brev(j)] holds a_j (times chirp_j for
// Bluestein, zeros at brev(j) for j >= n).  On exit the transform value X_k
// is at buf[out_pos(k)] (times chirp_k for Bluestein).
__device__ void dft_core(double2* buf, const FftLenDev& L, const RingArgs& A) {
    if (!L.bluestein) {
        fft_dit(buf, L.M, L.logM, A.logMmax, A.tw, false);
    } else {
        fft_dit(buf, L.M, L.logM, A.logMmax, A.tw, false);
        const double2* bh = A.bhat + L.bhat_off;
        for (int q = threadIdx.x; q < L.M; q += blockDim.x) buf[pidx(q)] = cmul(buf[pidx(q)], bh[q]);
        __syncthreads();
        fft_dif(buf, L.M, L.logM, A.logMmax, A.tw, true);
    }
}

// Inverse-direction core for the synthesis: on entry buf holds conj(c)
// placed for the transform; on exit x_j = conj(value at brev(j)) (times
// chirp for Bluestein).  For powers of two the input is in natural order.
__device__ void idft_core(double2* buf, const FftLenDev& L, const RingArgs& A) {
    if (!L.bluestein) {
        fft_dif(buf, L.M, L.logM, A.logMmax, A.tw, false);
    } else {
        dft_core(buf, L, A);
    }
}

template <int MODE>
__global__ __launch_bounds__(512) void ring_kernel(RingArgs A, const double* __restrict__ map_in,
                                                   double* __restrict__ map_out, const double* __restrict__ Kp,
                                                   const double* __restrict__ bp, double2* __restrict__ phase) {
    extern __shared__ double2 buf[];
    const int p = blockIdx.x;
    const int rhs = blockIdx.y;
    const RingPairDev P = A.pairs[p];
    const FftLenDev L = A.lens[P.len_idx];
    const int n = P.nphi, M = L.M, logM = L.logM;
    const int nt = blockDim.x, tid = threadIdx.x;
    const int mmax = A.mmax;
    const int64_t fstride = (int64_t)A.npairs * (mmax + 1) * 2;
    const bool synth = (MODE == RING_SYNTH || MODE == RING_ITERATE);
    const bool anal = (MODE == RING_ANALYSIS || MODE == RING_ITERATE);
    const double2* chirp = L.bluestein ? A.chirp + L.chirp_off : nullptr;

    for (int f = 0; f < 3; ++f) {
        double2* ph = phase + (((int64_t)rhs * 3 + f) * A.npairs + p) * (mmax + 1) * 2;
        const int64_t moff = ((int64_t)rhs * 3 + f) * A.npix;
        if (synth) {
            // fold into n bins, place conj(C_N + i C_S) for the inverse transform
            for (int k = tid; k < M; k += nt) {
                double2 v = make_double2(0.0, 0.0);
                const int j = L.bluestein ? (int)brev(k, logM) : k;   // logical index of slot k
                if (j < n) {
                    double2 cn = make_double2(0.0, 0.0), cs = make_double2(0.0, 0.0);
                    const int mstart = j - n * ((j + mmax) / n);
                    for (int m = mstart; m <= mmax; m += n) {
                        const int a = m < 0 ? -m : m;
                        double2 fn = ph[2 * a], fs = ph[2 * a + 1];
                        if (m < 0) { fn.y = -fn.y; fs.y = -fs.y; }
                        const double2 rot = phase_rot(m, P.phi0_den);
                        const double2 tn = cmul(fn, rot), ts = cmul(fs, rot);
                        cn.x += tn.x; cn.y += tn.y;
                        cs.x += ts.x; cs.y += ts.y;
                    }
                    // z = C_N + i C_S ; store conj(z)
                    v = make_double2(cn.x - cs.y, -(cn.y + cs.x));
                    if (L.bluestein) v = cmul(v, chirp[j]);
                }
                buf[pidx(k)] = v;
            }
            __syncthreads();
            idft_core(buf, L, A);
            // now x_j (packed N + i S) = conj(buf[brev(j)] * chirp_j)
            for (int j = tid; j < n; j += nt) {
                const int q = (int)brev(j, logM);
                double2 y = buf[pidx(q)];
                if (L.bluestein) y = cmul(y, chirp[j]);
                const double xn = y.x, xs = -y.y;
                if (MODE == RING_SYNTH) {
                    map_out[moff + P.off_n + j] = xn;
                    if (P.has_s) map_out[moff + P.off_s + j] = xs;
                } else {
                    const int64_t kn = (int64_t)f * A.npix + P.off_n + j;
                    double tn = Kp[kn] * xn + bp[moff + P.off_n + j];
                    double ts = 0.0;
                    if (P.has_s) {
                        const int64_t ks = (int64_t)f * A.npix + P.off_s + j;
                        ts = Kp[ks] * xs + bp[moff + P.off_s + j];
                    }
                    if (map_out) {
                        map_out[moff + P.off_n + j] = tn;
                        if (P.has_s) map_out[moff + P.off_s + j] = ts;
                    }
                    double2 a = make_double2(tn, ts);
                    if (L.bluestein) a = cmul(a, chirp[j]);
                    buf[pidx(q)] = a;
                }
            }
            if (MODE == RING_ITERATE && L.bluestein) {
                for (int j = n + tid; j < M; j += nt) buf[pidx((int)brev(j, logM))] = make_double2(0.0, 0.0);
            }
            __syncthreads();
        }
        if (MODE == RING_ANALYSIS) {
            for (int q = tid; q < M; q += nt) {
                const int j = (int)brev(q, logM);
                double2 a = make_double2(0.0, 0.0);
                if (j < n) {
                    a.x = map_in[moff + P.off_n + j];
                    a.y = P.has_s ? map_in[moff + P.off_s + j] : 0.0;
                    if (L.bluestein) a = cmul(a, chirp[j]);
                }
                buf[pidx(q)] = a;
            }
            __syncthreads();
        }
        if (anal) {
            dft_core(buf, L, A);
            for (int m = tid; m <= mmax; m += nt) {
                const int k = m % n;
                const int k2 = (n - k) % n;
                const int q1 = L.bluestein ? (int)brev(k, logM) : k;
                const int q2 = L.bluestein ? (int)brev(k2, logM) : k2;
                double2 z1 = buf[pidx(q1)], z2 = buf[pidx(q2)];
                if (L.bluestein) { z1 = cmul(z1, chirp[k]); z2 = cmul(z2, chirp[k2]); }
                // X_N = (Z_k + conj Z_{-k}) / 2,  X_S = (Z_k - conj Z_{-k}) / (2i)
                const double2 xn = make_double2(0.5 * (z1.x + z2.x), 0.5 * (z1.y - z2.y));
                const double2 xs = make_double2(0.5 * (z1.y + z2.y), -0.5 * (z1.x - z2.x));
                const double2 rot = conjd(phase_rot(m, P.phi0_den));
                ph[2 * m] = cmul(xn, rot);
                ph[2 * m + 1] = P.has_s ? cmul(xs, rot) : make_double2(0.0, 0.0);
            }
            __syncthreads();
        }
    }
}

}  // namespace

hipError_t launch_ring(dm_plan* p, int mode, int nrhs, const double* map_in, double* map_out, const double* K,
                       const double* b, double* phase, hipStream_t s) {
    RingArgs A;
    A.npairs = p->npairs;
    A.mmax = p->mmax;
    int lm = 0;
    while ((1 << lm) < p->fft.Mmax) ++lm;
    A.logMmax = lm;
    A.npix = p->npix;
    A.pairs = p->d_pairs;
    A.lens = p->d_fftlen;
    A.chirp = reinterpret_cast<const double2*>(p->d_chirp);
    A.bhat = reinterpret_cast<const double2*>(p->d_bhat);
    A.tw = reinterpret_cast<const double2*>(p->d_tw);
    dim3 grid(p->npairs, nrhs);
    dim3 block(p->fft_threads);
    const size_t lds = p->fft_lds_bytes;
    double2* ph = reinterpret_cast<double2*>(phase);
    switch (mode) {
        case RING_ANALYSIS:
            hipLaunchKernelGGL(ring_kernel<RING_ANALYSIS>, grid, block, lds, s, A, map_in, map_out, K, b, ph);
            break;
        case RING_SYNTH:
            hipLaunchKernelGGL(ring_kernel<RING_SYNTH>, grid, block, lds, s, A, map_in, map_out, K, b, ph);
            break;
        default:
            hipLaunchKernelGGL(ring_kernel<RING_ITERATE>, grid, block, lds, s, A, map_in, map_out, K, b, ph);
            break;
    }
    return hipGetLastError();
}

hipError_t ring_set_lds_limit(size_t bytes) {
    hipError_t e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ring_kernel<RING_ANALYSIS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ring_kernel<RING_SYNTH>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&ring_kernel<RING_ITERATE>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace dmwf
