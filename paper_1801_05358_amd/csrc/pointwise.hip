// Per-pixel setup of the messenger update (eq 4 and Algorithm 1's
// initialisation), per-pixel pieces of the diagnostics (eq 3 chi^2 and the
// residual of Appendix C), and deterministic fixed-order reductions.
//
// Observation is per component: bit 0 of obs[p] = I observed, bit 1 = Q
// and U observed (distinct temperature and polarization masks, Appendix
// B).  With P_p the inverse noise covariance on the observed components
// (zero rows and columns elsewhere):
//
//   alpha_p = 1 / lambda_max(P_p)  (the smallest eigenvalue of N_p when
//             every component is observed),
//   tau     = min over pixels with an observed component of alpha_p w_p,
//   T_p     = tau / w_p,   K = 1 - T_p P_p,   b = T_p P_p d0,
//   d0      = d on observed components, 0 elsewhere.
//
// Diagonal noise (II, QQ, UU) keeps P, K and T P as [3][npix].  The
// correlated 3x3 block of eq 11 keeps P and T P as symmetric 3x3 per pixel,
// [6][npix] in the order (II, IQ, IU, QQ, QU, UU); there P_p is the block of
// N_p^-1 on the observed components, i.e. Appendix B's N = Sigma C Sigma
// with Sigma^-1 = 0 on the unobserved ones.
#include "dmwf_internal.h"

namespace dmwf {

namespace {

constexpr int kBlk = 256;

__device__ __forceinline__ double block_min(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) sh[tid] = fmin(sh[tid], sh[tid + o]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) sh[tid] += sh[tid + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ int comp_bit(int f) { return f == 0 ? 1 : 2; }

// one block per ring
__global__ void tau_kernel(int64_t npix, const int64_t* __restrict__ roff, const int* __restrict__ rn,
                           const double* __restrict__ rw, const double* __restrict__ ncov,
                           const uint8_t* __restrict__ obs, double* __restrict__ ring_min) {
    __shared__ double sh[kBlk];
    const int r = blockIdx.x;
    const int64_t o = roff[r];
    const int n = rn[r];
    const double w = rw[r];
    double v = INFINITY;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int64_t q = o + j;
        const int m = obs[q];
        double a = INFINITY;
        if (m & 1) a = ncov[q];
        if (m & 2) a = fmin(a, fmin(ncov[npix + q], ncov[2 * npix + q]));
        v = fmin(v, a * w);
    }
    v = block_min(v, sh);
    if (threadIdx.x == 0) ring_min[r] = v;
}

// grid (nrings, 3)
__global__ void noise_kernel(int64_t npix, const int64_t* __restrict__ roff, const int* __restrict__ rn,
                             const double* __restrict__ rw, const double* __restrict__ ncov,
                             const uint8_t* __restrict__ obs, double tau, double* __restrict__ K,
                             double* __restrict__ tn, double* __restrict__ ninv) {
    const int r = blockIdx.x, f = blockIdx.y;
    const int64_t o = roff[r];
    const int n = rn[r];
    const double T = tau / rw[r];
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int64_t q = (int64_t)f * npix + o + j;
        const bool ok = (obs[o + j] & comp_bit(f)) != 0;
        const double ni = ok ? 1.0 / ncov[q] : 0.0;
        ninv[q] = ni;
        tn[q] = T * ni;
        K[q] = 1.0 - T * ni;
    }
}

__global__ void data_kernel(int64_t npix, int64_t total, const double* __restrict__ d,
                            const uint8_t* __restrict__ obs, const double* __restrict__ tn,
                            double* __restrict__ d0, double* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = i % (3 * npix);
        const int64_t pix = q % npix;
        const int f = (int)(q / npix);
        const double v = (obs[pix] & comp_bit(f)) ? d[i] : 0.0;
        d0[i] = v;
        b[i] = tn[q] * v;
    }
}

// ---------------------------------------------------------------------------
// correlated 3x3 pixel noise
// ---------------------------------------------------------------------------
// symmetric [[a b c] [b d e] [c e f]]
struct Sym3 {
    double a, b, c, d, e, f;
};

__device__ __forceinline__ Sym3 load_sym(const double* __restrict__ m, int64_t npix, int64_t q) {
    return Sym3{m[q], m[npix + q], m[2 * npix + q], m[3 * npix + q], m[4 * npix + q], m[5 * npix + q]};
}

__device__ __forceinline__ void store_sym(double* __restrict__ m, int64_t npix, int64_t q, const Sym3& s) {
    m[q] = s.a;
    m[npix + q] = s.b;
    m[2 * npix + q] = s.c;
    m[3 * npix + q] = s.d;
    m[4 * npix + q] = s.e;
    m[5 * npix + q] = s.f;
}

// inverse by cofactors (N symmetric positive definite, checked on the host)
__device__ __forceinline__ Sym3 sym_inverse(const Sym3& n) {
    const double c00 = n.d * n.f - n.e * n.e;
    const double c01 = n.c * n.e - n.b * n.f;
    const double c02 = n.b * n.e - n.c * n.d;
    const double c11 = n.a * n.f - n.c * n.c;
    const double c12 = n.b * n.c - n.a * n.e;
    const double c22 = n.a * n.d - n.b * n.b;
    const double id = 1.0 / (n.a * c00 + n.b * c01 + n.c * c02);
    return Sym3{c00 * id, c01 * id, c02 * id, c11 * id, c12 * id, c22 * id};
}

// largest eigenvalue of a symmetric 3x3: with q = tr/3 and p the scale of
// M - q 1, the eigenvalues are q + 2 p cos(phi + 2 pi k / 3) with
// cos(3 phi) = det((M - q 1) / p) / 2 (Smith 1961); k = 0 is the largest
__device__ __forceinline__ double sym_lambda_max(const Sym3& m) {
    const double q = (m.a + m.d + m.f) / 3.0;
    const double a0 = m.a - q, d0 = m.d - q, f0 = m.f - q;
    const double off = m.b * m.b + m.c * m.c + m.e * m.e;
    const double p2 = a0 * a0 + d0 * d0 + f0 * f0 + 2.0 * off;
    if (!(p2 > 0.0)) return q;
    const double p = sqrt(p2 / 6.0), ip = 1.0 / p;
    const double ba = a0 * ip, bb = m.b * ip, bc = m.c * ip, bd = d0 * ip, be = m.e * ip, bf = f0 * ip;
    const double det = ba * (bd * bf - be * be) - bb * (bb * bf - be * bc) + bc * (bb * be - bd * bc);
    const double r = fmin(1.0, fmax(-1.0, 0.5 * det));
    return q + 2.0 * p * cos(acos(r) / 3.0);
}

__device__ __forceinline__ void sym_apply(const Sym3& m, double x0, double x1, double x2, double& y0, double& y1,
                                          double& y2) {
    y0 = m.a * x0 + m.b * x1 + m.c * x2;
    y1 = m.b * x0 + m.d * x1 + m.e * x2;
    y2 = m.c * x0 + m.e * x1 + m.f * x2;
}

// one block per ring: P_p into ninv6, and the ring's min of alpha_p w_p
__global__ void tau6_kernel(int64_t npix, const int64_t* __restrict__ roff, const int* __restrict__ rn,
                            const double* __restrict__ rw, const double* __restrict__ ncov6,
                            const uint8_t* __restrict__ obs, double* __restrict__ ninv6,
                            double* __restrict__ ring_min) {
    __shared__ double sh[kBlk];
    const int r = blockIdx.x;
    const int64_t o = roff[r];
    const int n = rn[r];
    const double w = rw[r];
    double v = INFINITY;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int64_t q = o + j;
        const int m = obs[q];
        Sym3 P{0, 0, 0, 0, 0, 0};
        if (m) {
            P = sym_inverse(load_sym(ncov6, npix, q));
            if (!(m & 1)) P.a = P.b = P.c = 0.0;
            if (!(m & 2)) P.b = P.c = P.d = P.e = P.f = 0.0;
            v = fmin(v, w / sym_lambda_max(P));
        }
        store_sym(ninv6, npix, q, P);
    }
    v = block_min(v, sh);
    if (threadIdx.x == 0) ring_min[r] = v;
}

// grid (nrings): T P
__global__ void noise6_kernel(int64_t npix, const int64_t* __restrict__ roff, const int* __restrict__ rn,
                              const double* __restrict__ rw, const double* __restrict__ ninv6, double tau,
                              double* __restrict__ tn6) {
    const int r = blockIdx.x;
    const int64_t o = roff[r];
    const int n = rn[r];
    const double T = tau / rw[r];
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        for (int k = 0; k < 6; ++k) tn6[k * npix + o + j] = T * ninv6[k * npix + o + j];
}

// over (rhs, pixel): d0 = d on observed components, b = T P d0
__global__ void data6_kernel(int64_t npix, int64_t total, const double* __restrict__ d,
                             const uint8_t* __restrict__ obs, const double* __restrict__ tn6,
                             double* __restrict__ d0, double* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rhs = i / npix, q = i % npix;
        const int64_t base = rhs * 3 * npix + q;
        const int m = obs[q];
        const double x0 = (m & 1) ? d[base] : 0.0;
        const double x1 = (m & 2) ? d[base + npix] : 0.0;
        const double x2 = (m & 2) ? d[base + 2 * npix] : 0.0;
        double y0, y1, y2;
        sym_apply(load_sym(tn6, npix, q), x0, x1, x2, y0, y1, y2);
        d0[base] = x0;
        d0[base + npix] = x1;
        d0[base + 2 * npix] = x2;
        b[base] = y0;
        b[base + npix] = y1;
        b[base + 2 * npix] = y2;
    }
}

// over pixels, in place: ux <- t = ux - T P ux + b (eq 9 with the 3x3 K)
// for every RHS; t_out (nullable) receives a copy.  T P is read once per
// pixel for all RHS.
__global__ void update6_kernel(int64_t npix, int nrhs, double* __restrict__ ux, const double* __restrict__ tn6,
                               const double* __restrict__ b, double* __restrict__ t_out) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < npix;
         q += (int64_t)gridDim.x * blockDim.x) {
        const Sym3 M = load_sym(tn6, npix, q);
        for (int rhs = 0; rhs < nrhs; ++rhs) {
            const int64_t base = (int64_t)rhs * 3 * npix + q;
            const double x0 = ux[base], x1 = ux[base + npix], x2 = ux[base + 2 * npix];
            double y0, y1, y2;
            sym_apply(M, x0, x1, x2, y0, y1, y2);
            const double t0 = (x0 - y0) + b[base];
            const double t1 = (x1 - y1) + b[base + npix];
            const double t2 = (x2 - y2) + b[base + 2 * npix];
            ux[base] = t0;
            ux[base + npix] = t1;
            ux[base + 2 * npix] = t2;
            if (t_out) {
                t_out[base] = t0;
                t_out[base + npix] = t1;
                t_out[base + 2 * npix] = t2;
            }
        }
    }
}

// grid (nrings, nrhs): ux <- P (ux - d0), b <- P d0 (b nullable),
// chi_parts[rhs][ring] = sum (d0 - ux)^T P (d0 - ux)
__global__ void resid6_kernel(int64_t npix, int nrings, const int64_t* __restrict__ roff,
                              const int* __restrict__ rn, const double* __restrict__ ninv6, double* __restrict__ ux,
                              const double* __restrict__ d0, double* __restrict__ b, double* __restrict__ chi) {
    __shared__ double sh[kBlk];
    const int r = blockIdx.x, rhs = blockIdx.y;
    const int64_t o = roff[r];
    const int n = rn[r];
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int64_t q = o + j;
        const int64_t base = (int64_t)rhs * 3 * npix + q;
        const Sym3 P = load_sym(ninv6, npix, q);
        const double e0 = ux[base] - d0[base], e1 = ux[base + npix] - d0[base + npix];
        const double e2 = ux[base + 2 * npix] - d0[base + 2 * npix];
        double y0, y1, y2, z0, z1, z2;
        sym_apply(P, e0, e1, e2, y0, y1, y2);
        sym_apply(P, d0[base], d0[base + npix], d0[base + 2 * npix], z0, z1, z2);
        acc += e0 * y0 + e1 * y1 + e2 * y2;
        ux[base] = y0;
        ux[base + npix] = y1;
        ux[base + 2 * npix] = y2;
        if (b) {
            b[base] = z0;
            b[base + npix] = z1;
            b[base + 2 * npix] = z2;
        }
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) chi[(int64_t)rhs * nrings + r] = acc;
}

// grid (nrings, nrhs): ux <- N^-1 (ux - d0), b <- N^-1 d0 (b nullable),
// chi_parts[rhs][ring] = sum (d0 - ux)^2 N^-1
__global__ void resid_kernel(int64_t npix, int nrings, const int64_t* __restrict__ roff, const int* __restrict__ rn,
                             const double* __restrict__ ninv, double* __restrict__ ux,
                             const double* __restrict__ d0, double* __restrict__ b, double* __restrict__ chi) {
    __shared__ double sh[kBlk];
    const int r = blockIdx.x, rhs = blockIdx.y;
    const int64_t o = roff[r];
    const int n = rn[r];
    double acc = 0.0;
    for (int f = 0; f < 3; ++f) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const int64_t q = (int64_t)f * npix + o + j;
            const int64_t i = (int64_t)rhs * 3 * npix + q;
            const double ni = ninv[q];
            const double res = ux[i] - d0[i];
            acc += res * res * ni;
            ux[i] = ni * res;
            if (b) b[i] = ni * d0[i];
        }
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) chi[(int64_t)rhs * nrings + r] = acc;
}

// grid (lblocks, mmax+1, nrhs); per (l, m) with weight 1 (m = 0) or 2:
//   q0 = |u - uprev|^2, q1 = |u|^2, q2 = |S^+1/2 u + S^1/2 r1|^2,
//   q3 = |S^1/2 y1|^2, q4 = u^T S^+ u
__global__ void norm_kernel(int lmax, int64_t nalm, const double2* __restrict__ u, const double2* __restrict__ up,
                            const double2* __restrict__ r1, const double2* __restrict__ y1,
                            const double* __restrict__ mats, double* __restrict__ parts) {
    __shared__ double sh[kBlk];
    const int m = blockIdx.y, rhs = blockIdx.z;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    double q[kNormQ] = {0, 0, 0, 0, 0};
    if (l <= lmax) {
        const int64_t idx = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
        const double wt = m == 0 ? 1.0 : 2.0;
        const double* sq = mats;                         // S^1/2
        const double* isq = mats + 4 * (lmax + 1);       // S^+1/2
        const double* inv = mats + 8 * (lmax + 1);       // S^+
        double2 uu[3], du[3], rr[3], yy[3];
        for (int f = 0; f < 3; ++f) {
            const int64_t k = ((int64_t)rhs * 3 + f) * nalm + idx;
            uu[f] = u[k];
            du[f] = up ? make_double2(u[k].x - up[k].x, u[k].y - up[k].y) : make_double2(0.0, 0.0);
            rr[f] = r1 ? r1[k] : make_double2(0.0, 0.0);
            yy[f] = y1 ? y1[k] : make_double2(0.0, 0.0);
        }
        auto apply = [&](const double* M, const double2* a, double2* o) {
            const double tt = M[4 * l], te = M[4 * l + 1], ee = M[4 * l + 2], bb = M[4 * l + 3];
            o[0] = make_double2(tt * a[0].x + te * a[1].x, tt * a[0].y + te * a[1].y);
            o[1] = make_double2(te * a[0].x + ee * a[1].x, te * a[0].y + ee * a[1].y);
            o[2] = make_double2(bb * a[2].x, bb * a[2].y);
        };
        double2 t1[3], t2[3], t3[3], t4[3];
        apply(isq, uu, t1);
        apply(sq, rr, t2);
        apply(sq, yy, t3);
        apply(inv, uu, t4);
        for (int f = 0; f < 3; ++f) {
            q[0] += wt * (du[f].x * du[f].x + du[f].y * du[f].y);
            q[1] += wt * (uu[f].x * uu[f].x + uu[f].y * uu[f].y);
            const double rx = t1[f].x + t2[f].x, ry = t1[f].y + t2[f].y;
            q[2] += wt * (rx * rx + ry * ry);
            q[3] += wt * (t3[f].x * t3[f].x + t3[f].y * t3[f].y);
            q[4] += wt * (uu[f].x * t4[f].x + uu[f].y * t4[f].y);
        }
    }
    const int64_t blk = ((int64_t)rhs * gridDim.y + m) * gridDim.x + blockIdx.x;
    for (int k = 0; k < kNormQ; ++k) {
        const double s = block_sum(q[k], sh);
        if (threadIdx.x == 0) parts[blk * kNormQ + k] = s;
    }
}

// Refinement residual (Appendix A) per (l, m), grid (lblocks, mmax+1, nrhs):
//   e <- Pi e + S^+ s   in place, with e = Y^T P (Y s - d0) on entry, so
//   that e = -r, r the residual of the Wiener filter equation on the range
//   of S;  Pi = S^+1/2 S^1/2 the projector onto that range.
//   parts[blk][0] = sum |e|^2,  parts[blk][1] = sum |Pi y|^2 (y nullable),
//   with weight 1 (m = 0) or 2 (m > 0).
__global__ void refine_resid_kernel(int lmax, int64_t nalm, double2* __restrict__ e, const double2* __restrict__ u,
                                    const double2* __restrict__ y, const double* __restrict__ mats,
                                    double* __restrict__ parts) {
    __shared__ double sh[kBlk];
    const int m = blockIdx.y, rhs = blockIdx.z;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    double q0 = 0.0, q1 = 0.0;
    if (l <= lmax) {
        const int64_t idx = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
        const double wt = m == 0 ? 1.0 : 2.0;
        const double* sq = mats;                         // S^1/2
        const double* isq = mats + 4 * (lmax + 1);       // S^+1/2
        const double* inv = mats + 8 * (lmax + 1);       // S^+
        // Pi = S^+1/2 S^1/2 (both functions of S_l, so the product is symmetric)
        const double at = isq[4 * l], ab = isq[4 * l + 1], ae = isq[4 * l + 2];
        const double bt = sq[4 * l], bb = sq[4 * l + 1], be = sq[4 * l + 2];
        const double ptt = at * bt + ab * bb, pte = at * bb + ab * be, pee = ab * bb + ae * be;
        const double pbb = isq[4 * l + 3] * sq[4 * l + 3];
        const double itt = inv[4 * l], ite = inv[4 * l + 1], iee = inv[4 * l + 2], ibb = inv[4 * l + 3];
        double2 ee[3], uu[3], yy[3];
        for (int f = 0; f < 3; ++f) {
            const int64_t k = ((int64_t)rhs * 3 + f) * nalm + idx;
            ee[f] = e[k];
            uu[f] = u[k];
            yy[f] = y ? y[k] : make_double2(0.0, 0.0);
        }
        double2 o[3], py[3];
        o[0] = make_double2(ptt * ee[0].x + pte * ee[1].x + itt * uu[0].x + ite * uu[1].x,
                            ptt * ee[0].y + pte * ee[1].y + itt * uu[0].y + ite * uu[1].y);
        o[1] = make_double2(pte * ee[0].x + pee * ee[1].x + ite * uu[0].x + iee * uu[1].x,
                            pte * ee[0].y + pee * ee[1].y + ite * uu[0].y + iee * uu[1].y);
        o[2] = make_double2(pbb * ee[2].x + ibb * uu[2].x, pbb * ee[2].y + ibb * uu[2].y);
        py[0] = make_double2(ptt * yy[0].x + pte * yy[1].x, ptt * yy[0].y + pte * yy[1].y);
        py[1] = make_double2(pte * yy[0].x + pee * yy[1].x, pte * yy[0].y + pee * yy[1].y);
        py[2] = make_double2(pbb * yy[2].x, pbb * yy[2].y);
        for (int f = 0; f < 3; ++f) {
            e[((int64_t)rhs * 3 + f) * nalm + idx] = o[f];
            q0 += wt * (o[f].x * o[f].x + o[f].y * o[f].y);
            q1 += wt * (py[f].x * py[f].x + py[f].y * py[f].y);
        }
    }
    const int64_t blk = ((int64_t)rhs * gridDim.y + m) * gridDim.x + blockIdx.x;
    const double s0 = block_sum(q0, sh);
    if (threadIdx.x == 0) parts[blk * 2] = s0;
    const double s1 = block_sum(q1, sh);
    if (threadIdx.x == 0) parts[blk * 2 + 1] = s1;
}

__global__ void scale_kernel(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i];
}

template <typename A, typename B>
__global__ void convert_kernel(B* __restrict__ y, const A* __restrict__ x, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (B)x[i];
}

__global__ void count_nonfinite_kernel(const double* __restrict__ x, int64_t n, int* count) {
    int c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) ++c;
    if (c) atomicAdd(count, c);
}

__global__ void axpby_kernel(double* __restrict__ y, const double* __restrict__ x, double a, double c, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + c * y[i];
}

// SplitMix64's output function (Steele, Lea and Flood 2014), as the
// per-element mix of the buffer fingerprints
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename E>
__global__ void hash_kernel(const E* __restrict__ x, int64_t n, unsigned long long* __restrict__ acc) {
    __shared__ unsigned long long sh[kBlk];
    unsigned long long h = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t v;
        if constexpr (sizeof(E) == 8) {
            v = reinterpret_cast<const uint64_t*>(x)[i];
        } else {
            v = (uint64_t)x[i];
        }
        h += mix64(v + (uint64_t)i * 0x9E3779B97F4A7C15ull);
    }
    const int tid = threadIdx.x;
    sh[tid] = h;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) sh[tid] += sh[tid + o];
        __syncthreads();
    }
    if (tid == 0) atomicAdd(acc, sh[0]);
}

int grid_for(int64_t n) {
    int64_t g = (n + kBlk - 1) / kBlk;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_tau_parts(dm_plan* p, const double* ncov, double* ring_min, hipStream_t s) {
    if (p->ncov_layout == DM_NCOV_SYM6)
        hipLaunchKernelGGL(tau6_kernel, dim3(p->nrings), dim3(kBlk), 0, s, p->npix, p->d_ring_off, p->d_ring_n,
                           p->d_ring_w, ncov, p->d_obs, p->d_ninv6, ring_min);
    else
        hipLaunchKernelGGL(tau_kernel, dim3(p->nrings), dim3(kBlk), 0, s, p->npix, p->d_ring_off, p->d_ring_n,
                           p->d_ring_w, ncov, p->d_obs, ring_min);
    return hipGetLastError();
}

hipError_t launch_noise_setup(dm_plan* p, const double* ncov, double tau, hipStream_t s) {
    if (p->ncov_layout == DM_NCOV_SYM6)
        hipLaunchKernelGGL(noise6_kernel, dim3(p->nrings), dim3(kBlk), 0, s, p->npix, p->d_ring_off, p->d_ring_n,
                           p->d_ring_w, p->d_ninv6, tau, p->d_tn6);
    else
        hipLaunchKernelGGL(noise_kernel, dim3(p->nrings, 3), dim3(kBlk), 0, s, p->npix, p->d_ring_off, p->d_ring_n,
                           p->d_ring_w, ncov, p->d_obs, tau, p->d_K, p->d_tn, p->d_ninv);
    return hipGetLastError();
}

hipError_t launch_data_setup(dm_plan* p, int nrhs, const double* d, double* d0, double* b, hipStream_t s) {
    if (p->ncov_layout == DM_NCOV_SYM6) {
        const int64_t total = (int64_t)nrhs * p->npix;
        hipLaunchKernelGGL(data6_kernel, dim3(grid_for(total)), dim3(kBlk), 0, s, p->npix, total, d, p->d_obs,
                           p->d_tn6, d0, b);
    } else {
        const int64_t total = (int64_t)nrhs * 3 * p->npix;
        hipLaunchKernelGGL(data_kernel, dim3(grid_for(total)), dim3(kBlk), 0, s, p->npix, total, d, p->d_obs,
                           p->d_tn, d0, b);
    }
    return hipGetLastError();
}

hipError_t launch_update6(dm_plan* p, int nrhs, double* ux, const double* b, double* t_out, hipStream_t s) {
    hipLaunchKernelGGL(update6_kernel, dim3(grid_for(p->npix)), dim3(kBlk), 0, s, p->npix, nrhs, ux, p->d_tn6, b,
                       t_out);
    return hipGetLastError();
}

hipError_t launch_residual_maps(dm_plan* p, int nrhs, double* ux, const double* d0, double* b, double* chi_parts,
                                hipStream_t s) {
    if (p->ncov_layout == DM_NCOV_SYM6)
        hipLaunchKernelGGL(resid6_kernel, dim3(p->nrings, nrhs), dim3(kBlk), 0, s, p->npix, p->nrings,
                           p->d_ring_off, p->d_ring_n, p->d_ninv6, ux, d0, b, chi_parts);
    else
        hipLaunchKernelGGL(resid_kernel, dim3(p->nrings, nrhs), dim3(kBlk), 0, s, p->npix, p->nrings,
                           p->d_ring_off, p->d_ring_n, p->d_ninv, ux, d0, b, chi_parts);
    return hipGetLastError();
}

uint64_t hash_mix(uint64_t x) { return mix64(x); }

hipError_t launch_hash(const void* buf, int64_t n, int elem_bytes, uint64_t* acc, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    unsigned long long* a = reinterpret_cast<unsigned long long*>(acc);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(hash_kernel<uint64_t>, dim3(grid_for(n)), dim3(kBlk), 0, s,
                           reinterpret_cast<const uint64_t*>(buf), n, a);
    else
        hipLaunchKernelGGL(hash_kernel<uint8_t>, dim3(grid_for(n)), dim3(kBlk), 0, s,
                           reinterpret_cast<const uint8_t*>(buf), n, a);
    return hipGetLastError();
}

int alm_norm_blocks(dm_plan* p) { return ((p->lmax + 1) + kBlk - 1) / kBlk * (p->mmax + 1); }

hipError_t launch_alm_norms(dm_plan* p, int nrhs, const double* u, const double* uprev, const double* r1,
                            const double* y1, const double* mats, double* parts, hipStream_t s) {
    dim3 grid(((p->lmax + 1) + kBlk - 1) / kBlk, p->mmax + 1, nrhs);
    hipLaunchKernelGGL(norm_kernel, grid, dim3(kBlk), 0, s, p->lmax, p->nalm, reinterpret_cast<const double2*>(u),
                       reinterpret_cast<const double2*>(uprev), reinterpret_cast<const double2*>(r1),
                       reinterpret_cast<const double2*>(y1), mats, parts);
    return hipGetLastError();
}

hipError_t launch_refine_residual(dm_plan* p, int nrhs, double* e, const double* u, const double* y, double* parts,
                                  hipStream_t s) {
    dim3 grid(((p->lmax + 1) + kBlk - 1) / kBlk, p->mmax + 1, nrhs);
    hipLaunchKernelGGL(refine_resid_kernel, grid, dim3(kBlk), 0, s, p->lmax, p->nalm, reinterpret_cast<double2*>(e),
                       reinterpret_cast<const double2*>(u), reinterpret_cast<const double2*>(y), p->d_mats, parts);
    return hipGetLastError();
}

hipError_t launch_scale(double* y, const double* x, double a, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(kBlk), 0, s, y, x, a, n);
    return hipGetLastError();
}

hipError_t launch_widen(double* y, const float* x, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(grid_for(n)), dim3(kBlk), 0, s, y, x, n);
    return hipGetLastError();
}

hipError_t launch_narrow(float* y, const double* x, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(grid_for(n)), dim3(kBlk), 0, s, y, x, n);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const double* x, int64_t n, int* count, hipStream_t s) {
    hipLaunchKernelGGL(count_nonfinite_kernel, dim3(grid_for(n)), dim3(kBlk), 0, s, x, n, count);
    return hipGetLastError();
}

hipError_t launch_axpby(double* y, const double* x, double a, double c, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(kBlk), 0, s, y, x, a, c, n);
    return hipGetLastError();
}

}  // namespace dmwf
