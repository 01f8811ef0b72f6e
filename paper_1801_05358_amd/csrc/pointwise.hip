// Per-pixel setup of the messenger update (eq 4 and Algorithm 1's
// initialisation), per-pixel pieces of the diagnostics (eq 3 chi^2 and the
// residual of Appendix C), and deterministic fixed-order reductions.
//
//   alpha_p = min_f N_p,f (smallest eigenvalue of a diagonal N_p),
//   tau     = min over observed p of alpha_p w_p  (w_p pixel weight),
//   T_p     = tau / w_p,   K = 1 - T_p N^-1,   T N^-1,  N^-1 = 0 if masked,
//   d0      = d on observed pixels, 0 in the mask,   b = T N^-1 d0.
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
        if (obs && !obs[q]) continue;
        const double a = fmin(ncov[q], fmin(ncov[npix + q], ncov[2 * npix + q]));
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
        const bool ok = !obs || obs[o + j];
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
        const double v = (!obs || obs[pix]) ? d[i] : 0.0;
        d0[i] = v;
        b[i] = tn[q] * v;
    }
}

// grid (nrings, nrhs): ux <- N^-1 (ux - d0), b <- N^-1 d0,
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
            b[i] = ni * d0[i];
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

int grid_for(int64_t n) {
    int64_t g = (n + kBlk - 1) / kBlk;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_tau_parts(dm_plan* p, const double* ncov, const uint8_t* obs, double* ring_min, hipStream_t s) {
    hipLaunchKernelGGL(tau_kernel, dim3(p->nrings), dim3(kBlk), 0, s, p->npix, p->d_ring_off, p->d_ring_n,
                       p->d_ring_w, ncov, obs, ring_min);
    return hipGetLastError();
}

hipError_t launch_noise_setup(dm_plan* p, const double* ncov, const uint8_t* obs, double tau, hipStream_t s) {
    hipLaunchKernelGGL(noise_kernel, dim3(p->nrings, 3), dim3(kBlk), 0, s, p->npix, p->d_ring_off, p->d_ring_n,
                       p->d_ring_w, ncov, obs, tau, p->d_K, p->d_tn, p->d_ninv);
    return hipGetLastError();
}

hipError_t launch_data_setup(dm_plan* p, int nrhs, const double* d, double* d0, double* b, hipStream_t s) {
    const int64_t total = (int64_t)nrhs * 3 * p->npix;
    hipLaunchKernelGGL(data_kernel, dim3(grid_for(total)), dim3(kBlk), 0, s, p->npix, total, d, p->d_obs, p->d_tn,
                       d0, b);
    return hipGetLastError();
}

hipError_t launch_residual_maps(dm_plan* p, int nrhs, double* ux, const double* d0, double* b, double* chi_parts,
                                hipStream_t s) {
    hipLaunchKernelGGL(resid_kernel, dim3(p->nrings, nrhs), dim3(kBlk), 0, s, p->npix, p->nrings, p->d_ring_off,
                       p->d_ring_n, p->d_ninv, ux, d0, b, chi_parts);
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

hipError_t launch_count_nonfinite(const double* x, int64_t n, int* count, hipStream_t s) {
    hipLaunchKernelGGL(count_nonfinite_kernel, dim3(grid_for(n)), dim3(kBlk), 0, s, x, n, count);
    return hipGetLastError();
}

hipError_t launch_axpby(double* y, const double* x, double a, double c, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(kBlk), 0, s, y, x, a, c, n);
    return hipGetLastError();
}

}  // namespace dmwf
