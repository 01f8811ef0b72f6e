// Host-side tables of libdmwf: ring geometry, Legendre recursion
// coefficients and seed prefactors, ring-FFT chirp tables, and the per-l
// 3x3 filter matrices of the messenger update.  All built once per plan
// (filters once per cooling step) in long double and rounded to double.
#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>

#include "dmwf_internal.h"

namespace dmwf {

typedef long double ld;
static const ld kPi = 3.141592653589793238462643383279502884L;

// ----------------------------------------------------------------------------
// ring grids
// ----------------------------------------------------------------------------
// Gauss-Legendre nodes (descending) and weights by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        ld z = cosl(kPi * (i + 0.75L) / (n + 0.5L));
        ld dp = 0;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1; }
            dp = n * (z * p1 - p0) / (z * z - 1);
            ld dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        // recompute derivative at the converged node
        ld p0 = 1, p1 = z;
        for (int k = 2; k <= n; ++k) {
            ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1);
        ld wt = 2 / ((1 - z * z) * dp * dp);
        x[i] = (double)z;
        x[n - 1 - i] = (double)(-z);
        w[i] = w[n - 1 - i] = (double)wt;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

bool build_rings(const dm_grid& g, RingTables& rt, int64_t& npix, std::string& err) {
    rt = RingTables();
    if (g.kind == DM_GRID_HEALPIX_RING) {
        const int ns = g.nside;
        if (ns < 1 || ns > 8192) { err = "nside must be in [1, 8192]"; return false; }
        const int nr = 4 * ns - 1;
        npix = 12LL * ns * ns;
        int64_t off = 0;
        for (int k = 0; k < nr; ++k) {
            const int i = k + 1;
            double z, p0;
            int n;
            if (i < ns) {
                z = 1.0 - (double)i * i / (3.0 * ns * ns);
                n = 4 * i;
                p0 = M_PI / (4.0 * i);
            } else if (i <= 3 * ns) {
                z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns);
                n = 4 * ns;
                p0 = ((i - ns) % 2 == 0) ? M_PI / (4.0 * ns) : 0.0;
            } else {
                const int j = 4 * ns - i;
                z = -(1.0 - (double)j * j / (3.0 * ns * ns));
                n = 4 * j;
                p0 = M_PI / (4.0 * j);
            }
            rt.z.push_back(z);
            rt.phi0.push_back(p0);
            rt.nphi.push_back(n);
            rt.offset.push_back(off);
            rt.w.push_back(4.0 * M_PI / (double)npix);
            off += n;
        }
    } else if (g.kind == DM_GRID_GAUSS_LEGENDRE) {
        if (g.ntheta < 1 || g.nphi < 1) { err = "ntheta and nphi must be >= 1"; return false; }
        std::vector<double> x, w;
        gauss_legendre(g.ntheta, x, w);
        npix = (int64_t)g.ntheta * g.nphi;
        for (int k = 0; k < g.ntheta; ++k) {
            rt.z.push_back(x[k]);
            rt.phi0.push_back(0.0);
            rt.nphi.push_back(g.nphi);
            rt.offset.push_back((int64_t)k * g.nphi);
            rt.w.push_back(2.0 * M_PI * w[k] / g.nphi);
        }
    } else {
        err = "unknown grid kind";
        return false;
    }
    const int nr = (int)rt.z.size();
    const int np = (nr + 1) / 2;
    for (int p = 0; p < np; ++p) {
        const int s = nr - 1 - p;
        rt.pair_n.push_back(p);
        rt.pair_s.push_back(s == p ? -1 : s);
    }
    return true;
}

// ----------------------------------------------------------------------------
// Legendre recursion coefficients
// ----------------------------------------------------------------------------
// Spin 0 (orthonormal Y_lm, Condon-Shortley phase):
//   lam_l = A0 x lam_{l-1} - B0 lam_{l-2},
//   A0 = sqrt((4l^2-1)/(l^2-m^2)),  B0 = A0(l) / A0(l-1).
// Spin +-2, from the Wigner-d three-term recurrence normalised by
// sqrt((2l+1)/4pi), run separately for (+2)lam and (-2)lam with L = l - 1
// and R(q) = sqrt((q^2-m^2)(q^2-4)):
//   (+-2)lam_l = (alpha x +- alpha beta) (+-2)lam_L - gamma (+-2)lam_{L-1}
//   alpha = (L+1) sqrt((2L+3)(2L+1)) / R(L+1),  beta = 2m / (L(L+1)),
//   gamma = (L+1) R(L) sqrt((2L+3)/(2L-1)) / (L R(L+1)).
// Entries that a recursion never uses are zero, so that running a
// recursion over zero state before its start keeps it at zero.
void build_coefficients(int lmax, std::vector<double>& coef, std::vector<double>& lp0,
                        std::vector<double>& lp2) {
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    coef.assign(nalm * kCoefStride, 0.0);
    for (int m = 0; m <= lmax; ++m) {
        const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
        const ld mm = (ld)m * m;
        auto A0 = [&](int l) -> ld { return sqrtl((4.0L * l * l - 1) / ((ld)l * l - mm)); };
        auto R = [&](int q) -> ld {
            ld v = ((ld)q * q - mm) * ((ld)q * q - 4);
            return v > 0 ? sqrtl(v) : 0.0L;
        };
        for (int l = m + 1; l <= lmax; ++l) {
            double* c = &coef[(base + l) * kCoefStride];
            const ld a0 = A0(l);
            c[0] = (double)a0;
            c[1] = (l - 1 > m) ? (double)(a0 / A0(l - 1)) : 0.0;
            const int L = l - 1;
            if (L >= 2 && L >= m && R(L + 1) > 0) {
                const ld al = (L + 1) * sqrtl((ld)(2 * L + 3) * (2 * L + 1)) / R(L + 1);
                const ld be = 2.0L * m / ((ld)L * (L + 1));
                const ld ga = (L + 1) * R(L) * sqrtl((ld)(2 * L + 3) / (2 * L - 1)) / ((ld)L * R(L + 1));
                c[2] = (double)al;
                c[3] = (double)(al * be);
                c[4] = (double)ga;
            }
        }
    }
    // log prefactors of the seeds at l = m:
    //   lam_mm = (-1)^m exp(lp0[m]) sin^m theta,
    //   lp0[m] = -log(4 pi)/2 + (1/2) sum_{k<=m} log((2k+1)/(2k));
    //   W_mm, X_mm carry exp(lp2[m]) (sin theta / 2)^(m-2) with
    //   lp2[m] = (1/2) log((2m+1)/(4 pi)) + (1/2) log((2m)! / ((m-2)! (m+2)!)).
    lp0.assign(lmax + 1, 0.0);
    lp2.assign(lmax + 1, 0.0);
    ld acc = -0.5L * logl(4 * kPi);
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) acc += 0.5L * logl((2.0L * m + 1) / (2.0L * m));
        lp0[m] = (double)acc;
        if (m >= 2)
            lp2[m] = (double)(0.5L * logl((2.0L * m + 1) / (4 * kPi)) +
                              0.5L * (lgammal(2.0L * m + 1) - lgammal((ld)m - 1) - lgammal((ld)m + 3)));
    }
}

// Scaled recursions for the batched kernels.  With S_l = B0_l S_{l-2}
// (spin 0) or S_l = gamma_l S_{l-2} (spin 2), and S = 1 at the first two
// degrees of a recursion (m, m+1 for spin 0; max(m,2), max(m,2)+1 for
// spin 2), mu_l = lam_l / S_l obeys
//   mu_l = A0' x mu_{l-1} - mu_{l-2},                 A0' = A0 S_{l-1} / S_l,
//   mu_l = (alpha' x +- (alpha beta)') mu_{l-1} - mu_{l-2},
//          alpha' = alpha S_{l-1} / S_l, (alpha beta)' likewise,
// which saves a multiplication per function and degree.  S stays within
// [0.2, 1.2] for lmax <= 4096 (products of ratios close to 1).
void build_scaled_coefficients(int lmax, std::vector<double>& coef_s, std::vector<double>& scale) {
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    coef_s.assign(nalm * kCoefSStride, 0.0);
    scale.assign(nalm * 2, 1.0);
    std::vector<ld> S0(lmax + 2), S2(lmax + 2);
    for (int m = 0; m <= lmax; ++m) {
        const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
        const ld mm = (ld)m * m;
        auto A0 = [&](int l) -> ld { return sqrtl((4.0L * l * l - 1) / ((ld)l * l - mm)); };
        auto R = [&](int q) -> ld {
            ld v = ((ld)q * q - mm) * ((ld)q * q - 4);
            return v > 0 ? sqrtl(v) : 0.0L;
        };
        for (int l = m; l <= lmax; ++l) {
            S0[l] = l >= m + 2 ? A0(l) / A0(l - 1) * S0[l - 2] : 1.0L;
            scale[(base + l) * 2] = (double)S0[l];
            if (l > m) coef_s[(base + l) * kCoefSStride] = (double)(A0(l) * S0[l - 1] / S0[l]);
        }
        const int l0 = std::max(m, 2);
        for (int l = l0; l <= lmax; ++l) {
            const int L = l - 1;
            if (l >= l0 + 2) {
                const ld ga = (L + 1) * R(L) * sqrtl((ld)(2 * L + 3) / (2 * L - 1)) / ((ld)L * R(L + 1));
                S2[l] = ga * S2[l - 2];
            } else {
                S2[l] = 1.0L;
            }
            scale[(base + l) * 2 + 1] = (double)S2[l];
            if (l > l0) {
                const ld al = (L + 1) * sqrtl((ld)(2 * L + 3) * (2 * L + 1)) / R(L + 1);
                const ld be = 2.0L * m / ((ld)L * (L + 1));
                const ld r = S2[l - 1] / S2[l];
                coef_s[(base + l) * kCoefSStride + 1] = (double)(al * r);
                coef_s[(base + l) * kCoefSStride + 2] = (double)(al * be * r);
            }
        }
    }
}

// ----------------------------------------------------------------------------
// ring FFT tables: power-of-two lengths are transformed directly; other
// lengths by Bluestein's chirp-z convolution of size M = 2^k >= 2n - 1.
// ----------------------------------------------------------------------------
static void fft_ld(std::vector<std::complex<ld>>& a) {
    const int n = (int)a.size();
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const ld ang = -2 * kPi / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const std::complex<ld> w(cosl(ang * k), sinl(ang * k));
                const std::complex<ld> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}

static int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

// DFT of length 3 P (P a power of two) by decimation in time:
// X[k1 + P k2] = sum_n2 W_3^{n2 k2} W_{3P}^{n2 k1} FFT_P(a[3 n1 + n2])[k1]
static void fft3_ld(std::vector<std::complex<ld>>& a) {
    const int M = (int)a.size(), P = M / 3;
    std::vector<std::complex<ld>> y[3];
    for (int r = 0; r < 3; ++r) {
        y[r].resize(P);
        for (int q = 0; q < P; ++q) y[r][q] = a[3 * q + r];
        fft_ld(y[r]);
    }
    for (int k1 = 0; k1 < P; ++k1)
        for (int k2 = 0; k2 < 3; ++k2) {
            std::complex<ld> s(0, 0);
            for (int r = 0; r < 3; ++r) {
                const ld ang = -2 * kPi * (ld)((int64_t)r * (k1 + (int64_t)P * k2) % M) / M;
                s += y[r][k1] * std::complex<ld>(cosl(ang), sinl(ang));
            }
            a[k1 + P * k2] = s;
        }
}

// the transform size of a length: n itself for 2^k and (from 24 on) 3 2^k;
// for Bluestein the smaller of the power of two and of 3 2^k (k >= 3) that
// holds 2n - 1 points
static bool pow2_len(int n) { return (n & (n - 1)) == 0; }
static bool r3_len(int n) { return n >= 24 && n % 3 == 0 && pow2_len(n / 3); }
static int blue_size(int n) {
    const int m2 = 1 << ilog2(2 * n - 1);
    int m3 = 24;
    while (m3 < 2 * n - 1) m3 *= 2;
    return std::min(m2, m3);
}

// A Bluestein length n = 4 i is split into four length-i DFTs when its own
// Bluestein buffer (a power of two >= 2n - 1) exceeds max_elems, the
// largest buffer one workgroup's LDS holds: the split needs max(n, M_i)
// elements instead (at Nside 2048: 8188 instead of 16384).
bool build_fft_tables(const RingTables& rt, int mmax, int max_elems, FftTables& ft, std::string& err) {
    (void)mmax;
    ft = FftTables();
    std::vector<int> lens(rt.nphi.begin(), rt.nphi.end());
    std::sort(lens.begin(), lens.end());
    lens.erase(std::unique(lens.begin(), lens.end()), lens.end());
    // a split length's quarter keeps a power-of-two Bluestein size (its
    // launch stages four of them in one buffer)
    auto blue2 = [](int v) { return 1 << ilog2(2 * v - 1); };
    int64_t coff = 0, boff = 0;
    for (int n : lens) {
        const bool direct = pow2_len(n) || r3_len(n);
        const bool split = !direct && n % 4 == 0 && blue_size(n) > max_elems;
        const int nb = split ? n / 4 : n;              // Bluestein length
        const int M = direct ? n : split ? blue2(nb) : blue_size(nb);
        const int r3 = (M % 3 == 0) ? 1 : 0;
        const int P = r3 ? M / 3 : M;
        ft.n.push_back(n);
        ft.split.push_back(split ? 1 : 0);
        ft.M.push_back(M);
        ft.logM.push_back(ilog2(P));
        ft.r3.push_back(r3);
        ft.chirp_off.push_back(direct ? -1 : coff);
        ft.bhat_off.push_back(direct ? -1 : boff);
        if (!direct) {
            coff += nb;
            boff += M;
        }
        ft.Mmax = std::max(ft.Mmax, P);
        if (r3) ft.P3max = std::max(ft.P3max, P);
        if (split)
            ft.lds_split = std::max(ft.lds_split, std::max(n, M));
        else
            ft.lds_elems = std::max(ft.lds_elems, M);
    }
    ft.chirp.assign(2 * coff, 0.0);
    ft.bhat.assign(2 * boff, 0.0);
    const int nl = (int)ft.n.size();
    auto work = [&](int t, int nt) {
        for (int i = t; i < nl; i += nt) {
            if (ft.chirp_off[i] < 0) continue;
            const int n = ft.split[i] ? ft.n[i] / 4 : ft.n[i], M = ft.M[i];
            std::vector<std::complex<ld>> b(M, std::complex<ld>(0, 0));
            for (int j = 0; j < n; ++j) {
                const int64_t r = ((int64_t)j * j) % (2 * (int64_t)n);   // exact j^2 mod 2n
                const ld ang = kPi * (ld)r / n;
                ft.chirp[2 * (ft.chirp_off[i] + j)] = (double)cosl(ang);
                ft.chirp[2 * (ft.chirp_off[i] + j) + 1] = (double)(-sinl(ang));
                const std::complex<ld> bj(cosl(ang), sinl(ang));
                b[j] = bj;
                if (j > 0) b[M - j] = bj;
            }
            if (ft.r3[i]) fft3_ld(b);
            else fft_ld(b);
            for (int k = 0; k < M; ++k) {
                ft.bhat[2 * (ft.bhat_off[i] + k)] = (double)(b[k].real() / M);
                ft.bhat[2 * (ft.bhat_off[i] + k) + 1] = (double)(b[k].imag() / M);
            }
        }
    };
    int nt = (int)std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(work, t, nt);
    for (auto& x : th) x.join();
    ft.tw.assign(ft.Mmax, 0.0);
    for (int k = 0; k < ft.Mmax / 2; ++k) {
        const ld ang = -2 * kPi * k / ft.Mmax;
        ft.tw[2 * k] = (double)cosl(ang);
        ft.tw[2 * k + 1] = (double)sinl(ang);
    }
    if (ft.Mmax < 2) {
        ft.tw.assign(2, 0.0);
        ft.tw[0] = 1.0;
    }
    // the radix-3 passes' twiddles W_{3P}^e = exp(-2 pi i e P3max / (3 P3max P))
    // for e < 2P, read at stride P3max / P
    const int n3 = 3 * ft.P3max;
    ft.tw3.assign(2 * (size_t)n3, 0.0);
    for (int e = 0; e < n3; ++e) {
        const ld ang = -2 * kPi * e / n3;
        ft.tw3[2 * e] = (double)cosl(ang);
        ft.tw3[2 * e + 1] = (double)sinl(ang);
    }
    (void)err;
    return true;
}

// ----------------------------------------------------------------------------
// per-l matrix functions of the signal covariance (eq 10): the TE block is
// diagonalised by a rotation, B is already diagonal.
// which: 0 = messenger filter max(s, mu) / (max(s, mu) + tau)
//        1 = s^1/2,  2 = pseudo-inverse s^-1/2,  3 = pseudo-inverse s^-1
// Output F [lmax+1][4] = (F_TT, F_TE, F_EE, F_BB).
// ----------------------------------------------------------------------------
static void matfun(const std::vector<double>& cl, int lmax, int which, ld mu, ld tau,
                   std::vector<double>& F) {
    F.assign((size_t)(lmax + 1) * 4, 0.0);
    auto f = [&](ld s, ld smax) -> ld {
        switch (which) {
            case 0: { ld v = s > mu ? s : mu; return v / (v + tau); }
            case 1: return s > 0 ? sqrtl(s) : 0.0L;
            case 2: return s > 1e-14L * smax && s > 0 ? 1.0L / sqrtl(s) : 0.0L;
            default: return s > 1e-14L * smax && s > 0 ? 1.0L / s : 0.0L;
        }
    };
    for (int l = 0; l <= lmax; ++l) {
        const ld TT = cl[0 * (lmax + 1) + l], EE = cl[1 * (lmax + 1) + l];
        const ld BB = cl[2 * (lmax + 1) + l], TE = cl[3 * (lmax + 1) + l];
        const ld phi = 0.5L * atan2l(2 * TE, TT - EE);
        const ld c = cosl(phi), s = sinl(phi);
        const ld s1 = TT * c * c + 2 * TE * s * c + EE * s * s;
        const ld s2 = TT * s * s - 2 * TE * s * c + EE * c * c;
        const ld smax = std::max(fabsl(s1), fabsl(s2));
        const ld f1 = f(s1, smax), f2 = f(s2, smax);
        F[4 * l + 0] = (double)(f1 * c * c + f2 * s * s);
        F[4 * l + 1] = (double)((f1 - f2) * s * c);
        F[4 * l + 2] = (double)(f1 * s * s + f2 * c * c);
        F[4 * l + 3] = (double)f(BB, fabsl(BB));
    }
}

void build_filter(const std::vector<double>& cl, int lmax, double mu, double tau, std::vector<double>& F) {
    matfun(cl, lmax, 0, mu, tau, F);
}

void build_matrix_function(const std::vector<double>& cl, int lmax, int which, std::vector<double>& F) {
    matfun(cl, lmax, which, 0, 1, F);
}

}  // namespace dmwf
