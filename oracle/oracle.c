/*
 * FP64 brute-force CPU oracle for the periodic-box O(N^2) power-spectrum and
 * bispectrum estimators of Philcox (2020), arXiv:2005.01739.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition that the
 * GPU library is checked against.  It shares no code, header, table or helper
 * with the GPU library, and nothing in the product calls it; only the tests,
 * the package smoke check and the benchmark's CPU-baseline leg load it.
 *
 * Everything is double precision, compiled without floating-point
 * contraction (-ffp-contract=off), so each expression rounds exactly as
 * written.
 *
 * Conventions (readings of the paper, each listed in the design notes):
 *  - pairs are ordered pairs (i, j), i != j by index (Sec. 2, discrete pair
 *    count; self-counts excluded), coincident distinct particles included;
 *  - separation x_ij = x_i - x_j, per axis wrapped to the nearest periodic
 *    image by one comparison each way (d > L/2 -> d - L, d < -L/2 -> d + L);
 *    r^2 = (dx*dx + dy*dy) + dz*dz, and a pair counts iff r^2 < R0*R0.  This
 *    FP64 predicate defines the integer pair count;
 *  - weights w_i enter as w_i w_j (Sec. 2 footnote on weights); the mean
 *    density is n_w = sum(w) / V;
 *  - the line of sight is a fixed box axis (Sec. 2, fixed LoS for
 *    simulations), default z; the survey-geometry estimator (no periodicity)
 *    takes it along each pair's midpoint, the observer at the origin.
 *
 * Parity status: every function below is pinned by tests against mpmath or
 * scipy evaluations, closed forms, brute-force triple sums or exact
 * expectations of random catalogues (see tests/test_oracle_*.py).  For
 * clustered catalogues the bispectrum's pin is the brute-force sum over
 * distinct triples (run on a clustered catalogue) and the invariances; no
 * closed-form expectation is derived for them.  The analytic DDR^II kernel
 * (oracle_eii) is pinned against the 3-D definition integrated by scipy in
 * other coordinates, its exact volume integral and its x -> 0 limit; the pair
 * sum over its interpolated table (oracle_ddr2) against random primaries on a
 * fine lattice and against per-pair kernel values.  The theory side
 * (oracle_omega, oracle_cov_gauss, oracle_pk_window_theory) is pinned against
 * scipy quadrature, Parseval's relation with the E^II kernel at zero
 * separation, and the Gaunt integral of Q by direct angular quadrature.  The
 * Poisson terms (oracle_cov_poisson2, oracle_cov_poisson3) are pinned, at
 * xi = 0, against the exact variance of the estimator for a uniform catalogue
 * with a fixed or a Poisson-distributed number of points (a degenerate
 * U-statistic, with the Poisson moments of N summed from the distribution);
 * their xi and P_L parts by direct angular quadrature and Parseval's relation.
 * The bispectrum term of 3C is added as printed: only the symmetry of the
 * result under (l, a) <-> (l', b) pins it (parity unpinned for that term).
 * The non-Gaussian term (oracle_cov_nongauss) is pinned by its reduction to
 * the (pinned) Gaussian term for a trispectrum diagonal on the quadrature
 * grid, and by its symmetry.  The anisotropic bispectrum (oracle_bk_aniso, a
 * reading of Sec. 10) is pinned by literal triple sums over distinct triples
 * with scipy's harmonics (data and random primaries), by the literal pair sum
 * of its DDR^I term, and by the identity that its m-sum at l1 = l2 is the
 * (pinned) isotropic estimator.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_ELL_MAX 6
#define ORACLE_NK_MAX 128
/* Below this argument D_ell is taken from its Taylor series; at and above it
 * from the Appendix C recursion.  Both are accurate to < 1e-15 relative at the
 * switch for ell <= 6 (checked against mpmath in the tests). */
#define U_SWITCH 5.0

static const double PI = 3.14159265358979323846264338327950288;

/* ---------------------------------------------------------------- window */
/* Smooth truncation window W(x), x = r / R0 (Sec. 2, eq. window_defn). */
double oracle_window(double x)
{
    if (x < 0.0) return 0.0;
    if (x < 0.5) return 1.0;
    if (x < 0.75) {
        double t = 2.0 * x - 1.0;
        return 1.0 - 8.0 * t * t * t + 8.0 * t * t * t * t;
    }
    if (x < 1.0) {
        double t = x - 1.0;
        return -64.0 * t * t * t - 128.0 * t * t * t * t;
    }
    return 0.0;
}

/* Legendre polynomial L_ell(mu) by Bonnet's recursion. */
double oracle_legendre(int ell, double mu)
{
    double p0 = 1.0, p1 = mu;
    if (ell == 0) return p0;
    for (int n = 1; n < ell; ++n) {
        double p2 = ((2.0 * n + 1.0) * mu * p1 - n * p0) / (n + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

/* ------------------------------------------------------- sine integral */
/* Si(u) = int_0^u sin(t)/t dt.  Power series for u <= 4; above, through the
 * exponential integral, Si(u) = pi/2 + Im E1(iu), with E1 from its continued
 * fraction E1(z) = e^{-z} / (z + 1 - 1/(z + 3 - 4/(z + 5 - ...))) evaluated
 * by the modified Lentz method (Lentz 1976; Thompson & Barnett 1986). */
double oracle_si(double u)
{
    if (u < 0.0) return -oracle_si(-u);
    if (u == 0.0) return 0.0;
    if (u <= 4.0) {
        double sum = 0.0, p = u; /* p = (-1)^n u^(2n+1) / (2n+1)! */
        for (int n = 0; n < 60; ++n) {
            double term = p / (2.0 * n + 1.0);
            sum += term;
            if (fabs(term) < 1e-18 * fabs(sum)) break;
            p = -p * u * u / ((2.0 * n + 2.0) * (2.0 * n + 3.0));
        }
        return sum;
    }
    const double tiny = 1e-300;
    double complex z = I * u;
    double complex b = z + 1.0;
    double complex c = 1.0 / tiny;
    double complex d = 1.0 / b;
    double complex h = d;
    for (int n = 1; n < 1000; ++n) {
        double a = -(double)n * (double)n;
        b += 2.0;
        d = 1.0 / (a * d + b);
        c = b + a / c;
        double complex del = c * d;
        h *= del;
        if (cabs(del - 1.0) < 1e-17) break;
    }
    double complex e1 = h * cexp(-z);
    return 0.5 * PI + cimag(e1);
}

/* Spherical Bessel j_0..j_nmax by upward recurrence
 * j_{n+1} = (2n+1)/u j_n - j_{n-1}.  Used only for u >= U_SWITCH, where the
 * recurrence is accurate for the orders needed here (n <= 7). */
void oracle_sph_bessel_up(int nmax, double u, double *j)
{
    double s = sin(u), c = cos(u);
    j[0] = s / u;
    if (nmax >= 1) j[1] = s / (u * u) - c / u;
    for (int n = 1; n < nmax; ++n) j[n + 1] = (2.0 * n + 1.0) / u * j[n] - j[n - 1];
}

/* (2n+1)!! */
static double dfact_odd(int n)
{
    double f = 1.0;
    for (int k = 3; k <= 2 * n + 1; k += 2) f *= k;
    return f;
}

/* D_ell(0) of the Appendix C recursion: with j_0(0)=1, j_n(0)=0 (n>0),
 * I_0(0) = Si(0) = 0, I_1(0) = -j_0(0) = -1 and ell I_ell = (ell-1) I_{ell-2}
 * - (2 ell - 1) j_{ell-1}, D_ell(0) = ell (ell+1) I_ell(0). */
double oracle_D_at_zero(int ell)
{
    double I0 = 0.0, I1 = -1.0;
    double Il[ORACLE_ELL_MAX + 2];
    Il[0] = I0;
    Il[1] = I1;
    for (int l = 2; l <= ell; ++l) {
        double jlm1 = (l - 1 == 0) ? 1.0 : 0.0;
        Il[l] = ((l - 1) * Il[l - 2] - (2.0 * l - 1.0) * jlm1) / l;
    }
    return ell * (ell + 1.0) * Il[ell];
}

/* D_ell(u), the antiderivative of u^2 j_ell(u) in the normalisation fixed by
 * the Appendix C recursion:
 *   D_ell = u^2 j_{ell+1} - ell u j_ell + ell (ell+1) I_ell,
 *   ell I_ell = (ell-1) I_{ell-2} - (2 ell - 1) j_{ell-1},
 *   I_0 = Si, I_1 = -j_0.
 * For u < U_SWITCH the recursion cancels catastrophically, so there
 * D_ell(u) = D_ell(0) + int_0^u t^2 j_ell(t) dt with the integral from the
 * term-by-term integrated Taylor series of j_ell. */
double oracle_D(int ell, double u)
{
    if (u < U_SWITCH) {
        /* sum_s (-1)^s u^(ell+2s+3) / ((ell+2s+3) 2^s s! (2ell+2s+1)!!) */
        double sum = 0.0;
        double t = pow(u, ell + 3) / dfact_odd(ell); /* s = 0, without 1/(ell+3) */
        for (int s = 0; s < 80; ++s) {
            double term = t / (ell + 2.0 * s + 3.0);
            sum += term;
            if (fabs(term) <= 1e-18 * fabs(sum) && s > 2) break;
            t = -t * u * u / (2.0 * (s + 1.0) * (2.0 * ell + 2.0 * s + 3.0));
        }
        return oracle_D_at_zero(ell) + sum;
    }
    double j[ORACLE_ELL_MAX + 3];
    oracle_sph_bessel_up(ell + 1, u, j);
    double Il[ORACLE_ELL_MAX + 2];
    Il[0] = oracle_si(u);
    Il[1] = -j[0];
    for (int l = 2; l <= ell; ++l)
        Il[l] = ((l - 1) * Il[l - 2] - (2.0 * l - 1.0) * j[l - 1]) / l;
    return u * u * j[ell + 1] - ell * u * j[ell] + ell * (ell + 1.0) * Il[ell];
}

/* k-bin averaged spherical Bessel function (Sec. 3, eq. jla-def):
 *   jbar^a_ell(x) = 3 [D_ell(x k2) - D_ell(x k1)] / (x^3 (k2^3 - k1^3)).
 * For x k2 < U_SWITCH the bin average is taken from the integrated Taylor
 * series instead,
 *   3/(k2^3-k1^3) sum_s (-1)^s x^(ell+2s) (k2^n - k1^n) / (n 2^s s! (2ell+2s+1)!!),
 * n = ell+2s+3, which is exact and free of the small-argument cancellation;
 * jbar^a_ell(0) = delta_{ell 0}. */
double oracle_jbar_series(int ell, double x, double k1, double k2)
{
    if (x == 0.0) return ell == 0 ? 1.0 : 0.0;
    double dk3 = k2 * k2 * k2 - k1 * k1 * k1;
    double sum = 0.0;
    double t = pow(x, ell) / dfact_odd(ell); /* (-1)^s x^(ell+2s) / (2^s s! (2l+2s+1)!!) */
    for (int s = 0; s < 80; ++s) {
        int n = ell + 2 * s + 3;
        double term = t * (pow(k2, n) - pow(k1, n)) / n;
        sum += term;
        if (fabs(term) <= 1e-18 * fabs(sum) && s > 2) break;
        t = -t * x * x / (2.0 * (s + 1.0) * (2.0 * ell + 2.0 * s + 3.0));
    }
    return 3.0 * sum / dk3;
}

double oracle_jbar(int ell, double x, double k1, double k2)
{
    if (x * k2 < U_SWITCH) return oracle_jbar_series(ell, x, k1, k2);
    double dk3 = k2 * k2 * k2 - k1 * k1 * k1;
    return 3.0 * (oracle_D(ell, x * k2) - oracle_D(ell, x * k1)) / (x * x * x * dk3);
}

/* jbar for all bins of one pair at once, from one D evaluation per edge. */
static void jbar_all_bins(int ell, double x, int n_k, const double *k, double *out)
{
    double Dedge[ORACLE_NK_MAX + 1];
    int have = 0;
    for (int a = 0; a < n_k; ++a) {
        if (x * k[a + 1] < U_SWITCH) {
            out[a] = oracle_jbar_series(ell, x, k[a], k[a + 1]);
            continue;
        }
        if (!have) {
            for (int e = a; e <= n_k; ++e) Dedge[e] = oracle_D(ell, x * k[e]);
            have = 1;
        }
        double dk3 = k[a + 1] * k[a + 1] * k[a + 1] - k[a] * k[a] * k[a];
        out[a] = 3.0 * (Dedge[a + 1] - Dedge[a]) / (x * x * x * dk3);
    }
}

/* --------------------------------------------------- spherical harmonics */
/* Complex orthonormal Y_lm(theta, phi) with the Condon-Shortley phase,
 * for 0 <= l <= lmax, -l <= m <= l, stored at index l*l + l + m.
 * (x, y, z) need not be normalised; the zero vector is treated as +z. */
void oracle_ylm(int lmax, double x, double y, double z, double *re, double *im)
{
    double r = sqrt(x * x + y * y + z * z);
    double ct = r > 0.0 ? z / r : 1.0;
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double phi = (x == 0.0 && y == 0.0) ? 0.0 : atan2(y, x);
    for (int m = 0; m <= lmax; ++m) {
        /* P_m^m = (-1)^m (2m-1)!! st^m */
        double pmm = 1.0;
        for (int k = 1; k <= m; ++k) pmm *= -(2.0 * k - 1.0) * st;
        double plm2 = 0.0, plm1 = pmm;
        for (int l = m; l <= lmax; ++l) {
            double plm;
            if (l == m) plm = pmm;
            else if (l == m + 1) plm = ct * (2.0 * m + 1.0) * pmm;
            else plm = ((2.0 * l - 1.0) * ct * plm1 - (l + m - 1.0) * plm2) / (l - m);
            if (l > m) { plm2 = plm1; plm1 = plm; }
            else { plm1 = plm; plm2 = 0.0; }
            /* normalisation sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) */
            double ratio = 1.0;
            for (int k = l - m + 1; k <= l + m; ++k) ratio /= k;
            double nrm = sqrt((2.0 * l + 1.0) / (4.0 * PI) * ratio);
            double yr = nrm * plm * cos(m * phi), yi = nrm * plm * sin(m * phi);
            re[l * l + l + m] = yr;
            im[l * l + l + m] = yi;
            if (m > 0) { /* Y_{l,-m} = (-1)^m conj(Y_lm) */
                double sg = (m & 1) ? -1.0 : 1.0;
                re[l * l + l - m] = sg * yr;
                im[l * l + l - m] = -sg * yi;
            }
        }
    }
}

/* ------------------------------------------------ window integral W~^a */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* W~^a(R0) = 4 pi int_0^R0 r^2 jbar^a_0(r) W(r/R0) dr (Sec. 3, eq. wka-def),
 * by composite 20-point Gauss-Legendre on the three smooth pieces of W,
 * [0, R0/2], [R0/2, 3R0/4], [3R0/4, R0], each cut into panels no wider than
 * (pi / 2) / (k2 * resolution). */
double oracle_wtilde(double r0, double k1, double k2, double resolution)
{
    enum { NG = 20 };
    double gx[NG], gw[NG];
    gauss_legendre(NG, gx, gw);
    double cuts[4] = {0.0, 0.5 * r0, 0.75 * r0, r0};
    double total = 0.0;
    for (int piece = 0; piece < 3; ++piece) {
        double a = cuts[piece], b = cuts[piece + 1];
        double hmax = 0.5 * PI / (k2 * resolution);
        int np = (int)ceil((b - a) / hmax);
        if (np < 1) np = 1;
        double h = (b - a) / np;
        for (int p = 0; p < np; ++p) {
            double lo = a + p * h, hi = lo + h, mid = 0.5 * (lo + hi), half = 0.5 * h;
            for (int q = 0; q < NG; ++q) {
                double r = mid + half * gx[q];
                double f = r * r * oracle_jbar(0, r, k1, k2) * oracle_window(r / r0);
                total += half * gw[q] * f;
            }
        }
    }
    return 4.0 * PI * total;
}

/* -------------------------------------------------------- pair geometry */
static inline double min_image(double d, double L)
{
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

static int nthreads_or_default(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* ------------------------------------------------------ power spectrum */
/* P^a_ell for even ell = 0, 2, ..., ell_max (Sec. 3, binned estimator):
 *   S^a_ell = sum_{i != j} w_i w_j (2 ell + 1) (-i)^ell W(r/R0) jbar^a_ell(r) L_ell(mu),
 *   P^a_ell = S^a_ell / (n_w^2 V) - delta_{ell 0} W~^a,
 * mu = (x_ij . los) / r (taken as 0 at r = 0, where jbar_{ell>0} = 0).
 * Ordered pairs run over primaries i with primary_mask[i] != 0 (all when the
 * mask is NULL) and every secondary j != i.
 * Outputs are [n_ell][n_k], n_ell = ell_max/2 + 1: pk, raw (= S), l1 (the sum
 * of |term|), wtilde [n_k]; *n_pairs counts the ordered pairs inside R0.
 * Returns 0, or -1 on an argument outside the oracle's range. */
int oracle_pk_ell(int64_t n, const double *pos, const double *w, double box, double r0,
                  int n_k, const double *k, int ell_max, int los_axis,
                  const uint8_t *primary_mask, double *pk, double *raw, double *l1,
                  double *wtilde, uint64_t *n_pairs, int nthreads)
{
    if (n < 1 || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 || ell_max > ORACLE_ELL_MAX ||
        (ell_max & 1) || los_axis < 0 || los_axis > 2 || !(r0 > 0.0) || r0 > 0.5 * box)
        return -1;
    const int n_ell = ell_max / 2 + 1;
    const int nt = nthreads_or_default(nthreads);
    const size_t nacc = (size_t)n_ell * n_k;
    double *acc = calloc((size_t)nt * nacc * 2, sizeof(double));
    uint64_t *cnt = calloc((size_t)nt, sizeof(uint64_t));
    const double r02 = r0 * r0;

#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *S = acc + (size_t)tid * nacc * 2, *A = S + nacc;
        double jb[ORACLE_NK_MAX];
        uint64_t c = 0;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            if (primary_mask && !primary_mask[i]) continue;
            const double wi = w ? w[i] : 1.0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double d[3];
                for (int ax = 0; ax < 3; ++ax) d[ax] = min_image(pos[3 * i + ax] - pos[3 * j + ax], box);
                double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                if (!(r2 < r02)) continue;
                ++c;
                double r = sqrt(r2);
                double wgt = wi * (w ? w[j] : 1.0) * oracle_window(r / r0);
                double mu = r > 0.0 ? d[los_axis] / r : 0.0;
                for (int li = 0; li < n_ell; ++li) {
                    int ell = 2 * li;
                    double phase = (li & 1) ? -1.0 : 1.0; /* (-i)^ell, ell even */
                    double lw = (2.0 * ell + 1.0) * phase * wgt * oracle_legendre(ell, mu);
                    jbar_all_bins(ell, r, n_k, k, jb);
                    for (int a = 0; a < n_k; ++a) {
                        double term = lw * jb[a];
                        S[li * n_k + a] += term;
                        A[li * n_k + a] += fabs(term);
                    }
                }
            }
        }
        cnt[tid] = c;
    }
    double p1 = 0.0;
    for (int64_t i = 0; i < n; ++i) p1 += w ? w[i] : 1.0;
    const double V = box * box * box, nw = p1 / V;
    uint64_t ctot = 0;
    for (int t = 0; t < nt; ++t) ctot += cnt[t];
    for (int a = 0; a < n_k; ++a) wtilde[a] = oracle_wtilde(r0, k[a], k[a + 1], 4.0);
    for (size_t q = 0; q < nacc; ++q) {
        double s = 0.0, m = 0.0;
        for (int t = 0; t < nt; ++t) {
            s += acc[(size_t)t * nacc * 2 + q];
            m += acc[(size_t)t * nacc * 2 + nacc + q];
        }
        if (raw) raw[q] = s;
        if (l1) l1[q] = m;
        int li = (int)(q / n_k), a = (int)(q % n_k);
        pk[q] = s / (nw * nw * V) - (li == 0 ? wtilde[a] : 0.0);
    }
    if (n_pairs) *n_pairs = ctot;
    free(acc);
    free(cnt);
    return 0;
}

/* ----------------------------------------------- survey-geometry power spectrum */
/* The general estimator of Sec. 2 (eq. general-Pk-ell with the pair counts of
 * eq. general-XY-counts), binned in k as in Sec. 3 (eq. jla-def): data D and
 * randoms R at arbitrary positions, no periodicity, observer at the origin,
 * and the line of sight of pair (i, j) along its midpoint (x_i + x_j) / 2.
 *
 *   XY^a_l = (-i)^l (2l+1) sum_{i in X} sum_{j in Y, j != i if X = Y}
 *            v_i v_j jbar^a_l(r_ij) L_l(xhat_ij . nhat_ij) W(r_ij / R0)
 *   P^a_l  = [DD - (DR + RD) + RR]^a_l / (n_w^2 V),   n_w = sum(w_D) / V
 *
 * with v = w for data and v = s_R w for randoms, s_R = sum(w_D) / sum(w_R)
 * (random catalogues normalised to the data, the reading also used for the
 * bispectrum), and DR + RD = 2 DR for even l.  V is the caller's survey
 * volume.  A pair counts iff r^2 < R0^2 with r^2 = (dx^2 + dy^2) + dz^2 in
 * FP64; mu = 0 when r = 0 or the midpoint is the observer.  Masks: only
 * ordered pairs (i, j) whose first point has mask != 0 contribute.
 * Accumulates the ordered pairs (i in X, j in Y) of one kind into S, |S| into
 * A, with the factor f = v-scale of the pair kind. */
static uint64_t survey_pair_sums(int64_t nx, const double *px, const double *wx, const uint8_t *mx,
                                 int64_t ny, const double *py, const double *wy, int same, double f,
                                 double r0, int n_k, const double *k, int n_ell, double *S, double *A,
                                 int nthreads)
{
    const size_t nacc = (size_t)n_ell * n_k;
    const int nt = nthreads_or_default(nthreads);
    double *acc = calloc((size_t)nt * nacc * 2, sizeof(double));
    uint64_t *cnt = calloc((size_t)nt, sizeof(uint64_t));
    const double r02 = r0 * r0;
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *Sl = acc + (size_t)tid * nacc * 2, *Al = Sl + nacc;
        double jb[ORACLE_NK_MAX];
        uint64_t c = 0;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nx; ++i) {
            if (mx && !mx[i]) continue;
            const double wi = wx ? wx[i] : 1.0;
            for (int64_t j = 0; j < ny; ++j) {
                if (same && j == i) continue;
                double d[3], m[3];
                for (int ax = 0; ax < 3; ++ax) {
                    d[ax] = px[3 * i + ax] - py[3 * j + ax];
                    m[ax] = px[3 * i + ax] + py[3 * j + ax];
                }
                double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                if (!(r2 < r02)) continue;
                ++c;
                double r = sqrt(r2);
                double mn = sqrt((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2]);
                double mu = (r > 0.0 && mn > 0.0) ? ((d[0] * m[0] + d[1] * m[1]) + d[2] * m[2]) / (r * mn) : 0.0;
                double wgt = f * wi * (wy ? wy[j] : 1.0) * oracle_window(r / r0);
                for (int li = 0; li < n_ell; ++li) {
                    int ell = 2 * li;
                    double phase = (li & 1) ? -1.0 : 1.0; /* (-i)^ell, ell even */
                    double lw = (2.0 * ell + 1.0) * phase * wgt * oracle_legendre(ell, mu);
                    jbar_all_bins(ell, r, n_k, k, jb);
                    for (int a = 0; a < n_k; ++a) {
                        double term = lw * jb[a];
                        Sl[li * n_k + a] += term;
                        Al[li * n_k + a] += fabs(term);
                    }
                }
            }
        }
        cnt[tid] = c;
    }
    uint64_t ctot = 0;
    for (int t = 0; t < nt; ++t) {
        ctot += cnt[t];
        for (size_t q = 0; q < nacc; ++q) {
            S[q] += acc[(size_t)t * nacc * 2 + q];
            A[q] += acc[(size_t)t * nacc * 2 + nacc + q];
        }
    }
    free(acc);
    free(cnt);
    return ctot;
}

int oracle_pk_survey(int64_t nd, const double *pd, const double *wd, const uint8_t *md,
                     int64_t nr, const double *pr, const double *wr, const uint8_t *mr,
                     double volume, double r0, int n_k, const double *k, int ell_max,
                     double *pk, double *raw_dd, double *raw_dr, double *raw_rr, double *l1,
                     uint64_t *counts, int nthreads)
{
    if (nd < 1 || nr < 1 || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 || ell_max > ORACLE_ELL_MAX ||
        (ell_max & 1) || !(r0 > 0.0) || !(volume > 0.0))
        return -1;
    const int n_ell = ell_max / 2 + 1;
    const size_t nacc = (size_t)n_ell * n_k;
    double p1 = 0.0, pr1 = 0.0;
    for (int64_t i = 0; i < nd; ++i) p1 += wd ? wd[i] : 1.0;
    for (int64_t i = 0; i < nr; ++i) pr1 += wr ? wr[i] : 1.0;
    const double sR = p1 / pr1;
    memset(raw_dd, 0, nacc * sizeof(double));
    memset(raw_dr, 0, nacc * sizeof(double));
    memset(raw_rr, 0, nacc * sizeof(double));
    double *Add = calloc(nacc, sizeof(double)), *Adr = calloc(nacc, sizeof(double)), *Arr = calloc(nacc, sizeof(double));
    uint64_t c_dd = survey_pair_sums(nd, pd, wd, md, nd, pd, wd, 1, 1.0, r0, n_k, k, n_ell, raw_dd, Add, nthreads);
    uint64_t c_dr = survey_pair_sums(nd, pd, wd, md, nr, pr, wr, 0, sR, r0, n_k, k, n_ell, raw_dr, Adr, nthreads);
    c_dr += survey_pair_sums(nr, pr, wr, mr, nd, pd, wd, 0, sR, r0, n_k, k, n_ell, raw_dr, Adr, nthreads);
    uint64_t c_rr = survey_pair_sums(nr, pr, wr, mr, nr, pr, wr, 1, sR * sR, r0, n_k, k, n_ell, raw_rr, Arr, nthreads);
    const double nw = p1 / volume;
    for (size_t q = 0; q < nacc; ++q) {
        pk[q] = (raw_dd[q] - raw_dr[q] + raw_rr[q]) / (nw * nw * volume);
        if (l1) l1[q] = Add[q] + Adr[q] + Arr[q];
    }
    if (counts) {
        counts[0] = c_dd;
        counts[1] = c_dr;
        counts[2] = c_rr;
    }
    free(Add);
    free(Adr);
    free(Arr);
    return 0;
}

/* ------------------------------------------------------------ bispectrum */
/* Accumulate, for each primary p in [0, np) (mask permitting) against every
 * data secondary j (skipping j == p when `self_exclude`):
 *   A^a_lm(p) = sum_j w_j jbar^a_l(r) W(r/R0) Y_lm(x_pj / r)      (eq. AC-def, binned)
 *   C^ab_l(p) = sum_j w_j^2 jbar^a_l jbar^b_l W^2
 *   G^ab_l   += w_p (4 pi / (2l+1)) sum_m Re(A^a_lm conj(A^b_lm))
 *   Cs^ab_l  += w_p C^ab_l(p)
 *   S0^b     += w_p sum_j w_j jbar^b_0 W              (data primaries only)
 * with x_pj = x_p - x_j.  G, Cs: [lmax+1][n_k][n_k]. */
static uint64_t bk_primary_sums(int64_t np, const double *ppos, const double *pw,
                                const uint8_t *mask, int self_exclude, int64_t n,
                                const double *pos, const double *w, double box, double r0,
                                int n_k, const double *k, int lmax, double *G, double *Cs,
                                double *S0, int nt)
{
    const int nlm = (lmax + 1) * (lmax + 1);
    const size_t ng = (size_t)(lmax + 1) * n_k * n_k;
    double *acc = calloc((size_t)nt * (2 * ng + n_k), sizeof(double));
    uint64_t *cnt = calloc((size_t)nt, sizeof(uint64_t));
    const double r02 = r0 * r0;
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *tG = acc + (size_t)tid * (2 * ng + n_k), *tC = tG + ng, *tS = tC + ng;
        double complex *Alm = malloc(sizeof(double complex) * (size_t)n_k * nlm);
        double *Cp = malloc(sizeof(double) * ng);
        double *g = malloc(sizeof(double) * (size_t)(lmax + 1) * n_k);
        double yre[(ORACLE_ELL_MAX + 1) * (ORACLE_ELL_MAX + 1)], yim[(ORACLE_ELL_MAX + 1) * (ORACLE_ELL_MAX + 1)];
        uint64_t c = 0;
#pragma omp for schedule(static)
        for (int64_t p = 0; p < np; ++p) {
            if (mask && !mask[p]) continue;
            const double wp = pw ? pw[p] : 1.0;
            memset(Alm, 0, sizeof(double complex) * (size_t)n_k * nlm);
            memset(Cp, 0, sizeof(double) * ng);
            double s0loc[ORACLE_NK_MAX];
            for (int a = 0; a < n_k; ++a) s0loc[a] = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (self_exclude && j == p) continue;
                double d[3];
                for (int ax = 0; ax < 3; ++ax) d[ax] = min_image(ppos[3 * p + ax] - pos[3 * j + ax], box);
                double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                if (!(r2 < r02)) continue;
                ++c;
                double r = sqrt(r2);
                double wj = w ? w[j] : 1.0;
                double W = oracle_window(r / r0);
                for (int l = 0; l <= lmax; ++l) {
                    jbar_all_bins(l, r, n_k, k, g + (size_t)l * n_k);
                    for (int a = 0; a < n_k; ++a) g[(size_t)l * n_k + a] *= W;
                }
                oracle_ylm(lmax, d[0], d[1], d[2], yre, yim);
                for (int l = 0; l <= lmax; ++l)
                    for (int m = -l; m <= l; ++m) {
                        double complex y = yre[l * l + l + m] + I * yim[l * l + l + m];
                        for (int a = 0; a < n_k; ++a) Alm[(size_t)a * nlm + l * l + l + m] += wj * g[(size_t)l * n_k + a] * y;
                    }
                for (int l = 0; l <= lmax; ++l)
                    for (int a = 0; a < n_k; ++a)
                        for (int b = 0; b < n_k; ++b)
                            Cp[((size_t)l * n_k + a) * n_k + b] += wj * wj * g[(size_t)l * n_k + a] * g[(size_t)l * n_k + b];
                for (int a = 0; a < n_k; ++a) s0loc[a] += wj * g[a];
            }
            for (int l = 0; l <= lmax; ++l)
                for (int a = 0; a < n_k; ++a)
                    for (int b = 0; b < n_k; ++b) {
                        double s = 0.0;
                        for (int m = -l; m <= l; ++m)
                            s += creal(Alm[(size_t)a * nlm + l * l + l + m] * conj(Alm[(size_t)b * nlm + l * l + l + m]));
                        size_t q = ((size_t)l * n_k + a) * n_k + b;
                        tG[q] += wp * (4.0 * PI / (2.0 * l + 1.0)) * s;
                        tC[q] += wp * Cp[q];
                    }
            for (int a = 0; a < n_k; ++a) tS[a] += wp * s0loc[a];
        }
        cnt[tid] = c;
        free(Alm);
        free(Cp);
        free(g);
    }
    uint64_t ctot = 0;
    for (size_t q = 0; q < ng; ++q) { G[q] = 0.0; Cs[q] = 0.0; }
    for (int a = 0; a < n_k; ++a) if (S0) S0[a] = 0.0;
    for (int t = 0; t < nt; ++t) {
        const double *b = acc + (size_t)t * (2 * ng + n_k);
        for (size_t q = 0; q < ng; ++q) { G[q] += b[q]; Cs[q] += b[ng + q]; }
        if (S0) for (int a = 0; a < n_k; ++a) S0[a] += b[2 * ng + a];
        ctot += cnt[t];
    }
    free(acc);
    free(cnt);
    return ctot;
}

/* B^ab_ell for ell = 0..ell_max (Sec. 4, summary estimator), with the DDR^II
 * term from random primaries and every other random term analytic:
 *   B = (-1)^l (2l+1) / (V n_w^3) [(G_D - C_D) - s_R (G_R - C_R)]
 *       - delta_l0 / (V n_w^2) [W~^a S0^b + W~^b S0^a] + 2 delta_l0 W~^a W~^b,
 * n_w = sum(w)/V and s_R = sum(w)/sum(w_rand) (= 1/f_rand for unit weights).
 * With n_r == 0 the random-primary term is left out.  All matrix outputs are
 * [ell_max+1][n_k][n_k]; s0 and wtilde are [n_k]; any of gd..s0 may be NULL. */
int oracle_bk_ell(int64_t n, const double *pos, const double *w, int64_t n_r,
                  const double *rpos, const double *rw, double box, double r0, int n_k,
                  const double *k, int ell_max, const uint8_t *mask_d, const uint8_t *mask_r,
                  double *bk, double *gd, double *cd, double *gr, double *cr, double *s0,
                  double *wtilde, uint64_t *n_pairs_dd, uint64_t *n_pairs_rd, int nthreads)
{
    if (n < 1 || n_r < 0 || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 ||
        ell_max > ORACLE_ELL_MAX || !(r0 > 0.0) || r0 > 0.5 * box)
        return -1;
    const int nt = nthreads_or_default(nthreads);
    const size_t ng = (size_t)(ell_max + 1) * n_k * n_k;
    double *GD = calloc(ng, sizeof(double)), *CD = calloc(ng, sizeof(double));
    double *GR = calloc(ng, sizeof(double)), *CR = calloc(ng, sizeof(double));
    double *S0 = calloc((size_t)n_k, sizeof(double)), *Wt = calloc((size_t)n_k, sizeof(double));
    uint64_t cdd = bk_primary_sums(n, pos, w, mask_d, 1, n, pos, w, box, r0, n_k, k, ell_max, GD, CD, S0, nt);
    uint64_t crd = 0;
    if (n_r > 0)
        crd = bk_primary_sums(n_r, rpos, rw, mask_r, 0, n, pos, w, box, r0, n_k, k, ell_max, GR, CR, NULL, nt);
    double p1 = 0.0, pr = 0.0;
    for (int64_t i = 0; i < n; ++i) p1 += w ? w[i] : 1.0;
    for (int64_t i = 0; i < n_r; ++i) pr += rw ? rw[i] : 1.0;
    const double V = box * box * box, nw = p1 / V, sR = n_r > 0 ? p1 / pr : 0.0;
    for (int a = 0; a < n_k; ++a) Wt[a] = oracle_wtilde(r0, k[a], k[a + 1], 4.0);
    for (int l = 0; l <= ell_max; ++l)
        for (int a = 0; a < n_k; ++a)
            for (int b = 0; b < n_k; ++b) {
                size_t q = ((size_t)l * n_k + a) * n_k + b;
                double sgn = (l & 1) ? -1.0 : 1.0;
                double v = sgn * (2.0 * l + 1.0) / (V * nw * nw * nw) * ((GD[q] - CD[q]) - sR * (GR[q] - CR[q]));
                if (l == 0)
                    v += -(Wt[a] * S0[b] + Wt[b] * S0[a]) / (V * nw * nw) + 2.0 * Wt[a] * Wt[b];
                bk[q] = v;
            }
    if (gd) memcpy(gd, GD, ng * sizeof(double));
    if (cd) memcpy(cd, CD, ng * sizeof(double));
    if (gr) memcpy(gr, GR, ng * sizeof(double));
    if (cr) memcpy(cr, CR, ng * sizeof(double));
    if (s0) memcpy(s0, S0, (size_t)n_k * sizeof(double));
    if (wtilde) memcpy(wtilde, Wt, (size_t)n_k * sizeof(double));
    if (n_pairs_dd) *n_pairs_dd = cdd;
    if (n_pairs_rd) *n_pairs_rd = crd;
    free(GD); free(CD); free(GR); free(CR); free(S0); free(Wt);
    return 0;
}

/* ------------------------------------------- anisotropic bispectrum */
/* The anisotropic bispectrum (Sec. 10 names it: the sum over spherical
 * harmonics of the Sec. 4 estimators replaced by a product of harmonics of
 * different order about the fixed line of sight z).  The reading: the kernel
 * (-1)^l (2l+1) j_l j_l L_l(xhat_ij . xhat_ik) of Sec. 4 becomes
 *   s_{l1 l2} 4 pi jbar^a_{l1}(r_ij) W jbar^b_{l2}(r_ik) W
 *     sum_{mu in M(m)} Y_{l1 mu}(xhat_ij) Y*_{l2 mu}(xhat_ik),
 * M(m) = {0} for m = 0 and {m, -m} for m > 0, s_{l1 l2} = (-1)^{(l1+l2)/2}
 * for even l1 + l2 and (-1)^{(l1+l2-1)/2} for odd (the real factor of
 * (-i)^{l1+l2}; an odd l1 + l2 multipole is that factor times -i).  The
 * random integrals of Sec. 4 follow for a fixed line of sight: RRR survives
 * at l1 = l2 = m = 0 only; DDR^I at m = 0 with l2 = 0 (or l1 = 0), where it
 * is W~^b times the pair sum T^a_{l1} = sum_{i != j} w_i w_j jbar^a_{l1} W
 * Y_{l1 0}(xhat_ij) times sqrt(4 pi); DDR^II from random primaries.  Then
 *   B^{ab}_{l1 l2 m} = s 4 pi / (V n_w^3) [(G_D - C_D) - s_R (G_R - C_R)]
 *     - s sqrt(4 pi) / (V n_w^2) delta_m0 [delta_{l2 0} W~^b T^a_{l1}
 *       + delta_{l1 0} W~^a T^b_{l2}] + 2 delta_{l1 0} delta_{l2 0} delta_m0 W~^a W~^b,
 * G^{ab} = sum_p w_p sum_{mu in M(m)} A^a_{l1 mu} A^{b*}_{l2 mu} and
 * C^{ab} = sum_p w_p sum_{j != p} w_j^2 jbar^a_{l1} jbar^b_{l2} W^2
 *   sum_{mu in M(m)} Y_{l1 mu}(xhat_pj) Y*_{l2 mu}(xhat_pj) (its j = k part).
 * Summed over m at l1 = l2 = l it is the isotropic B^{ab}_l.
 * Combinations c: l1 <= l2 <= ell_max, m = 0 .. l1, in that (l1, l2, m)
 * order; outputs [n_c][n_k][n_k], t [ell_max+1][n_k].  Any of gd..t may be
 * NULL. */
int oracle_aniso_count(int ell_max)
{
    int c = 0;
    for (int l1 = 0; l1 <= ell_max; ++l1)
        for (int l2 = l1; l2 <= ell_max; ++l2) c += l1 + 1;
    return c;
}

static uint64_t bk_aniso_sums(int64_t np, const double *ppos, const double *pw, const uint8_t *mask,
                              int self_exclude, int64_t n, const double *pos, const double *w, double box,
                              double r0, int n_k, const double *k, int lmax, double *G, double *Cs, double *T,
                              int nt)
{
    const int nlm = (lmax + 1) * (lmax + 1), nc = oracle_aniso_count(lmax);
    const size_t ng = (size_t)nc * n_k * n_k, nT = (size_t)(lmax + 1) * n_k;
    int cl1[128], cl2[128], cm[128];
    {
        int c = 0;
        for (int l1 = 0; l1 <= lmax; ++l1)
            for (int l2 = l1; l2 <= lmax; ++l2)
                for (int m = 0; m <= l1; ++m) { cl1[c] = l1; cl2[c] = l2; cm[c] = m; ++c; }
    }
    double *acc = calloc((size_t)nt * (2 * ng + nT), sizeof(double));
    uint64_t *cnt = calloc((size_t)nt, sizeof(uint64_t));
    const double r02 = r0 * r0;
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *tG = acc + (size_t)tid * (2 * ng + nT), *tC = tG + ng, *tT = tC + ng;
        double complex *Alm = malloc(sizeof(double complex) * (size_t)n_k * nlm);
        double *Cp = malloc(sizeof(double) * ng);
        double *g = malloc(sizeof(double) * (size_t)(lmax + 1) * n_k);
        double yre[(ORACLE_ELL_MAX + 1) * (ORACLE_ELL_MAX + 1)], yim[(ORACLE_ELL_MAX + 1) * (ORACLE_ELL_MAX + 1)];
        uint64_t cn = 0;
#pragma omp for schedule(static)
        for (int64_t p = 0; p < np; ++p) {
            if (mask && !mask[p]) continue;
            const double wp = pw ? pw[p] : 1.0;
            memset(Alm, 0, sizeof(double complex) * (size_t)n_k * nlm);
            memset(Cp, 0, sizeof(double) * ng);
            for (int64_t j = 0; j < n; ++j) {
                if (self_exclude && j == p) continue;
                double d[3];
                for (int ax = 0; ax < 3; ++ax) d[ax] = min_image(ppos[3 * p + ax] - pos[3 * j + ax], box);
                double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                if (!(r2 < r02)) continue;
                ++cn;
                double r = sqrt(r2);
                double wj = w ? w[j] : 1.0;
                double W = oracle_window(r / r0);
                for (int l = 0; l <= lmax; ++l) {
                    jbar_all_bins(l, r, n_k, k, g + (size_t)l * n_k);
                    for (int a = 0; a < n_k; ++a) g[(size_t)l * n_k + a] *= W;
                }
                oracle_ylm(lmax, d[0], d[1], d[2], yre, yim);
                for (int l = 0; l <= lmax; ++l)
                    for (int m = -l; m <= l; ++m) {
                        double complex y = yre[l * l + l + m] + I * yim[l * l + l + m];
                        for (int a = 0; a < n_k; ++a) Alm[(size_t)a * nlm + l * l + l + m] += wj * g[(size_t)l * n_k + a] * y;
                    }
                /* j = k part: the product of the pair's own harmonics */
                for (int c = 0; c < nc; ++c) {
                    const int l1 = cl1[c], l2 = cl2[c], m = cm[c];
                    double q = 0.0;
                    for (int sgn = (m == 0 ? 1 : -1); sgn <= 1; sgn += 2) {
                        const int mu = sgn * m;
                        double complex y1 = yre[l1 * l1 + l1 + mu] + I * yim[l1 * l1 + l1 + mu];
                        double complex y2 = yre[l2 * l2 + l2 + mu] + I * yim[l2 * l2 + l2 + mu];
                        q += creal(y1 * conj(y2));
                    }
                    for (int a = 0; a < n_k; ++a)
                        for (int b = 0; b < n_k; ++b)
                            Cp[((size_t)c * n_k + a) * n_k + b] += wj * wj * g[(size_t)l1 * n_k + a] * g[(size_t)l2 * n_k + b] * q;
                }
            }
            for (int c = 0; c < nc; ++c) {
                const int l1 = cl1[c], l2 = cl2[c], m = cm[c];
                for (int a = 0; a < n_k; ++a)
                    for (int b = 0; b < n_k; ++b) {
                        double s = 0.0;
                        for (int sgn = (m == 0 ? 1 : -1); sgn <= 1; sgn += 2) {
                            const int mu = sgn * m;
                            s += creal(Alm[(size_t)a * nlm + l1 * l1 + l1 + mu] * conj(Alm[(size_t)b * nlm + l2 * l2 + l2 + mu]));
                        }
                        size_t q = ((size_t)c * n_k + a) * n_k + b;
                        tG[q] += wp * s;
                        tC[q] += wp * Cp[q];
                    }
            }
            for (int l = 0; l <= lmax; ++l)
                for (int a = 0; a < n_k; ++a) tT[(size_t)l * n_k + a] += wp * creal(Alm[(size_t)a * nlm + l * l + l]);
        }
        cnt[tid] = cn;
        free(Alm);
        free(Cp);
        free(g);
    }
    uint64_t ctot = 0;
    for (size_t q = 0; q < ng; ++q) { G[q] = 0.0; Cs[q] = 0.0; }
    if (T) for (size_t q = 0; q < nT; ++q) T[q] = 0.0;
    for (int t = 0; t < nt; ++t) {
        const double *b = acc + (size_t)t * (2 * ng + nT);
        for (size_t q = 0; q < ng; ++q) { G[q] += b[q]; Cs[q] += b[ng + q]; }
        if (T) for (size_t q = 0; q < nT; ++q) T[q] += b[2 * ng + q];
        ctot += cnt[t];
    }
    free(acc);
    free(cnt);
    return ctot;
}

int oracle_bk_aniso(int64_t n, const double *pos, const double *w, int64_t n_r, const double *rpos,
                    const double *rw, double box, double r0, int n_k, const double *k, int ell_max,
                    const uint8_t *mask_d, const uint8_t *mask_r, double *bk, double *gd, double *cd,
                    double *gr, double *cr, double *t, uint64_t *n_pairs_dd, uint64_t *n_pairs_rd, int nthreads)
{
    if (n < 1 || n_r < 0 || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 || ell_max > ORACLE_ELL_MAX ||
        !(r0 > 0.0) || r0 > 0.5 * box)
        return -1;
    const int nt = nthreads_or_default(nthreads), nc = oracle_aniso_count(ell_max);
    const size_t ng = (size_t)nc * n_k * n_k, nT = (size_t)(ell_max + 1) * n_k;
    double *GD = calloc(ng, sizeof(double)), *CD = calloc(ng, sizeof(double));
    double *GR = calloc(ng, sizeof(double)), *CR = calloc(ng, sizeof(double));
    double *TD = calloc(nT, sizeof(double)), *Wt = calloc((size_t)n_k, sizeof(double));
    uint64_t cdd = bk_aniso_sums(n, pos, w, mask_d, 1, n, pos, w, box, r0, n_k, k, ell_max, GD, CD, TD, nt);
    uint64_t crd = 0;
    if (n_r > 0) crd = bk_aniso_sums(n_r, rpos, rw, mask_r, 0, n, pos, w, box, r0, n_k, k, ell_max, GR, CR, NULL, nt);
    double p1 = 0.0, pr = 0.0;
    for (int64_t i = 0; i < n; ++i) p1 += w ? w[i] : 1.0;
    for (int64_t i = 0; i < n_r; ++i) pr += rw ? rw[i] : 1.0;
    const double V = box * box * box, nw = p1 / V, sR = n_r > 0 ? p1 / pr : 0.0;
    const double sq4pi = sqrt(4.0 * PI);
    for (int a = 0; a < n_k; ++a) Wt[a] = oracle_wtilde(r0, k[a], k[a + 1], 4.0);
    int c = 0;
    for (int l1 = 0; l1 <= ell_max; ++l1)
        for (int l2 = l1; l2 <= ell_max; ++l2)
            for (int m = 0; m <= l1; ++m, ++c) {
                const int L = l1 + l2;
                const double sgn = (((L & 1) ? (L - 1) / 2 : L / 2) & 1) ? -1.0 : 1.0;
                for (int a = 0; a < n_k; ++a)
                    for (int b = 0; b < n_k; ++b) {
                        size_t q = ((size_t)c * n_k + a) * n_k + b;
                        double v = sgn * 4.0 * PI / (V * nw * nw * nw) * ((GD[q] - CD[q]) - sR * (GR[q] - CR[q]));
                        if (m == 0) {
                            double d1 = 0.0;
                            if (l2 == 0) d1 += Wt[b] * TD[(size_t)l1 * n_k + a];
                            if (l1 == 0) d1 += Wt[a] * TD[(size_t)l2 * n_k + b];
                            v -= sgn * sq4pi / (V * nw * nw) * d1;
                            if (l1 == 0 && l2 == 0) v += 2.0 * Wt[a] * Wt[b];
                        }
                        bk[q] = v;
                    }
            }
    if (gd) memcpy(gd, GD, ng * sizeof(double));
    if (cd) memcpy(cd, CD, ng * sizeof(double));
    if (gr) memcpy(gr, GR, ng * sizeof(double));
    if (cr) memcpy(cr, CR, ng * sizeof(double));
    if (t) memcpy(t, TD, nT * sizeof(double));
    if (n_pairs_dd) *n_pairs_dd = cdd;
    if (n_pairs_rd) *n_pairs_rd = crd;
    free(GD); free(CD); free(GR); free(CR); free(TD); free(Wt);
    return 0;
}

/* ------------------------------------------ analytic DDR^II (Apps. A, B) */
/* The second data-data-random term of the bispectrum without randoms
 * (Sec. 4, eq. EII-intro; Appendix A, eq. DDRII-kernel; Appendix B): it is a
 * sum over data pairs out to 2 R0 of a kernel of the pair separation,
 *   E^{II,ab}_l(x) = (2 pi / x) int_0^R0 int_0^R0 dr1 dr2 r1 r2 beta(Delta)
 *                    g^a_l(r1) g^b_l(r2) L_l(Delta),
 *   Delta = (r1^2 + r2^2 - x^2) / (2 r1 r2),  g^a_l(r) = jbar^a_l(r) W(r/R0),
 * where beta(Delta) restricts the square to the band |r1 - r2| <= x <= r1 + r2
 * (Appendix B, last form).  Readings: E at x = 0 is its limit
 * 4 pi int_0^R0 r^2 g^a_l g^b_l dr (the band shrinks to r2 = r1, where
 * Delta = 1); E = 0 for x >= 2 R0.
 *
 * Quadrature: composite 16-point Gauss-Legendre.  Both integration ranges
 * are cut where the integrand or a limit of the inner range is not smooth --
 * the joins of W at R0/2 and 3R0/4, r1 = x (the inner range starts at
 * r2 = 0), and the values of r1 at which an inner limit |x - r1| or r1 + x
 * crosses a join of W or reaches R0 -- and every piece is split into panels
 * no wider than min(R0/8, (pi/2)/k_max). */
#define EII_NG 16

/* g^b_l(r) for all bins. */
static void eii_g(int ell, double r, double r0, int n_k, const double *k, double *g)
{
    const double W = oracle_window(r / r0);
    jbar_all_bins(ell, r, n_k, k, g);
    for (int b = 0; b < n_k; ++b) g[b] *= W;
}

/* Gauss-Legendre nodes and weights of [lo, hi] cut at cuts[] and into panels
 * no wider than hmax.  Returns the node count; xs, ws hold at least
 * EII_NG * (ceil((hi - lo) / hmax) + ncut + 1) entries. */
static int eii_nodes(double lo, double hi, const double *cuts, int ncut, double hmax,
                     const double *gx, const double *gw, double *xs, double *ws)
{
    double pts[16];
    int np = 0;
    pts[np++] = lo;
    for (int c = 0; c < ncut; ++c)
        if (cuts[c] > lo && cuts[c] < hi) pts[np++] = cuts[c];
    pts[np++] = hi;
    for (int i = 1; i < np; ++i) /* insertion sort */
        for (int j = i; j > 0 && pts[j] < pts[j - 1]; --j) {
            double t = pts[j]; pts[j] = pts[j - 1]; pts[j - 1] = t;
        }
    int n = 0;
    for (int s = 0; s + 1 < np; ++s) {
        double a = pts[s], b = pts[s + 1];
        if (!(b > a)) continue;
        int npan = (int)ceil((b - a) / hmax);
        if (npan < 1) npan = 1;
        double h = (b - a) / npan;
        for (int p = 0; p < npan; ++p) {
            double mid = a + (p + 0.5) * h, half = 0.5 * h;
            for (int q = 0; q < EII_NG; ++q) {
                xs[n] = mid + half * gx[q];
                ws[n] = half * gw[q];
                ++n;
            }
        }
    }
    return n;
}

/* E^{II,ab}_l(x) for all bins a, b: out [n_k][n_k]. */
int oracle_eii(double x, double r0, int ell, int n_k, const double *k, double *out)
{
    if (!(r0 > 0.0) || !(x >= 0.0) || ell < 0 || ell > ORACLE_ELL_MAX || n_k < 1 || n_k > ORACLE_NK_MAX)
        return -1;
    for (int q = 0; q < n_k * n_k; ++q) out[q] = 0.0;
    if (x >= 2.0 * r0) return 0;
    double gx[EII_NG], gw[EII_NG];
    gauss_legendre(EII_NG, gx, gw);
    double hmax = 0.125 * r0;
    if (0.5 * PI / k[n_k] < hmax) hmax = 0.5 * PI / k[n_k];
    const int cap = EII_NG * ((int)ceil(r0 / hmax) + 12);
    double *x1 = malloc(sizeof(double) * cap), *w1 = malloc(sizeof(double) * cap);
    double *x2 = malloc(sizeof(double) * cap), *w2 = malloc(sizeof(double) * cap);
    double *ga = malloc(sizeof(double) * n_k), *gb = malloc(sizeof(double) * n_k);
    double *H = malloc(sizeof(double) * n_k);
    const double joins[2] = {0.5 * r0, 0.75 * r0};
    if (x == 0.0) {
        int n = eii_nodes(0.0, r0, joins, 2, hmax, gx, gw, x1, w1);
        for (int i = 0; i < n; ++i) {
            double r = x1[i];
            eii_g(ell, r, r0, n_k, k, ga);
            for (int a = 0; a < n_k; ++a)
                for (int b = 0; b < n_k; ++b) out[a * n_k + b] += w1[i] * r * r * ga[a] * ga[b];
        }
        for (int q = 0; q < n_k * n_k; ++q) out[q] *= 4.0 * PI;
    } else {
        const double cuts1[10] = {0.5 * r0, 0.75 * r0, x, x - 0.5 * r0, x + 0.5 * r0,
                                  x - 0.75 * r0, x + 0.75 * r0, 0.5 * r0 - x, 0.75 * r0 - x, r0 - x};
        const double lo1 = x > r0 ? x - r0 : 0.0;
        int n1 = eii_nodes(lo1, r0, cuts1, 10, hmax, gx, gw, x1, w1);
        for (int i = 0; i < n1; ++i) {
            double r1 = x1[i];
            double lo2 = fabs(x - r1), hi2 = r1 + x < r0 ? r1 + x : r0;
            if (!(hi2 > lo2)) continue;
            int n2 = eii_nodes(lo2, hi2, joins, 2, hmax, gx, gw, x2, w2);
            for (int b = 0; b < n_k; ++b) H[b] = 0.0;
            for (int j = 0; j < n2; ++j) {
                double r2 = x2[j];
                /* Delta, with r1^2 - x^2 formed as (r1 - x)(r1 + x) */
                double D = ((r1 - x) * (r1 + x) + r2 * r2) / (2.0 * r1 * r2);
                if (D > 1.0) D = 1.0;
                if (D < -1.0) D = -1.0;
                double Lw = w2[j] * r2 * oracle_legendre(ell, D);
                eii_g(ell, r2, r0, n_k, k, gb);
                for (int b = 0; b < n_k; ++b) H[b] += Lw * gb[b];
            }
            eii_g(ell, r1, r0, n_k, k, ga);
            for (int a = 0; a < n_k; ++a)
                for (int b = 0; b < n_k; ++b) out[a * n_k + b] += w1[i] * r1 * ga[a] * H[b];
        }
        for (int q = 0; q < n_k * n_k; ++q) out[q] *= 2.0 * PI / x;
    }
    free(x1); free(w1); free(x2); free(w2); free(ga); free(gb); free(H);
    return 0;
}

/* E^{II,ab}_l on the n_x + 1 nodes x_m = m h, h = 2 R0 / n_x, l = 0..ell_max:
 * out [ell_max+1][n_k][n_k][n_x+1]. */
int oracle_eii_table(double r0, int n_k, const double *k, int ell_max, int n_x, double *out, int nthreads)
{
    if (!(r0 > 0.0) || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 || ell_max > ORACLE_ELL_MAX || n_x < 1)
        return -1;
    const int nt = nthreads_or_default(nthreads);
    const double h = 2.0 * r0 / n_x;
    const int njob = (ell_max + 1) * (n_x + 1);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(| : bad)
    for (int job = 0; job < njob; ++job) {
        int l = job / (n_x + 1), m = job % (n_x + 1);
        double *e = malloc(sizeof(double) * n_k * n_k);
        bad |= oracle_eii(m * h, r0, l, n_k, k, e) != 0;
        for (int a = 0; a < n_k; ++a)
            for (int b = 0; b < n_k; ++b)
                out[(((size_t)l * n_k + a) * n_k + b) * (n_x + 1) + m] = e[a * n_k + b];
        free(e);
    }
    return bad ? -1 : 0;
}

/* The tabulated kernel at separation r (0 <= r < 2 R0): the quintic through
 * the six nodes m-2 .. m+3 around r, m = floor(r / h), t = r / h - m
 * (six-point Lagrange interpolation), with the nodes outside the table taken
 * from the symmetry of E as a function of the pair vector (E(-x) = E(x)) and
 * from its support (E = 0 from 2 R0 on).  tab: one (a, b, l) row of n_x + 1
 * nodes. */
static double eii_interp(const double *tab, int n_x, double r, double h)
{
    double s = r / h;
    int m = (int)floor(s);
    if (m > n_x - 1) m = n_x - 1;
    double t = s - m;
    double sum = 0.0;
    for (int q = -2; q <= 3; ++q) {
        int node = m + q;
        double v;
        if (node < 0) node = -node;
        v = node > n_x ? 0.0 : tab[node];
        /* Lagrange basis of node q over the nodes -2 .. 3 */
        double num = 1.0, den = 1.0;
        for (int i = -2; i <= 3; ++i) {
            if (i == q) continue;
            num *= t - i;
            den *= q - i;
        }
        sum += v * (num / den);
    }
    return sum;
}

/* T^{ab}_l = sum_{i != j} w_i w_j E^{II,ab}_l(|x_i - x_j + n L|) over ordered
 * pairs of distinct points and every periodic image n with separation
 * < 2 R0 (squared, in double precision, as for the pair count inside R0).
 * With R0 <= L/2 every such image has n in {-1, 0, 1}^3, and the torus
 * integral over x3 of the two windows is exactly this sum over images.
 * E is the interpolated table (eii_interp).  Primaries i with mask[i] == 0 are
 * skipped.  T, l1 (sum of |term|): [ell_max+1][n_k][n_k].  *n_pairs counts
 * the ordered (pair, image) terms. */
int oracle_ddr2(int64_t n, const double *pos, const double *w, double box, double r0, int n_k,
                const double *k, int ell_max, int n_x, const double *table, const uint8_t *mask,
                double *T, double *l1, uint64_t *n_pairs, int nthreads)
{
    if (n < 1 || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 || ell_max > ORACLE_ELL_MAX ||
        !(r0 > 0.0) || r0 > 0.5 * box || n_x < 1)
        return -1;
    const int nt = nthreads_or_default(nthreads);
    const size_t ng = (size_t)(ell_max + 1) * n_k * n_k;
    const double h = 2.0 * r0 / n_x, lim2 = 4.0 * r0 * r0;
    double *acc = calloc((size_t)nt * 2 * ng, sizeof(double));
    uint64_t *cnt = calloc((size_t)nt, sizeof(uint64_t));
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *tT = acc + (size_t)tid * 2 * ng, *tL = tT + ng;
        uint64_t c = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            if (mask && !mask[i]) continue;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double wij = (w ? w[i] : 1.0) * (w ? w[j] : 1.0);
                for (int img = 0; img < 27; ++img) {
                    double d[3];
                    d[0] = pos[3 * i] - pos[3 * j] + (img / 9 - 1) * box;
                    d[1] = pos[3 * i + 1] - pos[3 * j + 1] + ((img / 3) % 3 - 1) * box;
                    d[2] = pos[3 * i + 2] - pos[3 * j + 2] + (img % 3 - 1) * box;
                    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                    if (!(r2 < lim2)) continue;
                    ++c;
                    double r = sqrt(r2);
                    for (size_t q = 0; q < ng; ++q) {
                        double v = wij * eii_interp(table + q * (n_x + 1), n_x, r, h);
                        tT[q] += v;
                        tL[q] += fabs(v);
                    }
                }
            }
        }
        cnt[tid] = c;
    }
    uint64_t ctot = 0;
    for (size_t q = 0; q < ng; ++q) { T[q] = 0.0; if (l1) l1[q] = 0.0; }
    for (int t = 0; t < nt; ++t) {
        for (size_t q = 0; q < ng; ++q) {
            T[q] += acc[(size_t)t * 2 * ng + q];
            if (l1) l1[q] += acc[(size_t)t * 2 * ng + ng + q];
        }
        ctot += cnt[t];
    }
    if (n_pairs) *n_pairs = ctot;
    free(acc);
    free(cnt);
    return 0;
}

/* B^ab_ell with the DDR^II term from the kernel E^II instead of random
 * primaries (Sec. 4 summary estimator; Appendix A, binned DDR^II):
 *   B = (-1)^l (2l+1) / (V n_w^3) [(G_D - C_D) - n_w T]
 *       - delta_l0 / (V n_w^2) [W~^a S0^b + W~^b S0^a] + 2 delta_l0 W~^a W~^b,
 * with T from oracle_ddr2 on the table `table` (n_x intervals).  The random
 * term of oracle_bk_ell, s_R (G_R - C_R), estimates n_w T by sampling the x3
 * integral at the randoms.  Outputs as oracle_bk_ell; t2 = T. */
int oracle_bk_ell_analytic(int64_t n, const double *pos, const double *w, double box, double r0, int n_k,
                           const double *k, int ell_max, int n_x, const double *table, const uint8_t *mask_d,
                           double *bk, double *gd, double *cd, double *t2, double *t2_l1, double *s0,
                           double *wtilde, uint64_t *n_pairs_dd, uint64_t *n_pairs_2r0, int nthreads)
{
    if (n < 1 || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 || ell_max > ORACLE_ELL_MAX ||
        !(r0 > 0.0) || r0 > 0.5 * box || n_x < 1)
        return -1;
    const int nt = nthreads_or_default(nthreads);
    const size_t ng = (size_t)(ell_max + 1) * n_k * n_k;
    double *GD = calloc(ng, sizeof(double)), *CD = calloc(ng, sizeof(double));
    double *T = calloc(ng, sizeof(double)), *TL = calloc(ng, sizeof(double));
    double *S0 = calloc((size_t)n_k, sizeof(double)), *Wt = calloc((size_t)n_k, sizeof(double));
    uint64_t cdd = bk_primary_sums(n, pos, w, mask_d, 1, n, pos, w, box, r0, n_k, k, ell_max, GD, CD, S0, nt);
    uint64_t c2 = 0;
    int rc = oracle_ddr2(n, pos, w, box, r0, n_k, k, ell_max, n_x, table, mask_d, T, TL, &c2, nt);
    double p1 = 0.0;
    for (int64_t i = 0; i < n; ++i) p1 += w ? w[i] : 1.0;
    const double V = box * box * box, nw = p1 / V;
    for (int a = 0; a < n_k; ++a) Wt[a] = oracle_wtilde(r0, k[a], k[a + 1], 4.0);
    for (int l = 0; l <= ell_max; ++l)
        for (int a = 0; a < n_k; ++a)
            for (int b = 0; b < n_k; ++b) {
                size_t q = ((size_t)l * n_k + a) * n_k + b;
                double sgn = (l & 1) ? -1.0 : 1.0;
                double v = sgn * (2.0 * l + 1.0) / (V * nw * nw * nw) * ((GD[q] - CD[q]) - nw * T[q]);
                if (l == 0)
                    v += -(Wt[a] * S0[b] + Wt[b] * S0[a]) / (V * nw * nw) + 2.0 * Wt[a] * Wt[b];
                bk[q] = v;
            }
    if (gd) memcpy(gd, GD, ng * sizeof(double));
    if (cd) memcpy(cd, CD, ng * sizeof(double));
    if (t2) memcpy(t2, T, ng * sizeof(double));
    if (t2_l1) memcpy(t2_l1, TL, ng * sizeof(double));
    if (s0) memcpy(s0, S0, (size_t)n_k * sizeof(double));
    if (wtilde) memcpy(wtilde, Wt, (size_t)n_k * sizeof(double));
    if (n_pairs_dd) *n_pairs_dd = cdd;
    if (n_pairs_2r0) *n_pairs_2r0 = c2;
    free(GD); free(CD); free(T); free(TL); free(S0); free(Wt);
    return rc;
}

/* ------------------------------------------------- theory side (Secs. 5, 6) */
/* Spherical Bessel j_ell(x): the power series
 *   j_l(x) = x^l / (2l+1)!! sum_s (-x^2/2)^s / (s! (2l+3)(2l+5)...(2l+2s+1))
 * below x = 5, upward recurrence above (as oracle_sph_bessel_up). */
double oracle_sph_jl(int ell, double x)
{
    if (x < U_SWITCH) {
        double t = pow(x, ell) / dfact_odd(ell), sum = 0.0;
        for (int s = 0; s < 60; ++s) {
            sum += t;
            if (fabs(t) <= 1e-18 * fabs(sum) && s > 1) break;
            t *= -0.5 * x * x / ((s + 1.0) * (2.0 * ell + 2.0 * s + 3.0));
        }
        return sum;
    }
    double j[ORACLE_ELL_MAX + 2];
    oracle_sph_bessel_up(ell, x, j);
    return j[ell];
}

/* Wigner 3j symbol (l1 l2 l3; 0 0 0) from its closed form: zero unless
 * J = l1 + l2 + l3 is even and the triangle holds; else
 *   (-1)^(J/2) sqrt((J-2l1)! (J-2l2)! (J-2l3)! / (J+1)!) (J/2)! / ((J/2-l1)! (J/2-l2)! (J/2-l3)!). */
double oracle_wigner3j_000(int l1, int l2, int l3)
{
    int J = l1 + l2 + l3;
    if (J & 1) return 0.0;
    if (l3 > l1 + l2 || l3 < abs(l1 - l2)) return 0.0;
    int g = J / 2;
    double lf = lgamma(J - 2.0 * l1 + 1) + lgamma(J - 2.0 * l2 + 1) + lgamma(J - 2.0 * l3 + 1) - lgamma(J + 2.0);
    double v = exp(0.5 * lf + lgamma(g + 1.0) - lgamma(g - l1 + 1.0) - lgamma(g - l2 + 1.0) - lgamma(g - l3 + 1.0));
    return (g & 1) ? -v : v;
}

/* omega^a_l(p; R0) = 4 pi int_0^R0 r^2 j_l(p r) jbar^a_l(r) W(r/R0) dr for all
 * bins (Sec. 6, eq. omega-ell-a-def), by composite 16-point Gauss-Legendre on
 * the three smooth pieces of W, each cut into panels no wider than
 * min(R0/8, (pi/2)/max(p, k_max)).  out [n_k]. */
int oracle_omega(double p, double r0, int ell, int n_k, const double *k, double *out)
{
    if (!(r0 > 0.0) || !(p >= 0.0) || ell < 0 || ell > ORACLE_ELL_MAX || n_k < 1 || n_k > ORACLE_NK_MAX)
        return -1;
    double gx[EII_NG], gw[EII_NG];
    gauss_legendre(EII_NG, gx, gw);
    double kmax = k[n_k] > p ? k[n_k] : p;
    double hmax = 0.125 * r0;
    if (0.5 * PI / kmax < hmax) hmax = 0.5 * PI / kmax;
    const int cap = EII_NG * ((int)ceil(r0 / hmax) + 4);
    double *xs = malloc(sizeof(double) * cap), *ws = malloc(sizeof(double) * cap), *g = malloc(sizeof(double) * n_k);
    const double joins[2] = {0.5 * r0, 0.75 * r0};
    int n = eii_nodes(0.0, r0, joins, 2, hmax, gx, gw, xs, ws);
    for (int a = 0; a < n_k; ++a) out[a] = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = xs[i];
        eii_g(ell, r, r0, n_k, k, g);
        double f = ws[i] * r * r * oracle_sph_jl(ell, p * r);
        for (int a = 0; a < n_k; ++a) out[a] += f * g[a];
    }
    for (int a = 0; a < n_k; ++a) out[a] *= 4.0 * PI;
    free(xs); free(ws); free(g);
    return 0;
}

/* Windowed power-spectrum multipoles of a model 2PCF (Sec. 5):
 *   P^a_l(R0) = 4 pi (-i)^l int r^2 xi_l(r) W(r/R0) jbar^a_l(r) dr,
 * for even l = 0, 2, .., ell_max, with the integral taken as the caller's
 * quadrature sum over nodes r[m] with weights wr[m] (m < n_r):
 *   P^a_l = 4 pi (-i)^l sum_m wr[m] r[m]^2 xi[l/2][m] W(r[m]/R0) jbar^a_l(r[m]).
 * xi [ell_max/2+1][n_r]; out [ell_max/2+1][n_k]. */
int oracle_pk_window_theory(double r0, int n_k, const double *k, int ell_max, int n_r, const double *r,
                            const double *wr, const double *xi, double *out)
{
    if (!(r0 > 0.0) || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 || ell_max > ORACLE_ELL_MAX || (ell_max & 1) ||
        n_r < 1)
        return -1;
    const int n_ell = ell_max / 2 + 1;
    double g[ORACLE_NK_MAX];
    for (int li = 0; li < n_ell; ++li) {
        const int ell = 2 * li;
        const double phase = (li & 1) ? -1.0 : 1.0; /* (-i)^l for even l */
        for (int a = 0; a < n_k; ++a) out[li * n_k + a] = 0.0;
        for (int m = 0; m < n_r; ++m) {
            eii_g(ell, r[m], r0, n_k, k, g);
            const double f = wr[m] * r[m] * r[m] * xi[(size_t)li * n_r + m];
            for (int a = 0; a < n_k; ++a) out[li * n_k + a] += f * g[a];
        }
        for (int a = 0; a < n_k; ++a) out[li * n_k + a] *= 4.0 * PI * phase;
    }
    return 0;
}

/* Gaussian intrinsic covariance of the binned multipoles (Sec. 6, eq.
 * cov-int, for even l, l' <= ell_max):
 *   C^ab_ll' = 2 (2l+1)(2l'+1)/V int p^2 dp/(2 pi^2) omega^a_l(p) omega^b_l'(p) Q_ll'(p),
 *   Q_ll'(p) = sum_{L, l1, l2} (2L+1) (l l' L; 0 0 0)^2 (l1 l2 L; 0 0 0)^2 P_l1(p) P_l2(p),
 * with the p integral the caller's quadrature sum over nodes p[i], weights
 * wp[i] (i < n_p), and pk [n_ell][n_p] the model multipoles P_l1(p[i]) for
 * even l1 = 0 .. ell_max (higher multipoles of P taken as zero).
 * out [n_ell][n_k][n_ell][n_k]: entry ((l n_k + a) n_ell + l') n_k + b. */
int oracle_cov_gauss(double r0, double volume, int n_k, const double *k, int ell_max, int n_p, const double *p,
                     const double *wp, const double *pk, double *out, int nthreads)
{
    if (!(r0 > 0.0) || !(volume > 0.0) || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 ||
        ell_max > ORACLE_ELL_MAX || (ell_max & 1) || n_p < 1)
        return -1;
    const int n_ell = ell_max / 2 + 1, nt = nthreads_or_default(nthreads);
    const size_t nout = (size_t)n_ell * n_k * n_ell * n_k;
    /* omega^a_l at every node */
    double *om = malloc(sizeof(double) * (size_t)n_p * n_ell * n_k);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int i = 0; i < n_p; ++i)
        for (int li = 0; li < n_ell; ++li) oracle_omega(p[i], r0, 2 * li, n_k, k, om + ((size_t)i * n_ell + li) * n_k);
    for (size_t q = 0; q < nout; ++q) out[q] = 0.0;
    for (int i = 0; i < n_p; ++i) {
        for (int li = 0; li < n_ell; ++li)
            for (int lj = 0; lj < n_ell; ++lj) {
                const int l = 2 * li, lp = 2 * lj;
                double Q = 0.0;
                for (int L = 0; L <= 2 * ORACLE_ELL_MAX; L += 2) {
                    double t1 = oracle_wigner3j_000(l, lp, L);
                    if (t1 == 0.0) continue;
                    double s = 0.0;
                    for (int m1 = 0; m1 < n_ell; ++m1)
                        for (int m2 = 0; m2 < n_ell; ++m2) {
                            double t2 = oracle_wigner3j_000(2 * m1, 2 * m2, L);
                            s += t2 * t2 * pk[(size_t)m1 * n_p + i] * pk[(size_t)m2 * n_p + i];
                        }
                    Q += (2.0 * L + 1.0) * t1 * t1 * s;
                }
                const double f = 2.0 * (2.0 * l + 1.0) * (2.0 * lp + 1.0) / volume * wp[i] * p[i] * p[i] /
                                 (2.0 * PI * PI) * Q;
                for (int a = 0; a < n_k; ++a)
                    for (int b = 0; b < n_k; ++b)
                        out[(((size_t)li * n_k + a) * n_ell + lj) * n_k + b] +=
                            f * om[((size_t)i * n_ell + li) * n_k + a] * om[((size_t)i * n_ell + lj) * n_k + b];
            }
    }
    free(om);
    return 0;
}

/* Poisson two-point covariance of the binned multipoles (Sec. 6, eq.
 * cov-poiss, the 2C term), even l, l' <= ell_max:
 *   C^ab_ll' = 2/(n^2 V) (2l+1)(2l'+1) (-i)^(l+l') 4 pi int x^2 W^2 jbar^a_l jbar^b_l'
 *              [delta_ll'/(2l+1) + sum_L (L l l'; 0 0 0)^2 xi_L(x)] dx,
 * with the x integral the caller's quadrature (nodes r[m] in [0, R0],
 * weights wr[m]) and xi [ell_max/2+1][n_r] the model multipoles xi_L(r[m]) for
 * even L <= ell_max (higher ones taken as zero).  Reading: the prefactor 2
 * (the paper prints 4 here and 2 elsewhere); with xi = 0 it is the
 * infinite-volume limit of the exact fixed-N variance of the estimator.
 * out [n_ell][n_k][n_ell][n_k]. */
int oracle_cov_poisson2(double r0, double nbar, double volume, int n_k, const double *k, int ell_max, int n_r,
                        const double *r, const double *wr, const double *xi, double *out)
{
    if (!(r0 > 0.0) || !(nbar > 0.0) || !(volume > 0.0) || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 ||
        ell_max > ORACLE_ELL_MAX || (ell_max & 1) || n_r < 1)
        return -1;
    const int n_ell = ell_max / 2 + 1;
    double *g = malloc(sizeof(double) * (size_t)n_ell * n_r * n_k);
    for (int li = 0; li < n_ell; ++li)
        for (int m = 0; m < n_r; ++m) eii_g(2 * li, r[m], r0, n_k, k, g + ((size_t)li * n_r + m) * n_k);
    for (int li = 0; li < n_ell; ++li)
        for (int lj = 0; lj < n_ell; ++lj) {
            const int l = 2 * li, lp = 2 * lj;
            const double ph = ((li + lj) & 1) ? -1.0 : 1.0; /* (-i)^(l+l') for even l, l' */
            const double pref = 2.0 / (nbar * nbar * volume) * (2.0 * l + 1.0) * (2.0 * lp + 1.0) * ph * 4.0 * PI;
            for (int a = 0; a < n_k; ++a)
                for (int b = 0; b < n_k; ++b) {
                    double s = 0.0;
                    for (int m = 0; m < n_r; ++m) {
                        double br = (li == lj) ? 1.0 / (2.0 * l + 1.0) : 0.0;
                        for (int L = 0; L < n_ell; ++L) {
                            double t = oracle_wigner3j_000(2 * L, l, lp);
                            br += t * t * xi[(size_t)L * n_r + m];
                        }
                        s += wr[m] * r[m] * r[m] * g[((size_t)li * n_r + m) * n_k + a] *
                             g[((size_t)lj * n_r + m) * n_k + b] * br;
                    }
                    out[(((size_t)li * n_k + a) * n_ell + lj) * n_k + b] = pref * s;
                }
        }
    free(g);
    return 0;
}

/* Poisson three-point covariance of the binned multipoles (Sec. 6, eq.
 * cov-poiss, the 3C term), even l, l' <= ell_max:
 *   C^ab_ll' = 4/(n V) [W~^a W~^b d_l0 d_l'0 + W~^a P^b_l' d_l0 + W~^b P^a_l d_l'0 + B^ab_l d_ll']
 *            + 4/(n V) (2l+1)(2l'+1)(-1)^l sum_L (L l l'; 0 0 0)^2
 *                int p^2 dp/(2 pi^2) P_L(p) omega^a_l(p) omega^b_l'(p),
 * with the p integral the caller's quadrature (nodes p[i], weights wp[i]),
 * pk [ell_max/2+1][n_p] the model multipoles P_L(p[i]) for even L <= ell_max
 * (higher ones taken as zero), pbin [ell_max/2+1][n_k] the windowed binned
 * multipoles P^a_l and bk [ell_max/2+1][n_k][n_k] the binned bispectrum
 * B^ab_l at even l (either NULL: zero).  The B term is added as printed.
 * out [n_ell][n_k][n_ell][n_k]. */
int oracle_cov_poisson3(double r0, double nbar, double volume, int n_k, const double *k, int ell_max, int n_p,
                        const double *p, const double *wp, const double *pk, const double *pbin, const double *bk,
                        double *out, int nthreads)
{
    if (!(r0 > 0.0) || !(nbar > 0.0) || !(volume > 0.0) || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 ||
        ell_max > ORACLE_ELL_MAX || (ell_max & 1) || n_p < 1)
        return -1;
    const int n_ell = ell_max / 2 + 1, nt = nthreads_or_default(nthreads);
    const double f0 = 4.0 / (nbar * volume);
    double Wt[ORACLE_NK_MAX];
    for (int a = 0; a < n_k; ++a) Wt[a] = oracle_wtilde(r0, k[a], k[a + 1], 4.0);
    double *om = malloc(sizeof(double) * (size_t)n_p * n_ell * n_k);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int i = 0; i < n_p; ++i)
        for (int li = 0; li < n_ell; ++li) oracle_omega(p[i], r0, 2 * li, n_k, k, om + ((size_t)i * n_ell + li) * n_k);
    for (int li = 0; li < n_ell; ++li)
        for (int lj = 0; lj < n_ell; ++lj) {
            const int l = 2 * li, lp = 2 * lj;
            for (int a = 0; a < n_k; ++a)
                for (int b = 0; b < n_k; ++b) {
                    double s = 0.0;
                    for (int i = 0; i < n_p; ++i) {
                        double pl = 0.0;
                        for (int L = 0; L < n_ell; ++L) {
                            double t = oracle_wigner3j_000(2 * L, l, lp);
                            pl += t * t * pk[(size_t)L * n_p + i];
                        }
                        s += wp[i] * p[i] * p[i] / (2.0 * PI * PI) * pl * om[((size_t)i * n_ell + li) * n_k + a] *
                             om[((size_t)i * n_ell + lj) * n_k + b];
                    }
                    double c = f0 * (2.0 * l + 1.0) * (2.0 * lp + 1.0) * ((l & 1) ? -1.0 : 1.0) * s;
                    if (li == 0 && lj == 0) c += f0 * Wt[a] * Wt[b];
                    if (pbin && li == 0) c += f0 * Wt[a] * pbin[(size_t)lj * n_k + b];
                    if (pbin && lj == 0) c += f0 * Wt[b] * pbin[(size_t)li * n_k + a];
                    if (bk && li == lj) c += f0 * bk[((size_t)li * n_k + a) * n_k + b];
                    out[(((size_t)li * n_k + a) * n_ell + lj) * n_k + b] = c;
                }
        }
    free(om);
    return 0;
}

/* Non-Gaussian intrinsic covariance of the binned multipoles (Sec. 6, the
 * 4C^NG term), even l, l' <= ell_max:
 *   C^ab_ll' = (2l+1)(2l'+1)/V (-1)^(l+l') sum_i sum_j u_i u_j T_ll'(p_i, p_j)
 *              omega^a_l(p_i) omega^b_l'(p_j),   u_i = wp[i] p_i^2 / (2 pi^2),
 * the double p integral as the caller's quadrature (nodes p[i], weights
 * wp[i]) and tbar [n_ell][n_ell][n_p][n_p] the collapsed-trispectrum
 * multipoles T_ll'(p_i, p_j).  out [n_ell][n_k][n_ell][n_k]. */
int oracle_cov_nongauss(double r0, double volume, int n_k, const double *k, int ell_max, int n_p, const double *p,
                        const double *wp, const double *tbar, double *out, int nthreads)
{
    if (!(r0 > 0.0) || !(volume > 0.0) || n_k < 1 || n_k > ORACLE_NK_MAX || ell_max < 0 ||
        ell_max > ORACLE_ELL_MAX || (ell_max & 1) || n_p < 1)
        return -1;
    const int n_ell = ell_max / 2 + 1, nt = nthreads_or_default(nthreads);
    double *om = malloc(sizeof(double) * (size_t)n_p * n_ell * n_k);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int i = 0; i < n_p; ++i)
        for (int li = 0; li < n_ell; ++li) oracle_omega(p[i], r0, 2 * li, n_k, k, om + ((size_t)i * n_ell + li) * n_k);
    for (int li = 0; li < n_ell; ++li)
        for (int lj = 0; lj < n_ell; ++lj) {
            const int l = 2 * li, lp = 2 * lj;
            const double pref = (2.0 * l + 1.0) * (2.0 * lp + 1.0) / volume * (((l + lp) & 1) ? -1.0 : 1.0);
            const double *T = tbar + ((size_t)li * n_ell + lj) * n_p * n_p;
            for (int a = 0; a < n_k; ++a)
                for (int b = 0; b < n_k; ++b) {
                    double s = 0.0;
                    for (int i = 0; i < n_p; ++i) {
                        const double ui = wp[i] * p[i] * p[i] / (2.0 * PI * PI);
                        for (int j = 0; j < n_p; ++j) {
                            const double uj = wp[j] * p[j] * p[j] / (2.0 * PI * PI);
                            s += ui * uj * T[(size_t)i * n_p + j] * om[((size_t)i * n_ell + li) * n_k + a] *
                                 om[((size_t)j * n_ell + lj) * n_k + b];
                        }
                    }
                    out[(((size_t)li * n_k + a) * n_ell + lj) * n_k + b] = pref * s;
                }
        }
    free(om);
    return 0;
}

