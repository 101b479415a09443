/*
 * hipster.h -- C ABI of the MI355X pair-sweep library for the periodic-box
 * small-scale power-spectrum and bispectrum estimators of Philcox (2020),
 * "A Faster Fourier Transform?", arXiv:2005.01739.
 *
 * The problem, as the paper states it: N tracer positions (optionally with
 * weights w_i entering pair counts as w_i w_j, Sec. 2 footnote) in a periodic
 * cube of side L (volume V = L^3), a truncation radius R0 with the smooth
 * window W(r/R0) (Sec. 2, eq. window_defn), k-bins given by their edges
 * (Sec. 3, eq. pk-binned) and Legendre multipoles ell about a fixed line of
 * sight (Sec. 2; a box axis for a simulation).
 *
 *   hipster_pk_ell: P^a_ell = (-i)^ell (2 ell+1)/(n^2 V) sum_{i!=j} W jbar^a_ell L_ell
 *                   - delta_{ell 0} W~^a          (Sec. 3, binned estimator)
 *   hipster_bk_ell: B^ab_ell from per-primary A^a_lm and C^ab_ell (Sec. 4,
 *                   eq. AC-def and the summary estimator), with the DDR^II term
 *                   from caller-supplied random primaries and all other random
 *                   terms analytic.
 *   hipster_bk_ell_analytic: the same with the DDR^II term from the kernel
 *                   E^II (Appendices A, B): no randoms at all.
 *
 * Conventions.  Pairs (i, j), i != j by index, separated by the minimum
 * periodic image; a pair counts iff r^2 < R0^2 in double precision.  With
 * weights, the density n is read as n_w = sum(w)/V and the random-primary
 * scale 1/f_rand as sum(w)/sum(w_rand).
 *
 * Errors.  Every call returns a hipster_status; HIPSTER_OK is 0.  All
 * arguments are checked before any device work; outputs are written only on
 * HIPSTER_OK.  hipster_last_error() gives a message for the last failure on a
 * context.  No C++ exception crosses this interface.
 *
 * Ownership.  The caller owns every input and output buffer; the library
 * never frees or modifies them.  A context owns its device scratch memory
 * (grown on demand, released by hipster_destroy).  One context serves one
 * host thread and one HIP stream at a time.
 *
 * Synchrony.  Calls return when the host outputs are valid.  Device work is
 * ordered on the context's stream; device input pointers must be valid on
 * that stream (pass torch.cuda.current_stream().cuda_stream to share torch's).
 */
#ifndef HIPSTER_H
#define HIPSTER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HIPSTER_OK = 0,
  HIPSTER_EINVAL = 1,       /* NULL pointer, bad enum, N < 2, bad sizes */
  HIPSTER_EDOMAIN = 2,      /* R0 outside (0, L/2], edges not increasing, ell out of range */
  HIPSTER_EOUTOFBOX = 3,    /* a coordinate is not finite or not in [0, L) */
  HIPSTER_ENOMEM = 4,       /* device allocation failed or exceeds the context cap */
  HIPSTER_EHIP = 5,         /* a HIP runtime call failed; see hipster_last_error */
  HIPSTER_EUNSUPPORTED = 6  /* a size beyond the compiled limits */
} hipster_status;

typedef enum { HIPSTER_F32 = 0, HIPSTER_F64 = 1 } hipster_dtype;

/* Arithmetic of the pair weights.  MIXED: geometry, phase reduction, sine
 * and cosine (table-driven) and all accumulation in double precision, the
 * sine integral's auxiliary functions in single precision; it requires
 * k_edges[n_k] * R0 <= 1e6 (the table reduction's exact range), else
 * HIPSTER_EUNSUPPORTED.  FP64: every step in double precision, no limit.
 * TABLE (hipster_pk_ell and hipster_pk_survey): the pair sum of Sec. 3 with jbar^a_l(r) taken
 * from its quintic interpolant on n_c = max(64, 64 ceil(k_max R0 / 8.32))
 * intervals of [0, R0] (k_max h <= 0.13, interpolation error ~2.4e-8 of
 * jbar), built once per (R0, bins, ell_max) in double precision; each pair
 * adds w_i w_j W(r/R0) L_l(mu) times its six Lagrange weights to a 64-bit
 * fixed-point histogram per l, which is then contracted with the table.  The
 * cost per pair no longer grows with n_k; pair counts stay exact and the sums
 * do not depend on the order of the adds.  The histograms must fit the
 * device's LDS: (ell_max/2 + 1)(n_c + 3) <= ~16000 nodes, else
 * HIPSTER_EUNSUPPORTED.  diag->eii_nodes reports n_c. */
typedef enum { HIPSTER_MIXED = 0, HIPSTER_FP64 = 1, HIPSTER_TABLE = 2 } hipster_precision;

/* A catalogue.  pos: n x 3 row-major coordinates of `dtype`, each in [0, L).
 * w: n weights of `dtype`, or NULL for unit weights.  on_device: 1 if pos and
 * w are device pointers (HIP, same device as the context), 0 if host. */
typedef struct {
  int64_t n;
  int32_t dtype;
  int32_t on_device;
  const void *pos;
  const void *w;
} hipster_points;

/* Estimator parameters.  k_edges: n_k + 1 strictly increasing host doubles,
 * k_edges[0] >= 0; n_k <= 128 for P, <= 64 for B (<= 16 for the analytic
 * DDR^II form and for B's FP64 form).  ell_max: P uses even ell = 0, 2, ..,
 * ell_max (ell_max even, <= 6); B uses ell = 0 .. ell_max (<= 6).  The limit 6
 * covers every multipole the paper evaluates (B to ell = 6 in Sec. 9); larger
 * ell_max is HIPSTER_EDOMAIN.  los_axis: 0, 1 or 2 (P only).
 * primary_mask: NULL, or n host bytes; only primaries i with mask[i] != 0
 * contribute their ordered pairs (i, j) -- a hook for checking a subset of a
 * large catalogue against a brute-force reference. */
typedef struct {
  double box;
  double r0;
  int32_t n_k;
  int32_t ell_max;
  const double *k_edges;
  int32_t los_axis;
  int32_t precision;
  const uint8_t *primary_mask;
  const uint8_t *random_mask; /* B only: same role for the random primaries */
} hipster_params;

/* Optional diagnostics (host memory, caller-allocated; any pointer may be
 * NULL).  For P: raw [n_ell][n_k] = the pair sums S^a_ell before
 * normalisation.  For B: gd, cd, gr, cr [ell_max+1][n_k][n_k] = the data and
 * random primary sums of w_p (4 pi/(2l+1)) sum_m A^a_lm A^b_lm and of
 * w_p C^ab_l; s0 [n_k] = sum_{i!=j} w_i w_j jbar^b_0 W.  wtilde [n_k] = W~^a.
 * l1_mass: the size against which a cancelling bin's error is judged.  For
 * hipster_pk_ell, [n_ell][n_k] = sum over ordered pairs of
 * |w_i w_j (2l+1) W jbar^a_l L_l(mu)|, the L1 mass of raw, evaluated in
 * double precision by an extra sweep over the pairs (requested only when the
 * pointer is set; its time is not in ms_sweep).  For hipster_bk_ell(_analytic),
 * [ell_max+1][n_k][n_k] = (2l+1)/(V n_w^3) [sqrt(G_D^aa G_D^bb) +
 * sqrt(C_D^aa C_D^bb) + s_R (sqrt(G_R^aa G_R^bb) + sqrt(C_R^aa C_R^bb))]
 * + delta_l0 [(W~^a |S0^b| + W~^b |S0^a|)/(V n_w^2) + 2 W~^a W~^b], a
 * Cauchy-Schwarz bound on the terms of B^ab_l (with n_w |T^ab| in place of the
 * random-primary Gram in the analytic form).  Unused by hipster_pk_survey.
 * Timings are wall-clock milliseconds of the device work measured with HIP
 * events on the context stream. */
typedef struct {
  uint64_t n_pairs;       /* ordered data-data pairs inside R0 */
  uint64_t n_pairs_rand;  /* ordered random-data pairs inside R0 (B) */
  double *raw;
  double *gd, *cd, *gr, *cr, *s0;
  double *wtilde;
  double ms_build;   /* cell lists */
  double ms_pairs;   /* pair enumeration */
  double ms_sweep;   /* pair-weight kernels (the dominant cost) */
  double ms_total;   /* whole call */
  uint64_t sweep_launches; /* number of pair-weight kernel launches in ms_sweep */
  uint64_t n_pairs_rr;    /* survey power spectrum: ordered random-random pairs inside R0 */
  double ms_sweep_far;    /* P, mixed form: the far-pair kernel's part of ms_sweep */
  uint64_t n_pairs_far;   /* P, mixed form: unordered pairs swept by the far-pair kernel */
  double ms_eii_table;    /* B analytic: building the E^II table (0 when the context reused it) */
  double ms_ddr2;         /* B analytic: the 2 R0 pair sweep and its contraction with the table */
  uint64_t n_pairs_2r0;   /* B analytic: ordered (pair, periodic image) terms inside 2 R0 */
  int64_t eii_nodes;      /* B analytic: the table's n_x (intervals over [0, 2 R0]) */
  double ms_cterm;        /* B, mixed form: the C-term pair sweep of the data primaries */
  double *l1_mass;        /* see above */
  uint64_t n_rand;        /* B: random primaries used (given or generated) */
} hipster_diag;

typedef struct hipster_ctx hipster_ctx;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t or
 * NULL for the default stream.  Returns HIPSTER_EHIP if the device is absent. */
hipster_status hipster_create(hipster_ctx **out, int device, void *hip_stream);

/* Release the context and its device memory.  NULL is ignored. */
void hipster_destroy(hipster_ctx *ctx);

/* Power-spectrum multipoles (Sec. 3, binned estimator).
 * pk: host output, [ell_max/2 + 1][n_k] doubles, rows ell = 0, 2, .. */
hipster_status hipster_pk_ell(hipster_ctx *ctx, const hipster_points *pts,
                              const hipster_params *prm, double *pk, hipster_diag *diag);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and outputs as hipster_pk_ell, with every device buffer taken
 * from a static 256 MiB workspace that each device holds from the library's
 * load until the process ends; the call makes no hipMalloc or hipFree and
 * creates no HIP events (the diag timings read 0).  Inputs and outputs are
 * the caller's, as for hipster_pk_ell.  The pair stream is cut into as many
 * chunks as the workspace needs, so sums agree with hipster_pk_ell to
 * rounding.  A call whose cell lists, or one cell tile's pairs, do not fit
 * (about 75 B per point and 70 B per cell; some 2e6 points at most) returns
 * HIPSTER_ENOMEM with a message; diag->l1_mass must be NULL
 * (HIPSTER_EUNSUPPORTED otherwise).  All calls on one device share its
 * workspace: calls that overlap on one device race. */
hipster_status hipster_pk_ell_noalloc(hipster_ctx *ctx, const hipster_points *pts,
                                      const hipster_params *prm, double *pk, hipster_diag *diag);

/* Bispectrum multipoles (Sec. 4, summary estimator).  The DDR^II term is
 * sampled with uniform random primaries (Sec. 4, a random catalogue f_rand
 * times the size of the data): randoms, if non-NULL with n > 0, is that
 * catalogue (f_rand and seed are then ignored); otherwise the library draws
 * n_R = llround(f_rand * data->n) unit-weight points on the device, point i
 * taking block i + 1 of the Philox4x64-10 counter-based generator (Salmon et
 * al. 2011) with key (seed, 0) and the counter starting at 0 -- the stream of
 * numpy's Philox(key=[seed, 0]) -- as x_d = L * (word_d >> 11) * 2^-53,
 * d = 0, 1, 2 (a coordinate that rounds to L becomes 0).  With no catalogue
 * and f_rand <= 0 (or not finite) the call returns HIPSTER_EINVAL: the term
 * is never dropped (hipster_bk_ell_analytic computes it without randoms).
 * diag->n_rand reports n_R.  bk: host output, [ell_max + 1][n_k][n_k]
 * doubles (symmetric in a, b). */
hipster_status hipster_bk_ell(hipster_ctx *ctx, const hipster_points *data,
                              const hipster_points *randoms, double f_rand, uint64_t seed,
                              const hipster_params *prm, double *bk, hipster_diag *diag);

/* Anisotropic bispectrum multipoles about the line of sight z (Sec. 10: the
 * Sec. 4 estimators with the sum over harmonics of one order replaced by a
 * product of harmonics of different orders).  The reading:
 *   B^{ab}_{l1 l2 m} = s 4 pi / (V n_w^3) [(G_D - C_D) - s_R (G_R - C_R)]
 *     - s sqrt(4 pi) / (V n_w^2) delta_m0 [delta_{l2 0} W~^b T^a_{l1} + delta_{l1 0} W~^a T^b_{l2}]
 *     + 2 delta_{l1 0} delta_{l2 0} delta_m0 W~^a W~^b,
 * G = sum_p w_p sum_{mu = +-m} A^a_{l1 mu} A^b_{l2 mu} (A as for hipster_bk_ell,
 * real orthonormal harmonics), C its j = k part, T^a_l = sum_p w_p A^a_{l0}
 * over data primaries, s the real factor of (-i)^{l1+l2} ((-1)^{(l1+l2)/2},
 * or (-1)^{(l1+l2-1)/2} when l1 + l2 is odd: that multipole is s(...) times -i).
 * Summed over m at l1 = l2 = l it is hipster_bk_ell's B^{ab}_l.  Random
 * primaries as for hipster_bk_ell (a given catalogue, or f_rand and seed).
 * Mixed form only (HIPSTER_FP64 gives HIPSTER_EUNSUPPORTED: C comes from
 * fixed-point r-histograms of w_p w_q^2 W^2 P_L(mu), one per L, contracted with
 * tables of jbar^a_{l1} jbar^b_{l2}), n_k <= 16, ell_max <= 4.
 * bk: host output [n_c][n_k][n_k], the combinations c = (l1, l2, m) with
 * l1 <= l2 <= ell_max and m = 0 .. l1 in that order (n_c = 35 at ell_max 4);
 * B^{ab}_{l1 l2 m} = B^{ba}_{l2 l1 m} gives the others.  diag: the pair
 * counts, n_rand, wtilde and the timings (ms_sweep: the two sweeps; ms_cterm:
 * the C-term histograms); the other arrays are not filled. */
hipster_status hipster_bk_aniso(hipster_ctx *ctx, const hipster_points *data, const hipster_points *randoms,
                                double f_rand, uint64_t seed, const hipster_params *prm, double *bk,
                                hipster_diag *diag);

/* Bispectrum multipoles with the DDR^II term computed without randoms
 * (Sec. 4, eq. EII-intro; Appendix A, eq. DDRII-kernel and its binned form;
 * Appendix B): the random-primary sum of hipster_bk_ell,
 * s_R sum_r [(4 pi/(2l+1)) sum_m A A* - C], is replaced by the x3 integral it
 * samples, n_w T^ab_l with
 *   T^ab_l = sum_{i != j} w_i w_j E^{II,ab}_l(|x_i - x_j + n L|)
 * over ordered pairs of distinct data points and every periodic image with
 * separation < 2 R0 (double-precision r^2 predicate, as for R0), and
 *   E^{II,ab}_l(x) = (2 pi / x) int int dr1 dr2 r1 r2 g^a_l(r1) g^b_l(r2) L_l(Delta)
 * over the band |r1 - r2| <= x <= r1 + r2 of [0, R0]^2, g^a_l = jbar^a_l W,
 * Delta = (r1^2 + r2^2 - x^2)/(2 r1 r2).  As the paper suggests, E is
 * tabulated (double precision, composite Gauss-Legendre) on the nodes
 * x_m = m h, h = 2 R0 / n_x, m = 0..n_x, and interpolated per pair by the
 * quintic through the nodes m-2..m+3 around x (m = floor(x/h); E(-x) = E(x),
 * nodes at and beyond 2 R0 hold 0).  The interpolation error is about
 * 5e-3 (k_max h)^6 of the kernel.
 * n_x: table intervals, 0 for the default (the smallest multiple of 64 with
 * k_max h <= 0.15, at least 64, at most 8192); 2 <= n_x <= 8192 and the device
 * must hold an (n_x + 1)-entry double histogram in one workgroup's LDS, else
 * HIPSTER_EUNSUPPORTED.  k_edges[n_k] * R0 <= 1e6 (HIPSTER_EUNSUPPORTED).
 * The table is cached in the context and reused while (R0, n_x, ell_max,
 * k_edges) stay the same.  Other arguments, output and errors as
 * hipster_bk_ell; prm->random_mask is ignored.  In diag: gr = T, cr = 0,
 * n_pairs_rand = 0, n_pairs_2r0, ms_eii_table, ms_ddr2, eii_nodes.  The pair
 * sums go through 64-bit fixed-point histograms, so repeated calls give the
 * same bits. */
hipster_status hipster_bk_ell_analytic(hipster_ctx *ctx, const hipster_points *data, const hipster_params *prm,
                                       int32_t n_x, double *bk, hipster_diag *diag);

/* The E^{II,ab}_l table of hipster_bk_ell_analytic: table (host,
 * caller-allocated) [ell_max+1][n_k][n_k][n_x+1] doubles, entry
 * ((l n_k + a) n_k + b)(n_x + 1) + m = E^{II,ab}_l(m 2 R0 / n_x), l = 0..ell_max.
 * r0, n_k, k_edges, ell_max as in hipster_params (n_k <= 16, ell_max <= 6);
 * n_x >= 2 as in hipster_bk_ell_analytic (0 is not accepted here).  Errors:
 * HIPSTER_EINVAL (NULL pointers), HIPSTER_EDOMAIN (R0 <= 0, bad edges or
 * ell_max), HIPSTER_EUNSUPPORTED (sizes). */
hipster_status hipster_eii_table(hipster_ctx *ctx, double r0, int32_t n_k, const double *k_edges, int32_t ell_max,
                                 int32_t n_x, double *table);

/* Theory side (Secs. 5, 6), double precision throughout.  r0, n_k, k_edges
 * and ell_max as in hipster_params (n_k <= 128); all arrays are host memory
 * owned by the caller; the integrals over r or p that the paper leaves to the
 * user are the caller's quadrature (nodes and weights).  Errors:
 * HIPSTER_EINVAL (NULL pointers, counts < 1), HIPSTER_EDOMAIN (R0 <= 0, bad
 * edges, ell_max outside [0, 6] (or odd where even multipoles are meant),
 * p < 0, r outside [0, R0], volume <= 0), HIPSTER_EUNSUPPORTED
 * (max(p, k_max) R0 > 1e6). */

/* omega^a_l(p; R0) = 4 pi int_0^R0 r^2 j_l(p r) jbar^a_l(r) W(r/R0) dr (Sec. 6,
 * eq. omega-ell-a-def) at n_p momenta p, for l = 0..ell_max.
 * out: [ell_max+1][n_p][n_k]. */
hipster_status hipster_omega(hipster_ctx *ctx, double r0, int32_t n_k, const double *k_edges, int32_t ell_max,
                             int32_t n_p, const double *p, double *out);

/* Windowed power-spectrum multipoles of a model 2PCF (Sec. 5):
 *   P^a_l(R0) = 4 pi (-i)^l int r^2 xi_l(r) W(r/R0) jbar^a_l(r) dr, l = 0, 2, .., ell_max,
 * as the sum over the caller's quadrature nodes r[m] in [0, R0] with weights
 * wr[m]: xi [ell_max/2+1][n_r] holds xi_l(r[m]).  out: [ell_max/2+1][n_k]. */
hipster_status hipster_pk_window_theory(hipster_ctx *ctx, double r0, int32_t n_k, const double *k_edges,
                                        int32_t ell_max, int32_t n_r, const double *r, const double *wr,
                                        const double *xi, double *out);

/* Gaussian intrinsic covariance of the binned windowed multipoles (Sec. 6, eq.
 * cov-int), even l, l' <= ell_max:
 *   C^ab_ll' = 2 (2l+1)(2l'+1)/V int p^2 dp/(2 pi^2) omega^a_l(p) omega^b_l'(p) Q_ll'(p),
 *   Q_ll'(p) = sum_{L,l1,l2} (2L+1) (l l' L;0 0 0)^2 (l1 l2 L;0 0 0)^2 P_l1(p) P_l2(p),
 * with the p integral the sum over the caller's nodes p[i], weights wp[i];
 * pk [ell_max/2+1][n_p] holds the model multipoles P_l1(p[i]) (higher ones
 * taken as zero); volume V.  out: [ell_max/2+1][n_k][ell_max/2+1][n_k], entry
 * ((l/2 n_k + a)(ell_max/2+1) + l'/2) n_k + b. */
hipster_status hipster_cov_gauss(hipster_ctx *ctx, double r0, double volume, int32_t n_k, const double *k_edges,
                                 int32_t ell_max, int32_t n_p, const double *p, const double *wp, const double *pk,
                                 double *out);

/* Non-Gaussian intrinsic covariance of the binned windowed multipoles (Sec. 6,
 * the 4C^NG term), even l, l' <= ell_max:
 *   C^ab_ll' = (2l+1)(2l'+1)/V (-1)^(l+l') int p1^2 dp1/(2 pi^2) p2^2 dp2/(2 pi^2)
 *              Tbar_ll'(p1, p2) omega^a_l(p1) omega^b_l'(p2),
 * both p integrals as sums over the caller's nodes p[i] with weights wp[i];
 * tbar [ell_max/2+1][ell_max/2+1][n_p][n_p] holds the collapsed-trispectrum
 * multipoles Tbar_ll'(p[i], p[j]) (higher multipoles taken as zero); volume
 * V.  out: as hipster_cov_gauss.  Errors as hipster_cov_gauss. */
hipster_status hipster_cov_nongauss(hipster_ctx *ctx, double r0, double volume, int32_t n_k, const double *k_edges,
                                    int32_t ell_max, int32_t n_p, const double *p, const double *wp,
                                    const double *tbar, double *out);

/* Poisson two-point covariance term of the binned windowed multipoles (Sec. 6,
 * eq. cov-poiss, the 2C term), even l, l' <= ell_max:
 *   C^ab_ll' = 2/(n^2 V) (2l+1)(2l'+1) (-i)^(l+l') 4 pi int x^2 W^2 jbar^a_l jbar^b_l'
 *              [delta_ll'/(2l+1) + sum_L (L l l'; 0 0 0)^2 xi_L(x)] dx,
 * as the sum over the caller's nodes r[m] in [0, R0] with weights wr[m]; xi
 * [ell_max/2+1][n_r] holds xi_L(r[m]) for even L <= ell_max (higher ones taken
 * as zero); nbar the mean density, volume V.  The prefactor is 2, where the
 * paper prints 4 in this term and 2 in its unbinned form: with xi = 0 the
 * sum of this term and hipster_cov_poisson3 is then the estimator's exact
 * covariance for a uniform catalogue with a Poisson-distributed number of
 * points.  out: as hipster_cov_gauss.  Errors as the other
 * theory calls; nbar <= 0 is HIPSTER_EDOMAIN. */
hipster_status hipster_cov_poisson2(hipster_ctx *ctx, double r0, double nbar, double volume, int32_t n_k,
                                    const double *k_edges, int32_t ell_max, int32_t n_r, const double *r,
                                    const double *wr, const double *xi, double *out);

/* Poisson three-point covariance term of the binned windowed multipoles
 * (Sec. 6, eq. cov-poiss, the 3C term), even l, l' <= ell_max:
 *   C^ab_ll' = 4/(n V) [W~^a W~^b d_l0 d_l'0 + W~^a P^b_l' d_l0 + W~^b P^a_l d_l'0 + B^ab_l d_ll']
 *            + 4/(n V) (2l+1)(2l'+1) sum_L (L l l'; 0 0 0)^2
 *                int p^2 dp/(2 pi^2) P_L(p) omega^a_l(p) omega^b_l'(p),
 * the p integral the sum over the caller's nodes p[i], weights wp[i]; pk
 * [ell_max/2+1][n_p] holds P_L(p[i]) for even L <= ell_max (higher ones taken
 * as zero); pbin [ell_max/2+1][n_k] the windowed binned multipoles P^a_l (as
 * hipster_pk_ell or hipster_pk_window_theory return them) and bk
 * [ell_max/2+1][n_k][n_k] the binned bispectrum B^ab_l at even l (as
 * hipster_bk_ell returns it); either may be NULL (taken as zero).  With xi = 0
 * the sum of this term and hipster_cov_poisson2 is the exact covariance of the
 * estimator for a uniform catalogue with a Poisson-distributed number of
 * points.  out: as hipster_cov_gauss.  Errors as hipster_cov_gauss; nbar <= 0
 * is HIPSTER_EDOMAIN. */
hipster_status hipster_cov_poisson3(hipster_ctx *ctx, double r0, double nbar, double volume, int32_t n_k,
                                    const double *k_edges, int32_t ell_max, int32_t n_p, const double *p,
                                    const double *wp, const double *pk, const double *pbin, const double *bk,
                                    double *out);

/* Parameters of the survey-geometry power spectrum (hipster_pk_survey).
 * volume: V of the normalisation 1/(n_w^2 V), n_w = sum(w_data) / V (the
 * paper normalises by the ideal n^2 V, Sec. 2).  r0, n_k, ell_max, k_edges,
 * precision: as in hipster_params (ell_max even, <= 6; n_k <= 128).
 * primary_mask / random_mask: NULL, or one byte per data / random point; only
 * ordered pairs (i, j) whose first point has a non-zero byte contribute (a
 * hook for checking a subset of a large catalogue).  reserved: set to 0. */
typedef struct {
  double volume;
  double r0;
  int32_t n_k;
  int32_t ell_max;
  const double *k_edges;
  int32_t precision;
  int32_t reserved;
  const uint8_t *primary_mask;
  const uint8_t *random_mask;
} hipster_survey_params;

/* Power-spectrum multipoles of a survey (Sec. 2, the general estimator
 * DD - 2DR + RR of eq. general-Pk-ell with the pair counts of eq.
 * general-XY-counts, binned in k as in Sec. 3):
 *   P^a_l = [DD - 2 DR + RR]^a_l / (n_w^2 V),
 *   XY^a_l = (-i)^l (2l+1) sum_{i in X} sum_{j in Y, j != i if X = Y}
 *            v_i v_j jbar^a_l(r_ij) L_l(xhat_ij . nhat_ij) W(r_ij / R0),
 * the line of sight nhat_ij along the pair midpoint (x_i + x_j) / 2 with the
 * observer at the origin, and no periodicity.  v = w for data and
 * v = s_R w for randoms, s_R = sum(w_data) / sum(w_rand), so that the random
 * catalogue stands for the data's mean density.  data, randoms: catalogues at
 * any finite positions; randoms must be non-empty.  pk: host output,
 * [ell_max/2 + 1][n_k].  diag: raw = [DD - 2DR + RR]^a_l before the
 * normalisation; n_pairs / n_pairs_rand / n_pairs_rr = ordered DD, DR + RD and
 * RR pairs inside R0 (mask-weighted when masks are given); wtilde unused. */
hipster_status hipster_pk_survey(hipster_ctx *ctx, const hipster_points *data, const hipster_points *randoms,
                                 const hipster_survey_params *prm, double *pk, hipster_diag *diag);

/* One box of a batch: its catalogue(s), parameters and host outputs. */
typedef struct {
  hipster_points data;
  hipster_points randoms;   /* n = 0: no random primaries */
  hipster_params pk_params; /* n_k = 0: no power spectrum for this box */
  hipster_params bk_params; /* n_k = 0: no bispectrum for this box */
  double *pk;               /* [pk ell_max/2+1][pk n_k] */
  double *bk;               /* [bk ell_max+1][bk n_k][bk n_k] */
  uint64_t n_pairs;         /* out: ordered data-data pairs */
  int32_t bk_eii_nodes;     /* < 0: DDR^II from random primaries as hipster_bk_ell (`randoms`,
                               or f_rand and seed below); >= 0: from the E^II kernel as
                               hipster_bk_ell_analytic with this n_x (0: default), no randoms */
  int32_t reserved;
  double f_rand;            /* as hipster_bk_ell, used when randoms.n = 0 */
  uint64_t seed;
} hipster_box_job;

/* Many independent boxes in one pass: every box's pairs are enumerated into
 * one shared work stream, so the pair-weight kernels run as single launches
 * balanced across boxes of very different size.  Equivalent to calling
 * hipster_pk_ell / hipster_bk_ell per box. */
hipster_status hipster_batch(hipster_ctx *ctx, int n_boxes, hipster_box_job *jobs,
                             hipster_diag *diag);

/* The binned window transform W~^a(R0) = 4 pi int_0^R0 r^2 jbar^a_0(r) W(r/R0) dr
 * (Sec. 3, eq. wka-def) for the n_k bins given by k_edges (host doubles, as
 * in hipster_params); out: n_k host doubles.  Host-only, needs no device.
 * Returns HIPSTER_EINVAL / HIPSTER_EDOMAIN on bad arguments. */
hipster_status hipster_wtilde(double r0, int32_t n_k, const double *k_edges, double *out);

/* Message for the last failing call on ctx (never NULL). */
const char *hipster_last_error(const hipster_ctx *ctx);

/* Name of a status code. */
const char *hipster_status_string(hipster_status s);

/* Cap on the device memory a context may hold (bytes; 0 = no cap beyond the
 * device).  Requests past the cap fail with HIPSTER_ENOMEM. */
hipster_status hipster_set_memory_cap(hipster_ctx *ctx, uint64_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* HIPSTER_H */
