// The bispectrum's second data-data-random term without randoms (Sec. 4,
// eq. EII-intro; Appendix A, eq. DDRII-kernel; Appendix B).  It is a sum over
// data pairs out to 2 R0 of a kernel of the pair separation,
//   DDR^II,ab_l = n (-1)^l (2l+1) sum_{i!=j} w_i w_j E^{II,ab}_l(|x_ij|),
//   E^{II,ab}_l(x) = (2 pi / x) int int dr1 dr2 r1 r2 g^a_l(r1) g^b_l(r2) L_l(Delta)
// over the band |r1 - r2| <= x <= r1 + r2 of [0, R0]^2 (the beta(Delta) of the
// triple-Bessel identity), Delta = (r1^2 + r2^2 - x^2) / (2 r1 r2),
// g^a_l = jbar^a_l W.  As the paper suggests, E is tabulated once per (R0,
// bins) and interpolated per pair:
//
//   k_eii_table   E on the nodes x_m = m h, h = 2 R0 / n_x, by composite
//                 16-point Gauss-Legendre in double precision (one workgroup
//                 per (l, m); the outer r1 nodes are spread over the threads,
//                 each thread sums its inner r2 integral for every bin);
//   k_ddr2_hist   every (pair, periodic image) inside 2 R0 adds its six
//                 interpolation weights l_q(t), times w_i w_j, to the nodes
//                 m-2 .. m+3 of an LDS histogram: the pair sum of the
//                 interpolated kernel is then sum_m E_m H_m exactly, so the
//                 sweep does the same small work for any number of bins and
//                 multipoles;
//   k_hist_reduce_fix, k_ddr2_contract
//                 exact integer sums of the per-workgroup (64-bit fixed
//                 point) histograms and the fixed-order contraction
//                 T^ab_l = sum_m E^ab_l(x_m) H_m.
//
// Interpolation (a reading: the paper leaves the scheme open): on
// [x_m, x_{m+1}) the quintic through the nodes m-2 .. m+3, t = x/h - m; nodes
// below 0 take E(-x) = E(x) (E is a smooth function of the pair vector, even
// in x) and the nodes at and beyond 2 R0 hold E = 0 (its support).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "specfun.h"

namespace hipster {

constexpr int kEiiThreads = 256;
constexpr int kEiiMaxNk = 16;

// Gauss-Legendre nodes and weights on [-1, 1] (16 points), computed on the
// host by Newton's method on the Legendre polynomial.  Panels are at most
// 8 / k_max wide: the integrands oscillate at up to 2 k_max (a product of two
// bin averages), so a panel spans at most ~16 radians of phase, where the
// 16-point rule's error is ~1e-16 relative.
constexpr int kGL = 16;
struct GLRule {
  double x[kGL], w[kGL];
};

static GLRule gauss_legendre16() {
  GLRule g{};
  const int n = kGL;
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), d = 0.0;
    for (int it = 0; it < 50; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; ++k) {
        const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
      }
      d = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / d;
      z -= dz;
      if (fabs(dz) < 1e-17) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 1; k < n; ++k) {
      const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
      p0 = p1;
      p1 = p2;
    }
    d = n * (z * p1 - p0) / (z * z - 1.0);
    g.x[i] = z;
    g.w[i] = 2.0 / ((1.0 - z * z) * d * d);
  }
  return g;
}

// G_l(u) = Dt_l(u) / u^3 for one multipole l (uniform over the workgroup),
// double precision throughout: the Taylor series below U_BIG, above it the
// closed form with table-driven sine and cosine (exact reduction for
// u < ~1.6e6) and the 22-term fits of the sine integral's auxiliaries.
__device__ inline double G_one(int l, double u, const double2 *__restrict__ tab) {
  if (u < HIPSTER_U_BIG) {
    const double v = u * u;
    double ul = 1.0;
    for (int q = 0; q < l; ++q) ul *= u;
    return u < kUSmall ? taylor_G64<14>(l, v, ul) : taylor_G64<HIPSTER_N_TAYLOR>(l, v, ul);
  }
  double s, c;
  sincos_tab<kSinCosTab, true>(u, tab, s, c);
  const double w = 1.0 / u;
  double si = 0.0;
  if (l >= 2 && (l & 1) == 0) {
    const double t = HIPSTER_U_BIG * w;
    const double f = horner64(POLY_F64, t) * w;
    const double g = horner64(POLY_G64, t) * w * w;
    si = kHalfPi - f * c - g * s;
  }
  return Dt_closed<double>(l, u, w, s, c, si) * (w * w * w);
}

// g^b_l(r) = jbar^b_l(r) W(r/R0) for the n_k bins, from one G per edge:
//   jbar^b = 3 (k_{b+1}^3 G(k_{b+1} r) - k_b^3 G(k_b r)) / (k_{b+1}^3 - k_b^3).
__device__ inline void g_bins(int l, double r, double inv_r0, int n_k, const double *__restrict__ ek,
                              const double *__restrict__ coef, const double2 *__restrict__ tab,
                              double (&g)[kEiiMaxNk]) {
  const double W = window(r * inv_r0);
  double prev = ek[1] * G_one(l, ek[0] * r, tab);  // k_0^3 G(k_0 r)
#pragma unroll
  for (int b = 0; b < kEiiMaxNk; ++b) {
    if (b < n_k) {
      const double cur = ek[2 * (b + 1) + 1] * G_one(l, ek[2 * (b + 1)] * r, tab);
      g[b] = coef[b] * (cur - prev) * W;
      prev = cur;
    } else {
      g[b] = 0.0;
    }
  }
}

// Legendre polynomial L_l(mu) by the three-term recurrence.
__device__ inline double legendre_l(int l, double mu) {
  double p0 = 1.0, p1 = mu;
  if (l == 0) return 1.0;
  for (int n = 1; n < l; ++n) {
    const double p2 = ((2 * n + 1) * mu * p1 - n * p0) / double(n + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Pieces of [lo, hi] between sorted cut points, each split into panels no
// wider than hmax.
struct Pieces {
  double p[13];
  int npan[12];
  int start[13];  // first panel of each piece; start[n] = total panels
  int n;
};

__device__ inline void make_pieces(double lo, double hi, const double *cuts, int ncut, double hmax, Pieces &P) {
  int np = 0;
  P.p[np++] = lo;
  for (int c = 0; c < ncut; ++c)
    if (cuts[c] > lo && cuts[c] < hi) P.p[np++] = cuts[c];
  P.p[np++] = hi;
  for (int i = 1; i < np; ++i)
    for (int j = i; j > 0 && P.p[j] < P.p[j - 1]; --j) {
      const double t = P.p[j];
      P.p[j] = P.p[j - 1];
      P.p[j - 1] = t;
    }
  P.n = np - 1;
  int tot = 0;
  for (int s = 0; s < P.n; ++s) {
    const double len = P.p[s + 1] - P.p[s];
    int k = len > 0.0 ? int(ceil(len / hmax)) : 0;
    P.npan[s] = k;
    P.start[s] = tot;
    tot += k;
  }
  P.start[P.n] = tot;
}

// One workgroup per (l, m): E^{II,ab}_l(m h) for all a, b, written to
// table[((l n_k + a) n_k + b) (n_x + 1) + m].
__global__ __launch_bounds__(kEiiThreads) void k_eii_table(double r0, double h, int n_x, int n_k,
                                                           const double *__restrict__ ek_g,
                                                           const double *__restrict__ coef_g, GLRule gl, double hmax,
                                                           double *__restrict__ table) {
  __shared__ double2 tab[kSinCosTab];
  __shared__ double ek[2 * (kEiiMaxNk + 1)], coef[kEiiMaxNk];
  // the outer nodes' rows w1 r1 g^a(r1) and H^b(r1), staged half a
  // workgroup at a time
  __shared__ double A[kEiiThreads / 2][kEiiMaxNk + 1], Hs[kEiiThreads / 2][kEiiMaxNk + 1];
  __shared__ Pieces outer;
  const int m = blockIdx.x, l = blockIdx.y, tid = threadIdx.x;
  const int nab = n_k * n_k;
  const size_t stride = size_t(n_x) + 1;
  if (m == n_x) {  // x = 2 R0: outside the support
    for (int q = tid; q < nab; q += kEiiThreads) table[(size_t(l) * nab + q) * stride + m] = 0.0;
    return;
  }
  const double x = m * h, inv_r0 = 1.0 / r0;
  stage_sincos_tab<kSinCosTab>(tab);
  for (int i = tid; i < 2 * (n_k + 1); i += kEiiThreads) ek[i] = ek_g[i];
  for (int i = tid; i < n_k; i += kEiiThreads) coef[i] = coef_g[i];
  if (tid == 0) {
    // cuts of r1: the joins of W, r1 = x, and where |x - r1| or r1 + x meets a
    // join of W or R0
    const double cuts[10] = {0.5 * r0, 0.75 * r0, x, x - 0.5 * r0, x + 0.5 * r0,
                             x - 0.75 * r0, x + 0.75 * r0, 0.5 * r0 - x, 0.75 * r0 - x, r0 - x};
    make_pieces(x > r0 ? x - r0 : 0.0, r0, cuts, x > 0.0 ? 10 : 2, hmax, outer);
  }
  __syncthreads();
  const int n1 = kGL * outer.start[outer.n];
  const double joins[2] = {0.5 * r0, 0.75 * r0};
  double acc = 0.0;
  const int my_a = tid / n_k, my_b = tid - my_a * n_k;
  for (int q0 = 0; q0 < n1; q0 += kEiiThreads) {
    const int q = q0 + tid;
    double ga[kEiiMaxNk], H[kEiiMaxNk];
#pragma unroll
    for (int b = 0; b < kEiiMaxNk; ++b) {
      ga[b] = 0.0;
      H[b] = 0.0;
    }
    if (q < n1) {
      const int pan = q / kGL, node = q % kGL;
      int s = 0;
      while (pan >= outer.start[s + 1]) ++s;
      const double ph = (outer.p[s + 1] - outer.p[s]) / outer.npan[s];
      const double mid = outer.p[s] + (pan - outer.start[s] + 0.5) * ph;
      const double r1 = mid + 0.5 * ph * gl.x[node], w1 = 0.5 * ph * gl.w[node];
      g_bins(l, r1, inv_r0, n_k, ek, coef, tab, ga);
      if (x == 0.0) {
        // limit x -> 0: 4 pi int r^2 g^a g^b dr
#pragma unroll
        for (int b = 0; b < kEiiMaxNk; ++b) {
          H[b] = ga[b];
          ga[b] *= w1 * r1 * r1;
        }
      } else {
        const double lo2 = fabs(x - r1), hi2 = fmin(r0, r1 + x);
        const double c1 = (r1 - x) * (r1 + x), inv2r1 = 0.5 / r1;
        if (hi2 > lo2) {
          Pieces inner;
          make_pieces(lo2, hi2, joins, 2, hmax, inner);
          for (int s2 = 0; s2 < inner.n; ++s2) {
            const double a2 = inner.p[s2];
            const int np2 = inner.npan[s2];
            if (np2 == 0) continue;
            const double ph2 = (inner.p[s2 + 1] - a2) / np2;
            for (int p2 = 0; p2 < np2; ++p2) {
              const double mid2 = a2 + (p2 + 0.5) * ph2;
              for (int j = 0; j < kGL; ++j) {
                const double r2 = mid2 + 0.5 * ph2 * gl.x[j];
                double D = (c1 + r2 * r2) * inv2r1 / r2;
                D = fmin(1.0, fmax(-1.0, D));
                const double wl = 0.5 * ph2 * gl.w[j] * r2 * legendre_l(l, D);
                double gb[kEiiMaxNk];
                g_bins(l, r2, inv_r0, n_k, ek, coef, tab, gb);
#pragma unroll
                for (int b = 0; b < kEiiMaxNk; ++b) H[b] = fma(wl, gb[b], H[b]);
              }
            }
          }
        }
#pragma unroll
        for (int b = 0; b < kEiiMaxNk; ++b) ga[b] *= w1 * r1;
      }
    }
    for (int half = 0; half < 2; ++half) {
      constexpr int kHalf = kEiiThreads / 2;
      if ((tid >= kHalf) == (half == 1)) {
#pragma unroll
        for (int b = 0; b < kEiiMaxNk; ++b) {
          A[tid - half * kHalf][b] = ga[b];
          Hs[tid - half * kHalf][b] = H[b];
        }
      }
      __syncthreads();
      if (tid < nab) {
        const int cnt = min(kHalf, n1 - q0 - half * kHalf);
        for (int j = 0; j < cnt; ++j) acc = fma(A[j][my_a], Hs[j][my_b], acc);
      }
      __syncthreads();
    }
  }
  if (tid < nab) {
    const double pref = x == 0.0 ? 4.0 * kPi : 2.0 * kPi / x;
    table[(size_t(l) * nab + tid) * stride + m] = pref * acc;
  }
}

// ------------------------------------------------------------ pair sweep
constexpr int kHistThreads = 512;  // 8 waves; one home tile shared by all
constexpr int kHistTile = 64;

// Orders one wave's LDS accesses: a value a lane stored is seen by the loads
// of the wave's other lanes that follow (LDS serves a wave's accesses in
// order; the fence keeps the compiler from moving them across).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Persistent workgroups take home tiles (unit = a home cell's tile of up to
// 64 points) from a counter; the waves of a workgroup split the unit's
// neighbour tiles (14 half-stencil cells, each in tiles of 64 points): each
// lane holds one neighbour point and runs over the home tile, read from LDS
// by broadcast.  A (pair, image) with r^2 < (2 R0)^2 (the exact double
// predicate of the pair counts) adds w_i w_j l_q(t) to the six nodes m-2 ..
// m+3 around x = r; without masks every unordered pair counts both ways
// (factor 2).  Only ~15% of the candidates hit: a single-precision
// prefilter with a safe margin passes the candidates that may lie inside
// 2 R0 into a per-wave LDS queue (ballot + prefix count), and the exact
// double-precision test and the weights run on 64 of them at a time with
// every lane busy.
// What a pair adds to the histogram.
enum HistKind {
  kHistDdr2 = 0,   // pairs inside 2 R0, weight w_i w_j per orientation
  kHistCterm = 1,  // pairs inside R0, weight w_p w_q^2 W(r/R0)^2 per orientation (p, q)
  kHistPk = 2,     // pairs inside R0, weight w_i w_j W(r/R0) L_l(mu) per orientation, one section per even l
  kHistCtermL = 3, // pairs inside R0, weight w_p w_q^2 W(r/R0)^2 P_L(mu_pq) per orientation (p, q),
                   // mu_pq along x_p - x_q; one section per L = los .. los + NLP - 1
};

// CROSS: the home points (primaries) come from `s` and the neighbours from
// `b`, found once per (primary, neighbour) pair through all 27 cells (the C
// term of random primaries against the data); otherwise `b` is `s` and each
// unordered pair is found once through the half stencil.
// n_x: table intervals (the interval index is clamped to n_x - 1); nodes
// below n_keep receive weights, the others hold a zero kernel value;
// n_hist: histogram entries.  kHistDdr2: n_keep = n_x, n_hist = n_x + 1;
// kHistCterm: n_keep = n_hist = n_x + 3 (the table runs past R0); kHistPk:
// NLP sections (l = 0, 2, ..) of n_keep = n_x + 3 nodes each, n_hist = NLP
// n_keep, `los` the line-of-sight axis of mu (0, 1, 2) or 3 for the pair
// midpoint seen from an observer at the origin, and every pair's weight
// times pair_scale.  periodic = 0: no images, neighbour cells outside the
// grid are empty (the survey geometry).  pref_scale bounds the magnitude of
// every coordinate (with its image shift), for the prefilter's margin.  All
// sum in 64-bit fixed point with scale fix_scale, so the histogram does not
// depend on the order of the adds (bitwise reproducible).
// The table form with up to three sections: six waves per SIMD (at most 80
// VGPRs), three 8-wave workgroups per CU, which is what its LDS allows.
template <bool MASKED, int KIND, bool CROSS, int NLP = 1>
__global__ __launch_bounds__(kHistThreads) __attribute__((amdgpu_waves_per_eu(KIND == 2 && NLP <= 3 ? 6 : 1))) void
k_ddr2_hist(Sorted s, Sorted b, int nc, double L, double lim2,
                                                            double inv_h,
                                                            int n_x, int n_keep, int n_hist, double inv_r0,
                                                            double fix_scale, int los, int periodic,
                                                            double pref_scale, double pair_scale,
                                                            const int *__restrict__ unit_cell,
                                                            const int *__restrict__ unit_tile, int64_t n_units,
                                                            unsigned long long *__restrict__ counter,
                                                            unsigned long long *__restrict__ ordered,
                                                            double *__restrict__ partial) {
  extern __shared__ double hist[];  // n_hist nodes
  __shared__ double4 home[kHistTile];
  __shared__ int hm[kHistTile];
  // the neighbour cells as runs contiguous in memory: cells are numbered
  // with z fastest, so each (x, y) row of the stencil is one z-run, cut
  // where it wraps round the box in z into up to three runs (the wrapped cell
  // below, the cells inside, the wrapped cell above; with one cell per axis
  // all three are that cell).  Half stencil: the rows (0, 0) from the home
  // cell's z up, (0, +1) and (+1, -1..+1); full stencil: all nine rows.
  constexpr int kRows = CROSS ? 9 : 5;
  constexpr int kRuns = 3 * kRows;
  __shared__ int64_t nb_start[kRuns];
  __shared__ int nb_count[kRuns], nb_first[kRuns + 1], nb_self[kRuns];
  __shared__ double nb_off[kRuns][3];
  __shared__ int64_t cur_unit;
  constexpr int kWaves = kHistThreads / 64;
  // single-precision home coordinates for the prefilter
  __shared__ float4 homef[kHistTile];
  // per wave: candidates (home index * 64 + neighbour lane) that passed the
  // prefilter; the neighbour tile itself stays in registers, one point per
  // lane, and is read across lanes
  __shared__ unsigned short qc[kWaves][128];
  double4 qreg = make_double4(0.0, 0.0, 0.0, 0.0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  // prefilter bound: (sqrt(lim2) + delta)^2 in single precision, delta =
  // 2^-17 pref_scale covers the rounding of coordinates below pref_scale in
  // size to single precision (each within 2^-24 of its magnitude) and of the
  // single-precision distance
  const float lim2f =
      float((sqrt(lim2) + 0x1p-17 * pref_scale) * (sqrt(lim2) + 0x1p-17 * pref_scale));
  for (int i = tid; i < n_hist; i += kHistThreads) hist[i] = 0.0;
  unsigned long long ord = 0;
  int qn = 0;  // queued candidates of this wave (uniform over the wave)
  // one (pair, image) at x = sqrt(r2): six-point Lagrange weights of the
  // nodes m-2 .. m+3 times ww[sec] into each section; nodes below 0 fold onto
  // their mirror (every tabulated kernel is even in x), nodes >= n_keep hold
  // a zero kernel
  auto spread = [&](double r2, const double (&ww)[NLP]) {
    const double sx = sqrt(r2) * inv_h;
    int mi = int(sx);
    if (mi > n_x - 1) mi = n_x - 1;
    const double t = sx - double(mi);
    const double tp2 = t + 2.0, tp1 = t + 1.0, tm1 = t - 1.0, tm2 = t - 2.0, tm3 = t - 3.0;
    const double a01 = tp2 * tp1, a34 = tm2 * tm3, b = t * tm1;
    const double lw[6] = {-tp1 * b * a34 * (1.0 / 120.0), tp2 * b * a34 * (1.0 / 24.0),
                          -a01 * tm1 * a34 * (1.0 / 12.0), a01 * t * a34 * (1.0 / 12.0),
                          -a01 * b * tm3 * (1.0 / 24.0), a01 * b * tm2 * (1.0 / 120.0)};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      int node = mi + q - 2;
      node = node < 0 ? -node : node;
      if (node < n_keep) {
#pragma unroll
        for (int sec = 0; sec < NLP; ++sec) {
          // fixed point (scale 2^e chosen on the host so no sum can
          // overflow): integer sums do not depend on the order of the adds.
          // kHistPk's scale keeps every single add below 2^30 in size, so it
          // rounds with the native 32-bit conversion
          long long iv;
          if constexpr (KIND == kHistPk)
            iv = __double2int_rn(ww[sec] * lw[q] * fix_scale);
          else
            iv = llrint(ww[sec] * lw[q] * fix_scale);
          atomicAdd(reinterpret_cast<unsigned long long *>(&hist[sec * n_keep + node]),
                    static_cast<unsigned long long>(iv));
        }
      }
    }
  };
  // the exact double-precision test of candidate (home ii, neighbour
  // jbase + jl) and, inside the radius, its ordered-pair multiplicity and
  // weight; called by the whole wave (the neighbour is fetched from lane jl),
  // lanes with valid = false only take part in the fetch
  auto exact = [&](int ii, int jl, bool valid, int64_t jbase, double offx, double offy, double offz) {
    double4 q;
    q.x = __shfl(qreg.x, jl);
    q.y = __shfl(qreg.y, jl);
    q.z = __shfl(qreg.z, jl);
    q.w = __shfl(qreg.w, jl);
    if (!valid) return;
    const double4 p = home[ii];
    const int64_t j = jbase + jl;
    double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
    dx -= offx;
    dy -= offy;
    dz -= offz;
    double r2;
    {
#pragma clang fp contract(off)
      const double a = dx * dx, b = dy * dy, c = dz * dz;
      r2 = (a + b) + c;
    }
    if (r2 < lim2) {
      // the cross sweep of the power spectrum counts both orientations of a
      // (primary, neighbour) pair; that of the C term only the first
      const int mi_ = MASKED ? hm[ii] : 1,
                mj_ = (CROSS && KIND != kHistPk) ? 0 : (MASKED ? (b.m ? int(b.m[j]) : 1) : 1);
      ord += unsigned(mi_ + mj_);
      if (mi_ + mj_ > 0) {
        double wv[NLP];
        if constexpr (KIND == kHistPk) {
          // both orientations have the same |mu|, and L_l is even
          const double r = sqrt(r2);
          double mu = 0.0;
          if (los < 3) {
            const double d = los == 0 ? dx : (los == 1 ? dy : dz);
            mu = r2 > 0.0 ? d / r : 0.0;
          } else {
            // line of sight along the pair midpoint (x_i + x_j) / 2
            const double mx = p.x + (q.x + offx), my = p.y + (q.y + offy), mz = p.z + (q.z + offz);
            const double mn = sqrt((mx * mx + my * my) + mz * mz);
            mu = (r > 0.0 && mn > 0.0) ? ((dx * mx + dy * my) + dz * mz) / (r * mn) : 0.0;
          }
          const double m2 = mu * mu;
          const double base = pair_scale * p.w * q.w * double(mi_ + mj_) * window<double>(r * inv_r0);
          wv[0] = base;
          if constexpr (NLP > 1) wv[1] = base * (1.5 * m2 - 0.5);
          if constexpr (NLP > 2) wv[2] = base * (((35.0 * m2 - 30.0) * m2 + 3.0) * 0.125);
          if constexpr (NLP > 3) wv[3] = base * ((((231.0 * m2 - 315.0) * m2 + 105.0) * m2 - 5.0) * 0.0625);
        } else if constexpr (KIND == kHistCtermL) {
          // P_L of the (p, q) orientation; the (q, p) one has -mu, (-1)^L P_L
          const double r = sqrt(r2);
          const double mu = r2 > 0.0 ? dz / r : 0.0;
          const double W = window<double>(r * inv_r0);
          const double a = p.w * q.w * q.w * double(mi_) * (W * W);
          const double b = CROSS ? 0.0 : q.w * p.w * p.w * double(mj_) * (W * W);
          // (c0, c1) = (P_L, P_{L+1}), advanced by the three-term recurrence
          double c0 = 1.0, c1 = mu;
          int L = 0;
          for (; L < los; ++L) {
            const double nx = (double(2 * L + 3) * mu * c1 - double(L + 1) * c0) / double(L + 2);
            c0 = c1;
            c1 = nx;
          }
#pragma unroll
          for (int sec = 0; sec < NLP; ++sec, ++L) {
            wv[sec] = c0 * (a + ((L & 1) ? -b : b));
            const double nx = (double(2 * L + 3) * mu * c1 - double(L + 1) * c0) / double(L + 2);
            c0 = c1;
            c1 = nx;
          }
        } else if constexpr (CROSS) {
          // (primary i, neighbour j) only
          const double W = window<double>(sqrt(r2) * inv_r0);
          wv[0] = p.w * q.w * q.w * double(mi_) * (W * W);
        } else if constexpr (KIND == kHistDdr2) {
          wv[0] = p.w * q.w * double(mi_ + mj_);
        } else {
          // (i, j) as (p, q) if i is selected, and (j, i) if j is
          const double W = window<double>(sqrt(r2) * inv_r0);
          wv[0] = p.w * q.w * (double(mi_) * q.w + double(mj_) * p.w) * (W * W);
        }
        spread(r2, wv);
      }
    }
  };
  // the unit index is taken and published between two barriers (publishing
  // it at the end of the loop body instead, for a barrier at the top, let
  // waves read a stale index: the barrier did not wait for the store)
  for (;;) {
    __syncthreads();
    if (tid == 0) cur_unit = int64_t(atomicAdd(counter, 1ull));
    __syncthreads();
    const int64_t unit = cur_unit;
    if (unit >= n_units) break;
    const int cell = unit_cell[unit];
    const int i0 = unit_tile[unit] * kHistTile;
    const int cz = cell % nc, cy = (cell / nc) % nc, cx = cell / (nc * nc);
    const int64_t hs = s.cell_start[cell];
    const int ni = int(s.cell_start[cell + 1] - hs);
    const int ti = min(kHistTile, ni - i0);
    if (tid < ti) {
      const int64_t i = hs + i0 + tid;
      home[tid] = make_double4(s.x[i], s.y[i], s.z[i], s.w[i]);
      homef[tid] = make_float4(float(s.x[i]), float(s.y[i]), float(s.z[i]), 0.0f);
      if (MASKED) hm[tid] = s.m ? int(s.m[i]) : 1;
    }
    if (wave == 0) {
      // lane r < kRows sets up stencil row r as runs 3r .. 3r+2; the wave
      // then numbers the neighbour tiles with a prefix sum.  The self row's
      // inside run (run 1) starts at the home cell, whose tiles before the
      // home tile hold no pairs j > i and are skipped.
      int tiles_lo = 0, tiles_in = 0, tiles_hi = 0;
      if (lane < kRows) {
        int ox, oy, zlo;
        if (CROSS) {
          ox = lane / 3 - 1;
          oy = lane % 3 - 1;
          zlo = cz - 1;
        } else if (lane == 0) {
          ox = 0;
          oy = 0;
          zlo = cz;
        } else if (lane == 1) {
          ox = 0;
          oy = 1;
          zlo = cz - 1;
        } else {
          ox = 1;
          oy = lane - 3;
          zlo = cz - 1;
        }
        const int zhi = cz + 1;
        int sx = 0, sy = 0;
        int nx = cx + ox, ny = cy + oy;
        // without periodicity a row outside the grid holds nothing, and only
        // a row's inside run exists
        const bool row_out = !periodic && (nx < 0 || nx >= nc || ny < 0 || ny >= nc);
        if (nx >= nc) { nx -= nc; sx = 1; } else if (nx < 0) { nx += nc; sx = -1; }
        if (ny >= nc) { ny -= nc; sy = 1; } else if (ny < 0) { ny += nc; sy = -1; }
        const int64_t rowbase = (int64_t(nx) * nc + ny) * nc;
        // zlo >= -1 and zhi <= nc: the wrapped cells are z = -1 (cell nc - 1
        // shifted down) and z = nc (cell 0 shifted up); the inside run
        // [max(zlo, 0), min(zhi, nc - 1)] always holds z = cz
        const int in0 = max(zlo, 0), in1 = min(zhi, nc - 1);
        int64_t s_in = 0, s_lo = 0, s_hi = 0;
        int cnt_in = 0, cnt_lo = 0, cnt_hi = 0;
        if (!row_out) {
          s_in = b.cell_start[rowbase + in0];
          cnt_in = int(b.cell_start[rowbase + in1 + 1] - s_in);
          if (periodic && zlo < 0) {
            s_lo = b.cell_start[rowbase + nc - 1];
            cnt_lo = int(b.cell_start[rowbase + nc] - s_lo);
          }
          if (periodic && zhi >= nc) {
            s_hi = b.cell_start[rowbase];
            cnt_hi = int(b.cell_start[rowbase + 1] - s_hi);
          }
        }
        const bool self_row = !CROSS && lane == 0;
        const int r = 3 * lane;
        nb_start[r] = s_lo;
        nb_count[r] = cnt_lo;
        nb_self[r] = 0;
        nb_start[r + 1] = s_in;
        nb_count[r + 1] = cnt_in;
        nb_self[r + 1] = self_row ? ni : 0;
        nb_start[r + 2] = s_hi;
        nb_count[r + 2] = cnt_hi;
        nb_self[r + 2] = 0;
        for (int q = 0; q < 3; ++q) {
          nb_off[r + q][0] = double(sx) * L;
          nb_off[r + q][1] = double(sy) * L;
          nb_off[r + q][2] = double(q - 1) * L;
        }
        const int t0 = self_row ? i0 / kHistTile : 0;
        tiles_lo = (cnt_lo + kHistTile - 1) / kHistTile;
        tiles_in = max(0, (cnt_in + kHistTile - 1) / kHistTile - t0);
        tiles_hi = (cnt_hi + kHistTile - 1) / kHistTile;
      }
      int incl = tiles_lo + tiles_in + tiles_hi;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
      }
      if (lane < kRows) {
        nb_first[3 * lane] = incl - tiles_lo - tiles_in - tiles_hi;
        nb_first[3 * lane + 1] = incl - tiles_in - tiles_hi;
        nb_first[3 * lane + 2] = incl - tiles_hi;
      }
      if (lane == kRows - 1) nb_first[kRuns] = incl;
    }
    __syncthreads();
    const int items = nb_first[kRuns];
    for (int it = wave; it < items; it += kWaves) {
      int st = 0;
      while (it >= nb_first[st + 1]) ++st;
      const int j0 = ((!CROSS && st == 1 ? i0 / kHistTile : 0) + it - nb_first[st]) * kHistTile;
      const int tj = min(kHistTile, nb_count[st] - j0);
      const int self_n = nb_self[st];  // leading points of the run in the home cell
      const double offx = nb_off[st][0], offy = nb_off[st][1], offz = nb_off[st][2];
      const int64_t jbase = nb_start[st] + j0;
      // single-precision copy of this lane's neighbour image for the prefilter
      float fx = 0.0f, fy = 0.0f, fz = 0.0f;
      qreg = make_double4(0.0, 0.0, 0.0, 0.0);
      if (lane < tj) {
        const int64_t j = jbase + lane;
        qreg = make_double4(b.x[j], b.y[j], b.z[j], b.w[j]);
        fx = float(qreg.x + offx);
        fy = float(qreg.y + offy);
        fz = float(qreg.z + offz);
      }
      wave_sync();
      const int jg = j0 + lane;  // index of this lane's point within its run
      // four home points per step: their LDS reads issue together, so the
      // wave waits on one read latency per four points (ii < 64 always
      // indexes homef in bounds; entries from ti on are masked out)
      constexpr int kStep = 4;
      for (int ii0 = 0; ii0 < ti; ii0 += kStep) {
        bool cand[kStep];
#pragma unroll
        for (int u = 0; u < kStep; ++u) {
          const int ii = ii0 + u;
          const float4 p = homef[ii];
          const float dx = p.x - fx, dy = p.y - fy, dz = p.z - fz;
          cand[u] = ii < ti && lane < tj && !(jg < self_n && jg <= i0 + ii) &&
                    fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < lim2f;
        }
#pragma unroll
        for (int u = 0; u < kStep; ++u) {
          // compact the candidates into the wave's queue; test and weigh 64 at a time
          const unsigned long long bal = __ballot(cand[u]);
          if (bal) {
            if (cand[u]) {
              const int at = qn + __popcll(bal & below);
              qc[wave][at] = static_cast<unsigned short>((ii0 + u) * 64 + lane);
            }
            qn += __popcll(bal);
            if (qn >= 64) {
              wave_sync();
              const int e = qc[wave][lane];
              exact(e >> 6, e & 63, true, jbase, offx, offy, offz);
              const int rest = qn - 64;
              int a = 0;
              if (lane < rest) a = qc[wave][64 + lane];
              wave_sync();
              if (lane < rest) qc[wave][lane] = static_cast<unsigned short>(a);
              qn = rest;
              wave_sync();
            }
          }
        }
      }
      // the queue refers to this neighbour tile: drain it before the next
      wave_sync();
      if (qn > 0) {
        const int e = lane < qn ? int(qc[wave][lane]) : 0;
        exact(e >> 6, e & 63, lane < qn, jbase, offx, offy, offz);
      }
      qn = 0;
      wave_sync();
    }
  }
  // ordered (pair, image) terms of the workgroup, and its histogram
  for (int o = 32; o > 0; o >>= 1) ord += __shfl_xor(ord, o);
  if (lane == 0 && ord) atomicAdd(ordered, ord);
  __syncthreads();
  double *out = partial + size_t(blockIdx.x) * size_t(n_hist);
  for (int i = tid; i < n_hist; i += kHistThreads) out[i] = hist[i];
}

// H[m] = sum over workgroups of partial[wg][m] (the rows hold the int64 bit
// patterns of fixed-point sums): an exact integer sum, then H[m] = sum / scale.
// A block takes 64 nodes (one per lane, so every row read is one coalesced
// 512-byte segment); its 16 waves split the rows and add their integer
// partial sums in LDS, which gives the same bits in any order.
constexpr int kReduceWaves = 16;
__global__ __launch_bounds__(64 * kReduceWaves) void k_hist_reduce_fix(const double *__restrict__ partial, int nwg,
                                                                      int n_nodes, double inv_scale,
                                                                      double *__restrict__ H) {
  __shared__ long long red[kReduceWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = blockIdx.x * 64 + lane;
  const long long *p = reinterpret_cast<const long long *>(partial);
  long long s = 0;
  if (m < n_nodes) {
#pragma unroll 4
    for (int g = wave; g < nwg; g += kReduceWaves) s += p[size_t(g) * n_nodes + m];
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0) {
    long long t = 0;
    for (int w = 0; w < kReduceWaves; ++w) t += red[w][lane];
    if (m < n_nodes) H[m] = double(t) * inv_scale;
  }
}

static void hist_reduce(Ctx &c, const double *partial, int nwg, int n_hist, double inv_scale, double *H) {
  k_hist_reduce_fix<<<dim3(unsigned((n_hist + 63) / 64)), dim3(64 * kReduceWaves), 0, c.stream>>>(partial, nwg,
                                                                                                  n_hist, inv_scale, H);
  HIPSTER_HIP(hipGetLastError());
}

// Largest |w| of n doubles, as the bit pattern of a non-negative double
// (which orders like the integer).
__global__ void k_absmax(const double *__restrict__ w, int64_t n, unsigned long long *__restrict__ out) {
  unsigned long long best = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    best = max(best, static_cast<unsigned long long>(__double_as_longlong(fabs(w[i]))));
  for (int o = 32; o > 0; o >>= 1) best = max(best, static_cast<unsigned long long>(__shfl_xor(best, o)));
  if ((threadIdx.x & 63) == 0) atomicMax(out, best);
}

// T[row] = sum_m table[row][m] H_s[m], H_s the histogram section
// row / rows_per_hist; one workgroup per row, a fixed-order tree reduction.
__global__ __launch_bounds__(256) void k_ddr2_contract(const double *__restrict__ table, const double *__restrict__ H,
                                                       int n_nodes, int rows_per_hist, double *__restrict__ T) {
  __shared__ double red[256];
  const double *row = table + size_t(blockIdx.x) * n_nodes;
  H += size_t(blockIdx.x / rows_per_hist) * n_nodes;
  double s = 0.0;
  for (int m = threadIdx.x; m < n_nodes; m += 256) s = fma(row[m], H[m], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) T[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------ host
int eii_default_nodes(double r0, double k_max) {
  // k_max h <= 0.15: the quintic's error is ~5e-3 (k h)^6 ~ 6e-8 of the kernel
  const double want = 2.0 * k_max * r0 / 0.15;
  int n = int(std::min(double(kEiiMaxNodes), ceil(want / 64.0) * 64.0));
  return std::max(64, n);
}

void eii_table(Ctx &c, double r0, int n_k, const double *k_edges, int ell_max, int n_x, double *table) {
  std::vector<double> ek(static_cast<size_t>(2 * (n_k + 1))), coef(static_cast<size_t>(n_k));
  for (int e = 0; e <= n_k; ++e) {
    ek[size_t(2 * e)] = k_edges[e];
    ek[size_t(2 * e + 1)] = k_edges[e] * k_edges[e] * k_edges[e];
  }
  for (int b = 0; b < n_k; ++b) coef[size_t(b)] = 3.0 / (ek[size_t(2 * b + 3)] - ek[size_t(2 * b + 1)]);
  double *dk = static_cast<double *>(ensure(c, c.eii_consts, size_t(3 * n_k + 2) * 8));
  HIPSTER_HIP(hipMemcpyAsync(dk, ek.data(), ek.size() * 8, hipMemcpyHostToDevice, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(dk + ek.size(), coef.data(), coef.size() * 8, hipMemcpyHostToDevice, c.stream));
  const double k_max = k_edges[n_k];
  const double hmax = std::min(0.25 * r0, 8.0 / k_max);
  k_eii_table<<<dim3(unsigned(n_x + 1), unsigned(ell_max + 1)), dim3(kEiiThreads), 0, c.stream>>>(
      r0, 2.0 * r0 / n_x, n_x, n_k, dk, dk + ek.size(), gauss_legendre16(), hmax, table);
  HIPSTER_HIP(hipGetLastError());
}

size_t ddr2_max_nodes(Ctx &c) {
  int lds = 0;
  HIPSTER_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device));
  hipFuncAttributes fa{};
  HIPSTER_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&k_ddr2_hist<true, kHistCterm, true>)));
  const long avail = long(lds) - long(fa.sharedSizeBytes);
  return avail > 8 ? size_t(avail / 8) : 0;
}

// One histogram sweep of `s` (sorted on grid `g`) and its contraction
// out[row] = sum_m table[row][m] H[m] over n_hist nodes.
template <int KIND, bool CROSS>
static void hist_sweep(Ctx &c, const Sorted &s, const Sorted &b, const Grid &g, double lim2, double inv_h, int n_x,
                       int n_keep,
                       int n_hist, double inv_r0, double fix_scale, const double *table, int rows, double *out,
                       unsigned long long *ordered) {
  if (size_t(n_hist) > ddr2_max_nodes(c)) throw Error{HIPSTER_EUNSUPPORTED, "pair histogram exceeds the device's LDS"};
  const PairUnits u = make_pair_units(c, s, g);
  int nwg = 0;
  {
    int cus = 0;
    HIPSTER_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device));
    nwg = std::max(1, cus) * 4;
  }
  double *partial = static_cast<double *>(ensure(c, c.ddr2_partial, size_t(nwg) * n_hist * 8));
  double *H = static_cast<double *>(ensure(c, c.ddr2_hist, size_t(n_hist) * 8));
  unsigned long long *counter = static_cast<unsigned long long *>(ensure(c, c.ddr2_counter, 8));
  HIPSTER_HIP(hipMemsetAsync(counter, 0, 8, c.stream));
  const size_t lds = size_t(n_hist) * 8;
  if (u.n > 0) {
    if (s.m || (!CROSS && b.m))
      k_ddr2_hist<true, KIND, CROSS><<<dim3(unsigned(nwg)), dim3(kHistThreads), lds, c.stream>>>(
          s, b, g.nc, g.L, lim2, inv_h, n_x, n_keep, n_hist, inv_r0, fix_scale, 0, 1, g.L, 1.0, u.cell, u.tile, u.n,
          counter, ordered, partial);
    else
      k_ddr2_hist<false, KIND, CROSS><<<dim3(unsigned(nwg)), dim3(kHistThreads), lds, c.stream>>>(
          s, b, g.nc, g.L, lim2, inv_h, n_x, n_keep, n_hist, inv_r0, fix_scale, 0, 1, g.L, 1.0, u.cell, u.tile, u.n,
          counter, ordered, partial);
    HIPSTER_HIP(hipGetLastError());
  } else {
    HIPSTER_HIP(hipMemsetAsync(partial, 0, size_t(nwg) * n_hist * 8, c.stream));
  }
  hist_reduce(c, partial, nwg, n_hist, 1.0 / fix_scale, H);
  k_ddr2_contract<<<dim3(unsigned(rows)), dim3(256), 0, c.stream>>>(table, H, n_hist, rows, out);
  HIPSTER_HIP(hipGetLastError());
}

static double weight_max(Ctx &c, const Sorted &s);

// Upper bound of the ordered (pair, image) terms of a half-stencil sweep:
// twice the candidate pairs, sum over cells of n_cell times the points of
// its 14 half-stencil cells; with a primary mask (sel = selected points per
// cell) the sum of the pairs' multiplicities, sel_c m + n_c sel_m over the
// same cells, which is what the masked sweep adds.
__global__ void k_candidate_bound(const int64_t *__restrict__ cell_start, const int64_t *__restrict__ sel, int nc,
                                  unsigned long long *__restrict__ out) {
  const int64_t ncell = int64_t(nc) * nc * nc;
  unsigned long long acc = 0;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < ncell; c += int64_t(gridDim.x) * blockDim.x) {
    const int64_t n = cell_start[c + 1] - cell_start[c];
    if (n == 0) continue;
    const int cz = int(c % nc), cy = int((c / nc) % nc), cx = int(c / (int64_t(nc) * nc));
    int64_t m = 0, ms = 0;
    for (int t = 13; t < 27; ++t) {
      const int nx = (cx + t / 9 - 1 + nc) % nc, ny = (cy + (t / 3) % 3 - 1 + nc) % nc, nz = (cz + t % 3 - 1 + nc) % nc;
      const int64_t nb = (int64_t(nx) * nc + ny) * nc + nz;
      m += cell_start[nb + 1] - cell_start[nb];
      if (sel) ms += sel[nb];
    }
    acc += sel ? static_cast<unsigned long long>(sel[c] * m + n * ms) : static_cast<unsigned long long>(2 * n * m);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

// Selected points per cell (primary mask).
__global__ __launch_bounds__(256) void k_cell_selected(const int64_t *__restrict__ cell_start,
                                                       const uint8_t *__restrict__ mask, int64_t ncell,
                                                       int64_t *__restrict__ sel) {
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= ncell) return;
  int64_t k = 0;
  for (int64_t p = cell_start[c]; p < cell_start[c + 1]; ++p) k += mask[p] ? 1 : 0;
  sel[c] = k;
}

void ddr2_sweep(Ctx &c, const Sorted &s, const Grid &g, double r0, int n_x, const double *table, int rows,
                double *T, unsigned long long *ordered) {
  // fixed-point scale from the candidate bound: every node's sum of
  // |w_i w_j l_q(t)| is at most (ordered candidates) * w_max^2 * 2.5 (a node
  // takes at most two basis values of a pair, each below 1.25 in size)
  unsigned long long *cb = static_cast<unsigned long long *>(ensure(c, c.ct_wmax, 8));
  HIPSTER_HIP(hipMemsetAsync(cb, 0, 8, c.stream));
  const int64_t ncell = g.ncells();
  int64_t *sel = nullptr;
  if (s.m) {
    sel = static_cast<int64_t *>(ensure(c, c.ct_sel, size_t(ncell) * 8));
    k_cell_selected<<<dim3(unsigned((ncell + 255) / 256)), dim3(256), 0, c.stream>>>(s.cell_start, s.m, ncell, sel);
    HIPSTER_HIP(hipGetLastError());
  }
  k_candidate_bound<<<dim3(unsigned(std::min<int64_t>((ncell + 255) / 256, 1024))), dim3(256), 0, c.stream>>>(
      s.cell_start, sel, g.nc, cb);
  HIPSTER_HIP(hipGetLastError());
  unsigned long long cand = 0;
  HIPSTER_HIP(hipMemcpyAsync(&cand, cb, 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  const double wm = weight_max(c, s);
  const double bound = (double(cand) + 1.0) * 2.5 * std::max(wm * wm, 1e-300);
  const int e = std::min(52, 61 - int(ceil(log2(bound))));
  hist_sweep<kHistDdr2, false>(c, s, s, g, (2.0 * r0) * (2.0 * r0), n_x / (2.0 * r0), n_x, n_x, n_x + 1, 0.0,
                               ldexp(1.0, e), table, rows, T, ordered);
}

// ------------------------------------------------------------------ C term
// F^ab_l(x_m) = jbar^a_l(x_m) jbar^b_l(x_m) on the nodes x_m = m R0 / n_c,
// m = 0 .. n_c + 2 (past R0: the quintic around r < R0 reaches node
// n_c + 2); F is even in x (jbar_l ~ x^l times a series in x^2).  The window
// is not in the table: the sweep applies W(r/R0)^2 to each pair exactly, so
// the tabulated function is entire and the interpolation error stays at
// ~5e-3 (2 k_max h)^6 of it.
// jbar^a_l(x_m) on the nodes x_m = m h for l = 0 .. n_l - 1 (plain jbar: the
// window is applied per pair), one thread per (l, a, m): J[(l n_k + a) n_nodes + m].
__global__ __launch_bounds__(256) void k_cterm_jbar(double h, int n_nodes, int n_k, int n_l,
                                                    const double *__restrict__ ek, const double *__restrict__ coef,
                                                    double *__restrict__ J) {
  __shared__ double2 tab[kSinCosTab];
  stage_sincos_tab<kSinCosTab>(tab);
  __syncthreads();
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(n_l) * n_k * n_nodes) return;
  const int m = int(idx % n_nodes), a = int((idx / n_nodes) % n_k), l = int(idx / (int64_t(n_nodes) * n_k));
  const double x = m * h;
  const double lo = ek[2 * a + 1] * G_one(l, ek[2 * a] * x, tab);
  const double hi = ek[2 * a + 3] * G_one(l, ek[2 * a + 2] * x, tab);
  J[idx] = coef[a] * (hi - lo);
}

// F[((l n_k + a) n_k + b) n_nodes + m] = jbar^a_l(x_m) jbar^b_l(x_m).
__global__ __launch_bounds__(256) void k_cterm_table(int n_nodes, int n_k, int n_l, const double *__restrict__ J,
                                                     double *__restrict__ F) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(n_l) * n_k * n_k * n_nodes) return;
  const int m = int(idx % n_nodes);
  const int64_t r = idx / n_nodes;
  const int b = int(r % n_k), a = int((r / n_k) % n_k), l = int(r / (int64_t(n_k) * n_k));
  F[idx] = J[(int64_t(l) * n_k + a) * n_nodes + m] * J[(int64_t(l) * n_k + b) * n_nodes + m];
}

int cterm_default_nodes(double r0, double k_max) {
  // 2 k_max h <= 0.1: the quintic's error is ~5e-3 (0.1)^6 = 5e-9 of F
  const double want = 2.0 * k_max * r0 / 0.1;
  int n = int(std::min(double(kEiiMaxNodes - 64), ceil(want / 64.0) * 64.0));
  return std::max(64, n);
}

// Largest |w| of a sorted catalogue (host value).
static double weight_max(Ctx &c, const Sorted &s) {
  unsigned long long *wm = static_cast<unsigned long long *>(ensure(c, c.ct_wmax, 8));
  HIPSTER_HIP(hipMemsetAsync(wm, 0, 8, c.stream));
  if (s.n > 0) {
    k_absmax<<<dim3(unsigned(std::min<int64_t>((s.n + 255) / 256, 1024))), dim3(256), 0, c.stream>>>(s.w, s.n, wm);
    HIPSTER_HIP(hipGetLastError());
  }
  unsigned long long wbits = 0;
  HIPSTER_HIP(hipMemcpyAsync(&wbits, wm, 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  double w_max;
  memcpy(&w_max, &wbits, 8);
  return w_max;
}

void cterm_sweep(Ctx &c, const Sorted &s, const Sorted &b, bool cross, const Grid &g, double r0, int n_k,
                 const double *k_edges, int ell_max, int n_c, uint64_t n_ordered, double *C,
                 unsigned long long *ordered) {
  const int n_nodes = n_c + 3, n_l = ell_max + 1, rows = n_l * n_k * n_k;
  std::vector<double> ek(static_cast<size_t>(2 * (n_k + 1))), coef(static_cast<size_t>(n_k));
  for (int e = 0; e <= n_k; ++e) {
    ek[size_t(2 * e)] = k_edges[e];
    ek[size_t(2 * e + 1)] = k_edges[e] * k_edges[e] * k_edges[e];
  }
  for (int b = 0; b < n_k; ++b) coef[size_t(b)] = 3.0 / (ek[size_t(2 * b + 3)] - ek[size_t(2 * b + 1)]);
  double *dk = static_cast<double *>(ensure(c, c.ct_consts, size_t(3 * n_k + 2) * 8));
  HIPSTER_HIP(hipMemcpyAsync(dk, ek.data(), ek.size() * 8, hipMemcpyHostToDevice, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(dk + ek.size(), coef.data(), coef.size() * 8, hipMemcpyHostToDevice, c.stream));
  double *F = static_cast<double *>(ensure(c, c.ct_tab, size_t(rows) * n_nodes * 8));
  double *J = static_cast<double *>(ensure(c, c.ct_jbar, size_t(n_l) * n_k * n_nodes * 8));
  const double h = r0 / n_c;
  const int64_t nj = int64_t(n_l) * n_k * n_nodes, nf = int64_t(rows) * n_nodes;
  k_cterm_jbar<<<dim3(unsigned((nj + 255) / 256)), dim3(256), 0, c.stream>>>(h, n_nodes, n_k, n_l, dk, dk + ek.size(),
                                                                            J);
  HIPSTER_HIP(hipGetLastError());
  k_cterm_table<<<dim3(unsigned((nf + 255) / 256)), dim3(256), 0, c.stream>>>(n_nodes, n_k, n_l, J, F);
  HIPSTER_HIP(hipGetLastError());
  // fixed-point scale: every node's sum of |w_p w_q^2 W^2 l_q(t)| is at most
  // n_ordered * max w_p * (max w_q)^2 * 2.5 (a node takes at most two basis
  // values of a pair, each below 1.25 in size), kept below 2^61
  const double wa = weight_max(c, s), wb = cross ? weight_max(c, b) : wa;
  const double bound = (double(n_ordered) + 1.0) * 2.5 * std::max(wa * wb * wb, 1e-300);
  const int e = std::min(52, 61 - int(ceil(log2(bound))));
  const double fix_scale = ldexp(1.0, e);
  if (cross)
    hist_sweep<kHistCterm, true>(c, s, b, g, r0 * r0, 1.0 / h, n_c, n_nodes, n_nodes, 1.0 / r0, fix_scale, F, rows,
                                 C, ordered);
  else
    hist_sweep<kHistCterm, false>(c, s, s, g, r0 * r0, 1.0 / h, n_c, n_nodes, n_nodes, 1.0 / r0, fix_scale, F, rows,
                                  C, ordered);
}

// ------------------------------------------------ anisotropic C term
// Table of one pass of Legendre sections: row (c, a, b), entry (sec, m) =
// q[c][L0 + sec] jbar^a_{l1(c)}(x_m) jbar^b_{l2(c)}(x_m), from the jbar table
// J [n_l][n_k][n_nodes] of k_cterm_jbar.
__global__ __launch_bounds__(256) void k_aniso_ctable(int n_nodes, int n_k, const double *__restrict__ J,
                                                      const double *__restrict__ q, const int *__restrict__ cl1,
                                                      const int *__restrict__ cl2, int n_sec_all, int L0, int ns,
                                                      int64_t rows, double *__restrict__ F) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t cols = int64_t(ns) * n_nodes;
  if (idx >= rows * cols) return;
  const int64_t row = idx / cols;
  const int col = int(idx - row * cols), sec = col / n_nodes, m = col - sec * n_nodes;
  const int b = int(row % n_k), a = int((row / n_k) % n_k), cb = int(row / (int64_t(n_k) * n_k));
  const double ja = J[(int64_t(cl1[cb]) * n_k + a) * n_nodes + m];
  const double jb = J[(int64_t(cl2[cb]) * n_k + b) * n_nodes + m];
  F[idx] = q[int64_t(cb) * n_sec_all + L0 + sec] * ja * jb;
}

template <bool MASKED, bool CROSS, int NLP>
static void launch_ctl(Ctx &c, const Sorted &s, const Sorted &b, const Grid &g, const PairUnits &u, double lim2,
                       double inv_h, int n_c, int n_nodes, double inv_r0, double fix_scale, int L0,
                       unsigned long long *counter, unsigned long long *ordered, double *partial, int nwg) {
  const size_t lds = size_t(NLP) * n_nodes * 8;
  k_ddr2_hist<MASKED, kHistCtermL, CROSS, NLP><<<dim3(unsigned(nwg)), dim3(kHistThreads), lds, c.stream>>>(
      s, b, g.nc, g.L, lim2, inv_h, n_c, n_nodes, NLP * n_nodes, inv_r0, fix_scale, L0, 1, g.L, 1.0, u.cell, u.tile,
      u.n, counter, ordered, partial);
  HIPSTER_HIP(hipGetLastError());
}

template <bool MASKED, bool CROSS>
static void launch_ctl_n(Ctx &c, int ns, const Sorted &s, const Sorted &b, const Grid &g, const PairUnits &u,
                         double lim2, double inv_h, int n_c, int n_nodes, double inv_r0, double fix_scale, int L0,
                         unsigned long long *counter, unsigned long long *ordered, double *partial, int nwg) {
  switch (ns) {
    case 1: launch_ctl<MASKED, CROSS, 1>(c, s, b, g, u, lim2, inv_h, n_c, n_nodes, inv_r0, fix_scale, L0, counter, ordered, partial, nwg); break;
    case 2: launch_ctl<MASKED, CROSS, 2>(c, s, b, g, u, lim2, inv_h, n_c, n_nodes, inv_r0, fix_scale, L0, counter, ordered, partial, nwg); break;
    case 3: launch_ctl<MASKED, CROSS, 3>(c, s, b, g, u, lim2, inv_h, n_c, n_nodes, inv_r0, fix_scale, L0, counter, ordered, partial, nwg); break;
    default: launch_ctl<MASKED, CROSS, 4>(c, s, b, g, u, lim2, inv_h, n_c, n_nodes, inv_r0, fix_scale, L0, counter, ordered, partial, nwg); break;
  }
}

void cterm_aniso_sweep(Ctx &c, const Sorted &s, const Sorted &b, bool cross, const Grid &g, double r0, int n_k,
                       const double *k_edges, int ell_max, int n_c, uint64_t n_ordered, int n_comb, const int *cl1,
                       const int *cl2, const double *q, double *C, unsigned long long *ordered) {
  const int n_nodes = n_c + 3, n_l = ell_max + 1, n_sec = 2 * ell_max + 1;
  const int64_t rows = int64_t(n_comb) * n_k * n_k;
  const size_t max_nodes = ddr2_max_nodes(c);
  const int per_pass = int(std::min<size_t>(4, max_nodes / size_t(n_nodes)));
  if (per_pass < 1) throw Error{HIPSTER_EUNSUPPORTED, "anisotropic C term: k_max R0 too large for the LDS histogram"};
  // jbar^a_l on the nodes
  std::vector<double> ek(static_cast<size_t>(2 * (n_k + 1))), coef(static_cast<size_t>(n_k));
  for (int e = 0; e <= n_k; ++e) {
    ek[size_t(2 * e)] = k_edges[e];
    ek[size_t(2 * e + 1)] = k_edges[e] * k_edges[e] * k_edges[e];
  }
  for (int a = 0; a < n_k; ++a) coef[size_t(a)] = 3.0 / (ek[size_t(2 * a + 3)] - ek[size_t(2 * a + 1)]);
  double *dk = static_cast<double *>(ensure(c, c.ct_consts, size_t(3 * n_k + 2) * 8));
  HIPSTER_HIP(hipMemcpyAsync(dk, ek.data(), ek.size() * 8, hipMemcpyHostToDevice, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(dk + ek.size(), coef.data(), coef.size() * 8, hipMemcpyHostToDevice, c.stream));
  double *J = static_cast<double *>(ensure(c, c.ct_jbar, size_t(n_l) * n_k * n_nodes * 8));
  const double h = r0 / n_c;
  const int64_t nj = int64_t(n_l) * n_k * n_nodes;
  k_cterm_jbar<<<dim3(unsigned((nj + 255) / 256)), dim3(256), 0, c.stream>>>(h, n_nodes, n_k, n_l, dk, dk + ek.size(), J);
  HIPSTER_HIP(hipGetLastError());
  // combination tables
  double *dq = static_cast<double *>(ensure(c, c.ca_q, size_t(n_comb) * n_sec * 8));
  int *dl = static_cast<int *>(ensure(c, c.ca_l, size_t(2 * n_comb) * 4));
  HIPSTER_HIP(hipMemcpyAsync(dq, q, size_t(n_comb) * n_sec * 8, hipMemcpyHostToDevice, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(dl, cl1, size_t(n_comb) * 4, hipMemcpyHostToDevice, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(dl + n_comb, cl2, size_t(n_comb) * 4, hipMemcpyHostToDevice, c.stream));
  // fixed-point scale as for the isotropic C term (|P_L| <= 1)
  const double wa = weight_max(c, s), wb = cross ? weight_max(c, b) : wa;
  const double bound = (double(n_ordered) + 1.0) * 2.5 * std::max(wa * wb * wb, 1e-300);
  const int e = std::min(52, 61 - int(ceil(log2(bound))));
  const double fix_scale = ldexp(1.0, e);
  const PairUnits u = make_pair_units(c, s, g);
  int nwg = 0;
  {
    int cus = 0;
    HIPSTER_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device));
    nwg = std::max(1, cus) * 4;
  }
  unsigned long long *counter = static_cast<unsigned long long *>(ensure(c, c.ddr2_counter, 8));
  unsigned long long *spare = static_cast<unsigned long long *>(ensure(c, c.ca_count, 8));
  double *Cd = static_cast<double *>(ensure(c, c.ca_out, size_t(rows) * 8));
  std::vector<double> part(static_cast<size_t>(rows));
  for (int64_t i = 0; i < rows; ++i) C[i] = 0.0;
  for (int L0 = 0; L0 < n_sec; L0 += per_pass) {
    const int ns = std::min(per_pass, n_sec - L0);
    const int n_hist = ns * n_nodes;
    double *F = static_cast<double *>(ensure(c, c.ca_tab, size_t(rows) * n_hist * 8));
    const int64_t nf = rows * n_hist;
    k_aniso_ctable<<<dim3(unsigned((nf + 255) / 256)), dim3(256), 0, c.stream>>>(n_nodes, n_k, J, dq, dl, dl + n_comb,
                                                                                n_sec, L0, ns, rows, F);
    HIPSTER_HIP(hipGetLastError());
    double *partial = static_cast<double *>(ensure(c, c.ddr2_partial, size_t(nwg) * n_hist * 8));
    double *H = static_cast<double *>(ensure(c, c.ddr2_hist, size_t(n_hist) * 8));
    HIPSTER_HIP(hipMemsetAsync(counter, 0, 8, c.stream));
    // the ordered pairs are counted by the first pass only
    unsigned long long *ord = L0 == 0 ? ordered : spare;
    if (u.n > 0) {
      const bool masked = s.m || (!cross && b.m);
      if (cross) {
        if (masked) launch_ctl_n<true, true>(c, ns, s, b, g, u, r0 * r0, 1.0 / h, n_c, n_nodes, 1.0 / r0, fix_scale, L0, counter, ord, partial, nwg);
        else launch_ctl_n<false, true>(c, ns, s, b, g, u, r0 * r0, 1.0 / h, n_c, n_nodes, 1.0 / r0, fix_scale, L0, counter, ord, partial, nwg);
      } else {
        if (masked) launch_ctl_n<true, false>(c, ns, s, s, g, u, r0 * r0, 1.0 / h, n_c, n_nodes, 1.0 / r0, fix_scale, L0, counter, ord, partial, nwg);
        else launch_ctl_n<false, false>(c, ns, s, s, g, u, r0 * r0, 1.0 / h, n_c, n_nodes, 1.0 / r0, fix_scale, L0, counter, ord, partial, nwg);
      }
    } else {
      HIPSTER_HIP(hipMemsetAsync(partial, 0, size_t(nwg) * n_hist * 8, c.stream));
    }
    hist_reduce(c, partial, nwg, n_hist, 1.0 / fix_scale, H);
    k_ddr2_contract<<<dim3(unsigned(rows)), dim3(256), 0, c.stream>>>(F, H, n_hist, int(rows), Cd);
    HIPSTER_HIP(hipGetLastError());
    HIPSTER_HIP(hipMemcpyAsync(part.data(), Cd, size_t(rows) * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
    for (int64_t i = 0; i < rows; ++i) C[i] += part[size_t(i)];
  }
}

// ------------------------------------------------- power spectrum, table form
// F^a_l(x_m) = jbar^a_l(x_m) on the nodes x_m = m R0 / n_c, m = 0 .. n_c + 2,
// for even l = 2 li; one thread per (li, a, m).  jbar_l is entire and even in
// x; the window is applied to each pair exactly in the sweep.
__global__ __launch_bounds__(256) void k_pktab_table(double h, int n_nodes, int n_k, int n_l,
                                                     const double *__restrict__ ek, const double *__restrict__ coef,
                                                     double *__restrict__ F) {
  __shared__ double2 tab[kSinCosTab];
  stage_sincos_tab<kSinCosTab>(tab);
  __syncthreads();
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(n_l) * n_k * n_nodes) return;
  const int m = int(idx % n_nodes), a = int((idx / n_nodes) % n_k), li = int(idx / (int64_t(n_nodes) * n_k));
  const double x = m * h;
  const double lo = ek[2 * a + 1] * G_one(2 * li, ek[2 * a] * x, tab);
  const double hi = ek[2 * a + 3] * G_one(2 * li, ek[2 * a + 2] * x, tab);
  F[idx] = coef[a] * (hi - lo);
}

int pktab_default_nodes(double r0, double k_max) {
  // k_max h <= 0.13: the quintic's error is ~5e-3 (0.13)^6 = 2.4e-8 of jbar.
  // Not capped: a count the LDS cannot hold is rejected by the caller.
  const double want = std::min(1e7, k_max * r0 / 0.13);
  return std::max(64, int(ceil(want / 64.0) * 64.0));
}

struct PkTabSweep {
  const Sorted *s, *b;  // primaries and neighbours (b == s unless cross)
  bool cross, periodic;
  int los;               // 0, 1, 2: axis; 3: pair midpoint from the origin
  double pair_scale;     // signed factor of every pair weight
  double pref_scale;     // bound on |coordinate| (with image shift)
};

template <bool MASKED, bool CROSS, int NLP>
static void launch_pktab(Ctx &c, const PkTabSweep &z, const Grid &g, const PairUnits &u, double lim2, double inv_h,
                         int n_c, int n_nodes, double inv_r0, double fix_scale, unsigned long long *counter,
                         unsigned long long *ordered, double *partial, int nwg) {
  const size_t lds = size_t(NLP) * n_nodes * 8;
  k_ddr2_hist<MASKED, kHistPk, CROSS, NLP><<<dim3(unsigned(nwg)), dim3(kHistThreads), lds, c.stream>>>(
      *z.s, *z.b, g.nc, g.L, lim2, inv_h, n_c, n_nodes, NLP * n_nodes, inv_r0, fix_scale, z.los, z.periodic ? 1 : 0,
      z.pref_scale, z.pair_scale, u.cell, u.tile, u.n, counter, ordered, partial);
  HIPSTER_HIP(hipGetLastError());
}

// Upper bound of the ordered pair terms of a sweep of `a` against `b`: twice
// the candidate pairs, the sum over cells of n_a times the points of b in its
// stencil (27 cells when cross, else the 14 of the half stencil), without
// the cells outside the grid when not periodic.
__global__ void k_candidate_bound_ab(const int64_t *__restrict__ cs_a, const int64_t *__restrict__ cs_b, int nc,
                                     int cross, int periodic, unsigned long long *__restrict__ out) {
  const int64_t ncell = int64_t(nc) * nc * nc;
  unsigned long long acc = 0;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < ncell; c += int64_t(gridDim.x) * blockDim.x) {
    const int64_t n = cs_a[c + 1] - cs_a[c];
    if (n == 0) continue;
    const int cz = int(c % nc), cy = int((c / nc) % nc), cx = int(c / (int64_t(nc) * nc));
    int64_t m = 0;
    for (int t = cross ? 0 : 13; t < 27; ++t) {
      int nx = cx + t / 9 - 1, ny = cy + (t / 3) % 3 - 1, nz = cz + t % 3 - 1;
      if (!periodic && (nx < 0 || nx >= nc || ny < 0 || ny >= nc || nz < 0 || nz >= nc)) continue;
      nx = (nx + nc) % nc;
      ny = (ny + nc) % nc;
      nz = (nz + nc) % nc;
      const int64_t nb = (int64_t(nx) * nc + ny) * nc + nz;
      m += cs_b[nb + 1] - cs_b[nb];
    }
    acc += static_cast<unsigned long long>(2 * n * m);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

template <bool CROSS, int NLP>
static int pktab_blocks_per_cu(int n_nodes) {
  int per = 0;
  HIPSTER_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per, reinterpret_cast<const void *>(&k_ddr2_hist<false, kHistPk, CROSS, NLP>), kHistThreads,
      size_t(NLP) * n_nodes * 8));
  return std::max(1, per);
}

static void pktab_sweep_one(Ctx &c, const PkTabSweep &z, const Grid &g, double r0, int n_k, const double *k_edges,
                            int n_l, int n_c, double *T, unsigned long long *ordered);

void pktab_sweep(Ctx &c, const Sorted &s, const Grid &g, double r0, int n_k, const double *k_edges, int n_l, int los,
                 int n_c, double *T, unsigned long long *ordered) {
  const PkTabSweep z{&s, &s, false, true, los, 1.0, g.L};
  pktab_sweep_one(c, z, g, r0, n_k, k_edges, n_l, n_c, T, ordered);
}

void pktab_survey_sweep(Ctx &c, const Sorted &a, const Sorted &b, bool cross, const Grid &g, double coord_bound,
                        double pair_scale, double r0, int n_k, const double *k_edges, int n_l, int n_c, double *T,
                        unsigned long long *ordered) {
  const PkTabSweep z{&a, &b, cross, false, 3, pair_scale, coord_bound};
  pktab_sweep_one(c, z, g, r0, n_k, k_edges, n_l, n_c, T, ordered);
}

static void pktab_sweep_one(Ctx &c, const PkTabSweep &z, const Grid &g, double r0, int n_k, const double *k_edges,
                            int n_l, int n_c, double *T, unsigned long long *ordered) {
  const Sorted &s = *z.s;
  const int n_nodes = n_c + 3, rows = n_l * n_k;
  if (size_t(n_l) * n_nodes > ddr2_max_nodes(c))
    throw Error{HIPSTER_EUNSUPPORTED, "table form: k_max R0 too large for the LDS histogram; use HIPSTER_MIXED"};
  const double h = r0 / n_c;
  // the table, kept while (R0, bins, multipoles, nodes) repeat
  std::vector<double> key{r0, double(n_k), double(n_l), double(n_c)};
  key.insert(key.end(), k_edges, k_edges + n_k + 1);
  double *F = static_cast<double *>(ensure(c, c.pt_tab, size_t(rows) * n_nodes * 8));
  if (key != c.pt_key) {
    c.pt_key.clear();
    std::vector<double> ek(static_cast<size_t>(2 * (n_k + 1))), coef(static_cast<size_t>(n_k));
    for (int e = 0; e <= n_k; ++e) {
      ek[size_t(2 * e)] = k_edges[e];
      ek[size_t(2 * e + 1)] = k_edges[e] * k_edges[e] * k_edges[e];
    }
    for (int b = 0; b < n_k; ++b) coef[size_t(b)] = 3.0 / (ek[size_t(2 * b + 3)] - ek[size_t(2 * b + 1)]);
    double *dk = static_cast<double *>(ensure(c, c.pt_consts, size_t(3 * n_k + 2) * 8));
    HIPSTER_HIP(hipMemcpyAsync(dk, ek.data(), ek.size() * 8, hipMemcpyHostToDevice, c.stream));
    HIPSTER_HIP(hipMemcpyAsync(dk + ek.size(), coef.data(), coef.size() * 8, hipMemcpyHostToDevice, c.stream));
    const int64_t nt = int64_t(rows) * n_nodes;
    k_pktab_table<<<dim3(unsigned((nt + 255) / 256)), dim3(256), 0, c.stream>>>(h, n_nodes, n_k, n_l, dk,
                                                                               dk + ek.size(), F);
    HIPSTER_HIP(hipGetLastError());
    HIPSTER_HIP(hipStreamSynchronize(c.stream));  // the host arrays above go out of scope
    c.pt_key = key;
  }
  // fixed-point scale from the candidate bound: every node's sum of
  // |s w_i w_j W L_l l_q(t)| is at most (ordered candidates) * |s| w_a w_b * 2.5
  // (|W|, |L_l| <= 1; a node takes at most two basis values of a pair, each
  // below 1.25 in size), kept below 2^61; and one add, at most 2 |s| w_a w_b
  // 1.25 (both orientations), below 2^30.  The unit of the sums is then at
  // most 2^-29 of the largest add, so the rounding stays below ~2e-9 of the
  // bin's L1 mass
  unsigned long long *cb = static_cast<unsigned long long *>(ensure(c, c.ct_wmax, 8));
  HIPSTER_HIP(hipMemsetAsync(cb, 0, 8, c.stream));
  const int64_t ncell = g.ncells();
  k_candidate_bound_ab<<<dim3(unsigned(std::min<int64_t>((ncell + 255) / 256, 1024))), dim3(256), 0, c.stream>>>(
      s.cell_start, z.b->cell_start, g.nc, z.cross ? 1 : 0, z.periodic ? 1 : 0, cb);
  HIPSTER_HIP(hipGetLastError());
  unsigned long long cand = 0;
  HIPSTER_HIP(hipMemcpyAsync(&cand, cb, 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  const double wa = weight_max(c, s), wb = z.cross ? weight_max(c, *z.b) : wa;
  const double wab = std::max(fabs(z.pair_scale) * wa * wb, 1e-300);
  const double bound = (double(cand) + 1.0) * 2.5 * wab;
  const double one_add = 2.5 * wab;
  const int e = std::min(61 - int(ceil(log2(bound))), 30 - int(ceil(log2(one_add))));
  const double fix_scale = ldexp(1.0, e);

  const PairUnits u = make_pair_units(c, s, g);
  int cus = 0;
  HIPSTER_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device));
  int per = 1;
  switch (n_l) {
    case 1: per = z.cross ? pktab_blocks_per_cu<true, 1>(n_nodes) : pktab_blocks_per_cu<false, 1>(n_nodes); break;
    case 2: per = z.cross ? pktab_blocks_per_cu<true, 2>(n_nodes) : pktab_blocks_per_cu<false, 2>(n_nodes); break;
    case 3: per = z.cross ? pktab_blocks_per_cu<true, 3>(n_nodes) : pktab_blocks_per_cu<false, 3>(n_nodes); break;
    default: per = z.cross ? pktab_blocks_per_cu<true, 4>(n_nodes) : pktab_blocks_per_cu<false, 4>(n_nodes); break;
  }
  const int nwg = std::max(1, cus) * per;
  const int n_hist = n_l * n_nodes;
  double *partial = static_cast<double *>(ensure(c, c.ddr2_partial, size_t(nwg) * n_hist * 8));
  double *H = static_cast<double *>(ensure(c, c.ddr2_hist, size_t(n_hist) * 8));
  unsigned long long *counter = static_cast<unsigned long long *>(ensure(c, c.ddr2_counter, 8));
  HIPSTER_HIP(hipMemsetAsync(counter, 0, 8, c.stream));
  const double lim2 = r0 * r0, inv_h = 1.0 / h, inv_r0 = 1.0 / r0;
  if (u.n > 0) {
    const bool masked = s.m != nullptr || z.b->m != nullptr;
#define HIPSTER_PKTAB(M, X, N)                                                                                       \
  launch_pktab<M, X, N>(c, z, g, u, lim2, inv_h, n_c, n_nodes, inv_r0, fix_scale, counter, ordered, partial, nwg)
#define HIPSTER_PKTAB_M(X, N)                                                                                        \
  do {                                                                                                               \
    if (masked) HIPSTER_PKTAB(true, X, N); else HIPSTER_PKTAB(false, X, N);                                          \
  } while (0)
#define HIPSTER_PKTAB_XM(N)                                                                                          \
  do {                                                                                                               \
    if (z.cross) HIPSTER_PKTAB_M(true, N); else HIPSTER_PKTAB_M(false, N);                                           \
  } while (0)
    switch (n_l) {
      case 1: HIPSTER_PKTAB_XM(1); break;
      case 2: HIPSTER_PKTAB_XM(2); break;
      case 3: HIPSTER_PKTAB_XM(3); break;
      default: HIPSTER_PKTAB_XM(4); break;
    }
#undef HIPSTER_PKTAB_XM
#undef HIPSTER_PKTAB_M
#undef HIPSTER_PKTAB
  } else {
    HIPSTER_HIP(hipMemsetAsync(partial, 0, size_t(nwg) * n_hist * 8, c.stream));
  }
  hist_reduce(c, partial, nwg, n_hist, 1.0 / fix_scale, H);
  k_ddr2_contract<<<dim3(unsigned(rows)), dim3(256), 0, c.stream>>>(F, H, n_nodes, n_k, T);
  HIPSTER_HIP(hipGetLastError());
}

}  // namespace hipster

namespace hipster {

// ------------------------------------------------------------ theory side
// The transforms behind the windowed theory and the covariance of the binned
// multipoles (Secs. 5, 6):
//   omega^a_l(p) = 4 pi int_0^R0 r^2 j_l(p r) jbar^a_l(r) W(r/R0) dr,
// on one node set for all requested p: the three smooth pieces of W cut into
// 16-point Gauss-Legendre panels no wider than min(R0/4, 8/max(p_max, k_max))
// (the integrand oscillates at up to p + k, so a panel spans at most 16
// radians).  Tables g[l][m][a] = jbar^a_l(r_m) W(r_m/R0) and
// J[l][i][m] = w_m r_m^2 j_l(p_i r_m), then fixed-order sums.

// Spherical Bessel j_l(x), double precision: the power series
// x^l/(2l+1)!! sum_s (-x^2/2)^s/(s! (2l+3)..(2l+2s+1)) below x = l + 4 (at
// most ~3 digits of cancellation), else j_0 = sin x/x, j_1 = sin x/x^2 -
// cos x/x and the upward recurrence, stable for x > l.
__device__ inline double sph_jl(int l, double x, const double2 *__restrict__ tab) {
  if (x < double(l) + 4.0) {
    double t = 1.0;
    for (int q = 1; q <= l; ++q) t *= x / double(2 * q + 1);
    double sum = 0.0;
    const double h = -0.5 * x * x;
    for (int s = 0; s < 40; ++s) {
      sum += t;
      t *= h / (double(s + 1) * double(2 * l + 2 * s + 3));
    }
    return sum;
  }
  double sn, cs;
  sincos_tab<kSinCosTab, true>(x, tab, sn, cs);
  const double w = 1.0 / x;
  double j0 = sn * w, j1 = (sn * w - cs) * w;
  if (l == 0) return j0;
  for (int n = 1; n < l; ++n) {
    const double j2 = double(2 * n + 1) * w * j1 - j0;
    j0 = j1;
    j1 = j2;
  }
  return j1;
}

// jbar^a_l(r) from the edge values G_l(k r): 3 (k_{a+1}^3 G(k_{a+1} r) -
// k_a^3 G(k_a r)) / (k_{a+1}^3 - k_a^3).  ek: (k, k^3) per edge.
__device__ inline double jbar_one(int l, int a, double r, const double *__restrict__ ek,
                                  const double2 *__restrict__ tab) {
  const double ka = ek[2 * a], ka3 = ek[2 * a + 1], kb = ek[2 * a + 2], kb3 = ek[2 * a + 3];
  return 3.0 * (kb3 * G_one(l, kb * r, tab) - ka3 * G_one(l, ka * r, tab)) / (kb3 - ka3);
}

// g[l][m][a] = jbar^a_l(r_m) W(r_m / R0), one thread per entry.
__global__ __launch_bounds__(256) void k_theory_g(const double *__restrict__ r, int n_r, int n_k, int n_l,
                                                  int l_step, double inv_r0, const double *__restrict__ ek,
                                                  double *__restrict__ g) {
  __shared__ double2 tab[kSinCosTab];
  stage_sincos_tab<kSinCosTab>(tab);
  __syncthreads();
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(n_l) * n_r * n_k) return;
  const int a = int(idx % n_k), m = int((idx / n_k) % n_r), li = int(idx / (int64_t(n_k) * n_r));
  g[idx] = jbar_one(li * l_step, a, r[m], ek, tab) * window<double>(r[m] * inv_r0);
}

// J[l][i][m] = w_m r_m^2 j_l(p_i r_m), one thread per entry.
__global__ __launch_bounds__(256) void k_theory_j(const double *__restrict__ r, const double *__restrict__ wr,
                                                  int n_r, const double *__restrict__ p, int n_p, int n_l, int l_step,
                                                  double *__restrict__ J) {
  __shared__ double2 tab[kSinCosTab];
  stage_sincos_tab<kSinCosTab>(tab);
  __syncthreads();
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(n_l) * n_p * n_r) return;
  const int m = int(idx % n_r), i = int((idx / n_r) % n_p), li = int(idx / (int64_t(n_r) * n_p));
  J[idx] = wr[m] * r[m] * r[m] * sph_jl(li * l_step, p[i] * r[m], tab);
}

// omega[l][i][a] = 4 pi sum_m J[l][i][m] g[l][m][a], one thread per entry, m
// in order.
__global__ __launch_bounds__(256) void k_theory_omega(const double *__restrict__ J, const double *__restrict__ g,
                                                      int n_r, int n_p, int n_k, int n_l, double *__restrict__ om) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(n_l) * n_p * n_k) return;
  const int a = int(idx % n_k), i = int((idx / n_k) % n_p), li = int(idx / (int64_t(n_k) * n_p));
  const double *Jr = J + (int64_t(li) * n_p + i) * n_r, *gr = g + int64_t(li) * n_r * n_k + a;
  double s = 0.0;
  for (int m = 0; m < n_r; ++m) s = fma(Jr[m], gr[int64_t(m) * n_k], s);
  om[idx] = 4.0 * kPi * s;
}

// Windowed multipoles of a model 2PCF: out[l][a] = 4 pi (-i)^l sum_m wr_m
// r_m^2 xi_l(r_m) g[l][m][a] (even l), one thread per entry.
__global__ __launch_bounds__(256) void k_theory_pk(const double *__restrict__ r, const double *__restrict__ wr,
                                                   const double *__restrict__ xi, const double *__restrict__ g,
                                                   int n_r, int n_k, int n_l, double *__restrict__ out) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= n_l * n_k) return;
  const int a = idx % n_k, li = idx / n_k;
  double s = 0.0;
  for (int m = 0; m < n_r; ++m)
    s = fma(wr[m] * r[m] * r[m] * xi[int64_t(li) * n_r + m], g[(int64_t(li) * n_r + m) * n_k + a], s);
  out[idx] = 4.0 * kPi * ((li & 1) ? -1.0 : 1.0) * s;
}

// fq[l][l'][i] = wp_i p_i^2/(2 pi^2) Q_ll'(p_i), Q_ll'(p) = sum_{l1 l2}
// K[l][l'][l1][l2] P_l1(p) P_l2(p); one thread per entry.
__global__ __launch_bounds__(256) void k_theory_q(const double *__restrict__ p, const double *__restrict__ wp,
                                                  const double *__restrict__ pk, const double *__restrict__ K,
                                                  int n_p, int n_l, double *__restrict__ fq) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(n_l) * n_l * n_p) return;
  const int i = int(idx % n_p), ll = int(idx / n_p);
  const double *Kll = K + ll * n_l * n_l;
  double Q = 0.0;
  for (int m1 = 0; m1 < n_l; ++m1) {
    double t = 0.0;
    for (int m2 = 0; m2 < n_l; ++m2) t = fma(Kll[m1 * n_l + m2], pk[int64_t(m2) * n_p + i], t);
    Q = fma(t, pk[int64_t(m1) * n_p + i], Q);
  }
  fq[idx] = wp[i] * p[i] * p[i] * (1.0 / (2.0 * kPi * kPi)) * Q;
}

// Gaussian covariance: out[(l a)(l' b)] = 2 (2l+1)(2l'+1)/V sum_i
// fq[l][l'][i] omega[l][i][a] omega[l'][i][b]; one thread per entry, i in
// order.
__global__ __launch_bounds__(256) void k_theory_cov(const double *__restrict__ om, const double *__restrict__ fq,
                                                    int n_p, int n_k, int n_l, double inv_volume,
                                                    double *__restrict__ out) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t nrow = int64_t(n_l) * n_k;
  if (idx >= nrow * nrow) return;
  const int b = int(idx % n_k), lj = int((idx / n_k) % n_l), a = int((idx / (int64_t(n_k) * n_l)) % n_k),
            li = int(idx / (int64_t(n_k) * n_l * n_k));
  const double *f = fq + int64_t(li * n_l + lj) * n_p;
  const double *oa = om + int64_t(li) * n_p * n_k + a, *ob = om + int64_t(lj) * n_p * n_k + b;
  double s = 0.0;
  for (int i = 0; i < n_p; ++i) s = fma(f[i] * oa[int64_t(i) * n_k], ob[int64_t(i) * n_k], s);
  out[idx] = 2.0 * double(4 * li + 1) * double(4 * lj + 1) * inv_volume * s;
}

// Poisson two-point covariance: out[(l a)(l' b)] = pref_ll' sum_m wr_m r_m^2
// g[l][m][a] g[l'][m][b] (delta_ll'/(2l+1) + sum_L K3[L][l][l'] xi_L(r_m)),
// pref_ll' = 2/(n^2 V) (2l+1)(2l'+1)(-1)^((l+l')/2) 4 pi; one thread per
// entry, m in order.
__global__ __launch_bounds__(256) void k_theory_c2(const double *__restrict__ r, const double *__restrict__ wr,
                                                   const double *__restrict__ xi, const double *__restrict__ g,
                                                   const double *__restrict__ K3, int n_r, int n_k, int n_l,
                                                   double scale, double *__restrict__ out) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t nrow = int64_t(n_l) * n_k;
  if (idx >= nrow * nrow) return;
  const int b = int(idx % n_k), lj = int((idx / n_k) % n_l), a = int((idx / (int64_t(n_k) * n_l)) % n_k),
            li = int(idx / (int64_t(n_k) * n_l * n_k));
  const double diag = li == lj ? 1.0 / double(4 * li + 1) : 0.0;
  double s = 0.0;
  for (int m = 0; m < n_r; ++m) {
    double br = diag;
    for (int L = 0; L < n_l; ++L) br = fma(K3[(L * n_l + li) * n_l + lj], xi[int64_t(L) * n_r + m], br);
    s = fma(wr[m] * r[m] * r[m] * g[(int64_t(li) * n_r + m) * n_k + a] * br, g[(int64_t(lj) * n_r + m) * n_k + b], s);
  }
  const double pref = scale * double(4 * li + 1) * double(4 * lj + 1) * (((li + lj) & 1) ? -1.0 : 1.0) * 4.0 * kPi;
  out[idx] = pref * s;
}

// fq[l][l'][i] = wp_i p_i^2/(2 pi^2) sum_L K3[L][l][l'] P_L(p_i): the P_L
// part of the Poisson three-point term, one thread per entry.
__global__ __launch_bounds__(256) void k_theory_q3(const double *__restrict__ p, const double *__restrict__ wp,
                                                   const double *__restrict__ pk, const double *__restrict__ K3,
                                                   int n_p, int n_l, double *__restrict__ fq) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(n_l) * n_l * n_p) return;
  const int i = int(idx % n_p), ll = int(idx / n_p);
  double s = 0.0;
  for (int L = 0; L < n_l; ++L) s = fma(K3[L * n_l * n_l + ll], pk[int64_t(L) * n_p + i], s);
  fq[idx] = wp[i] * p[i] * p[i] * (1.0 / (2.0 * kPi * kPi)) * s;
}

// The measured-quantity terms of the Poisson three-point covariance:
// out[(l a)(l' b)] += f0 [W~_a W~_b d_l0 d_l'0 + W~_a P[l'][b] d_l0
// + W~_b P[l][a] d_l'0 + B[l][a][b] d_ll'] (P, B may be null: zero).
__global__ __launch_bounds__(256) void k_theory_c3_add(const double *__restrict__ wt, const double *__restrict__ pb,
                                                       const double *__restrict__ bk, int n_k, int n_l, double f0,
                                                       double *__restrict__ out) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t nrow = int64_t(n_l) * n_k;
  if (idx >= nrow * nrow) return;
  const int b = int(idx % n_k), lj = int((idx / n_k) % n_l), a = int((idx / (int64_t(n_k) * n_l)) % n_k),
            li = int(idx / (int64_t(n_k) * n_l * n_k));
  double t = 0.0;
  if (li == 0 && lj == 0) t += wt[a] * wt[b];
  if (pb && li == 0) t += wt[a] * pb[lj * n_k + b];
  if (pb && lj == 0) t += wt[b] * pb[li * n_k + a];
  if (bk && li == lj) t += bk[(int64_t(li) * n_k + a) * n_k + b];
  out[idx] += f0 * t;
}

// Non-Gaussian term, first contraction: X[l l'][i][b] = sum_j T[l l'][i][j]
// u_j omega[l'][j][b], u_j = wp_j p_j^2/(2 pi^2); one thread per entry, j in
// order.
__global__ __launch_bounds__(256) void k_theory_ng_x(const double *__restrict__ p, const double *__restrict__ wp,
                                                     const double *__restrict__ T, const double *__restrict__ om,
                                                     int n_p, int n_k, int n_l, double *__restrict__ X) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(n_l) * n_l * n_p * n_k) return;
  const int b = int(idx % n_k), i = int((idx / n_k) % n_p), ll = int(idx / (int64_t(n_k) * n_p));
  const int lj = ll % n_l;
  const double *Ti = T + (int64_t(ll) * n_p + i) * n_p, *ob = om + int64_t(lj) * n_p * n_k + b;
  double s = 0.0;
  for (int j = 0; j < n_p; ++j)
    s = fma(Ti[j] * (wp[j] * p[j] * p[j] * (1.0 / (2.0 * kPi * kPi))), ob[int64_t(j) * n_k], s);
  X[idx] = s;
}

// Non-Gaussian term: out[(l a)(l' b)] = (2l+1)(2l'+1)/V sum_i u_i
// omega[l][i][a] X[l l'][i][b] ((-1)^(l+l') = 1 for even l, l'); one thread
// per entry, i in order.
__global__ __launch_bounds__(256) void k_theory_ng_c(const double *__restrict__ p, const double *__restrict__ wp,
                                                     const double *__restrict__ om, const double *__restrict__ X,
                                                     int n_p, int n_k, int n_l, double inv_volume,
                                                     double *__restrict__ out) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t nrow = int64_t(n_l) * n_k;
  if (idx >= nrow * nrow) return;
  const int b = int(idx % n_k), lj = int((idx / n_k) % n_l), a = int((idx / (int64_t(n_k) * n_l)) % n_k),
            li = int(idx / (int64_t(n_k) * n_l * n_k));
  const double *oa = om + int64_t(li) * n_p * n_k + a, *xb = X + int64_t(li * n_l + lj) * n_p * n_k + b;
  double s = 0.0;
  for (int i = 0; i < n_p; ++i)
    s = fma((wp[i] * p[i] * p[i] * (1.0 / (2.0 * kPi * kPi))) * oa[int64_t(i) * n_k], xb[int64_t(i) * n_k], s);
  out[idx] = double(4 * li + 1) * double(4 * lj + 1) * inv_volume * s;
}

// The r node set: 16-point Gauss-Legendre panels on [0, R0/2], [R0/2, 3R0/4],
// [3R0/4, R0], each no wider than hmax.
static void theory_nodes(double r0, double hmax, std::vector<double> &r, std::vector<double> &w) {
  const GLRule gl = gauss_legendre16();
  const double cut[4] = {0.0, 0.5 * r0, 0.75 * r0, r0};
  for (int s = 0; s < 3; ++s) {
    const int np = std::max(1, int(ceil((cut[s + 1] - cut[s]) / hmax)));
    const double ph = (cut[s + 1] - cut[s]) / np;
    for (int q = 0; q < np; ++q)
      for (int j = 0; j < kGL; ++j) {
        r.push_back(cut[s] + (q + 0.5) * ph + 0.5 * ph * gl.x[j]);
        w.push_back(0.5 * ph * gl.w[j]);
      }
  }
}

static double *upload(Ctx &c, DevBuf &b, const double *h, size_t n) {
  double *d = static_cast<double *>(ensure(c, b, std::max<size_t>(n, 1) * 8));
  if (n) HIPSTER_HIP(hipMemcpyAsync(d, h, n * 8, hipMemcpyHostToDevice, c.stream));
  return d;
}

static double *edge_table(Ctx &c, int n_k, const double *k_edges) {
  std::vector<double> ek(static_cast<size_t>(2 * (n_k + 1)));
  for (int e = 0; e <= n_k; ++e) {
    ek[size_t(2 * e)] = k_edges[e];
    ek[size_t(2 * e + 1)] = k_edges[e] * k_edges[e] * k_edges[e];
  }
  return upload(c, c.th_ek, ek.data(), ek.size());
}

static unsigned blocks(int64_t n) { return unsigned((n + 255) / 256); }

void theory_omega(Ctx &c, double r0, int n_k, const double *k_edges, int n_l, int l_step, int n_p, const double *p,
                  double *om_dev) {
  double pmax = 0.0;
  for (int i = 0; i < n_p; ++i) pmax = std::max(pmax, p[i]);
  std::vector<double> r, w;
  theory_nodes(r0, std::min(0.25 * r0, 8.0 / std::max(pmax, k_edges[n_k])), r, w);
  const int n_r = int(r.size());
  const double *rd = upload(c, c.th_r, r.data(), r.size()), *wd = upload(c, c.th_w, w.data(), w.size());
  const double *pd = upload(c, c.th_p, p, size_t(n_p));
  const double *ek = edge_table(c, n_k, k_edges);
  double *g = static_cast<double *>(ensure(c, c.th_g, size_t(n_l) * n_r * n_k * 8));
  double *J = static_cast<double *>(ensure(c, c.th_J, size_t(n_l) * n_p * n_r * 8));
  k_theory_g<<<blocks(int64_t(n_l) * n_r * n_k), 256, 0, c.stream>>>(rd, n_r, n_k, n_l, l_step, 1.0 / r0, ek, g);
  HIPSTER_HIP(hipGetLastError());
  k_theory_j<<<blocks(int64_t(n_l) * n_p * n_r), 256, 0, c.stream>>>(rd, wd, n_r, pd, n_p, n_l, l_step, J);
  HIPSTER_HIP(hipGetLastError());
  k_theory_omega<<<blocks(int64_t(n_l) * n_p * n_k), 256, 0, c.stream>>>(J, g, n_r, n_p, n_k, n_l, om_dev);
  HIPSTER_HIP(hipGetLastError());
}

void theory_pk(Ctx &c, double r0, int n_k, const double *k_edges, int n_l, int n_r, const double *r, const double *wr,
               const double *xi, double *out_dev) {
  const double *rd = upload(c, c.th_r, r, size_t(n_r)), *wd = upload(c, c.th_w, wr, size_t(n_r));
  const double *xd = upload(c, c.th_p, xi, size_t(n_l) * n_r);
  const double *ek = edge_table(c, n_k, k_edges);
  double *g = static_cast<double *>(ensure(c, c.th_g, size_t(n_l) * n_r * n_k * 8));
  k_theory_g<<<blocks(int64_t(n_l) * n_r * n_k), 256, 0, c.stream>>>(rd, n_r, n_k, n_l, 2, 1.0 / r0, ek, g);
  HIPSTER_HIP(hipGetLastError());
  k_theory_pk<<<blocks(int64_t(n_l) * n_k), 256, 0, c.stream>>>(rd, wd, xd, g, n_r, n_k, n_l, out_dev);
  HIPSTER_HIP(hipGetLastError());
}

// K[l][l'][l1][l2] = sum_L (2L+1) (l l' L; 0 0 0)^2 (l1 l2 L; 0 0 0)^2 for even
// l, l', l1, l2 <= 2 (n_l - 1), from the Gaunt relation
//   (1/2) int_{-1}^{1} L_a L_b L_c L_d dmu = sum_L (2L+1) (a b L;000)^2 (c d L;000)^2,
// taken as a Gauss-Legendre sum (exact: the integrand has degree <= 24).
static std::vector<double> gaunt_coefficients(int n_l) {
  constexpr int kN = 16;
  GLRule gl = gauss_legendre16();
  (void)kN;
  const int lmax = 2 * (n_l - 1);
  std::vector<double> P(size_t((lmax + 1) * kGL));
  for (int q = 0; q < kGL; ++q) {
    const double mu = gl.x[q];
    double p0 = 1.0, p1 = mu;
    P[size_t(q)] = 1.0;
    if (lmax >= 1) P[size_t(kGL + q)] = mu;
    for (int n = 1; n < lmax; ++n) {
      const double p2 = ((2 * n + 1) * mu * p1 - n * p0) / (n + 1);
      p0 = p1;
      p1 = p2;
      P[size_t((n + 1) * kGL + q)] = p2;
    }
  }
  std::vector<double> K(size_t(n_l * n_l * n_l * n_l));
  for (int a = 0; a < n_l; ++a)
    for (int b = 0; b < n_l; ++b)
      for (int c = 0; c < n_l; ++c)
        for (int d = 0; d < n_l; ++d) {
          double s = 0.0;
          for (int q = 0; q < kGL; ++q)
            s += gl.w[q] * P[size_t(2 * a * kGL + q)] * P[size_t(2 * b * kGL + q)] * P[size_t(2 * c * kGL + q)] *
                 P[size_t(2 * d * kGL + q)];
          K[size_t(((a * n_l + b) * n_l + c) * n_l + d)] = 0.5 * s;
        }
  return K;
}

// K3[L][l][l'] = (L l l'; 0 0 0)^2 = (1/2) int_{-1}^{1} L_L L_l L_l' dmu for
// even L, l, l' <= 2 (n_l - 1), as an exact 16-point Gauss-Legendre sum.
static std::vector<double> gaunt3(int n_l) {
  const GLRule gl = gauss_legendre16();
  const int lmax = 2 * (n_l - 1);
  std::vector<double> P(size_t((lmax + 1) * kGL));
  for (int q = 0; q < kGL; ++q) {
    const double mu = gl.x[q];
    double p0 = 1.0, p1 = mu;
    P[size_t(q)] = 1.0;
    if (lmax >= 1) P[size_t(kGL + q)] = mu;
    for (int n = 1; n < lmax; ++n) {
      const double p2 = ((2 * n + 1) * mu * p1 - n * p0) / (n + 1);
      p0 = p1;
      p1 = p2;
      P[size_t((n + 1) * kGL + q)] = p2;
    }
  }
  std::vector<double> K(size_t(n_l * n_l * n_l));
  for (int L = 0; L < n_l; ++L)
    for (int a = 0; a < n_l; ++a)
      for (int b = 0; b < n_l; ++b) {
        double s = 0.0;
        for (int q = 0; q < kGL; ++q)
          s += gl.w[q] * P[size_t(2 * L * kGL + q)] * P[size_t(2 * a * kGL + q)] * P[size_t(2 * b * kGL + q)];
        K[size_t((L * n_l + a) * n_l + b)] = 0.5 * s;
      }
  return K;
}

void theory_c2(Ctx &c, double r0, double nbar, double volume, int n_k, const double *k_edges, int n_l, int n_r,
               const double *r, const double *wr, const double *xi, double *out_dev) {
  const double *rd = upload(c, c.th_r, r, size_t(n_r)), *wd = upload(c, c.th_w, wr, size_t(n_r));
  const double *xd = upload(c, c.th_p, xi, size_t(n_l) * n_r);
  const double *ek = edge_table(c, n_k, k_edges);
  const std::vector<double> K3 = gaunt3(n_l);
  const double *Kd = upload(c, c.th_K, K3.data(), K3.size());
  double *g = static_cast<double *>(ensure(c, c.th_g, size_t(n_l) * n_r * n_k * 8));
  k_theory_g<<<blocks(int64_t(n_l) * n_r * n_k), 256, 0, c.stream>>>(rd, n_r, n_k, n_l, 2, 1.0 / r0, ek, g);
  HIPSTER_HIP(hipGetLastError());
  const int64_t nout = int64_t(n_l) * n_k * n_l * n_k;
  k_theory_c2<<<blocks(nout), 256, 0, c.stream>>>(rd, wd, xd, g, Kd, n_r, n_k, n_l, 2.0 / (nbar * nbar * volume),
                                                   out_dev);
  HIPSTER_HIP(hipGetLastError());
}

void theory_cov(Ctx &c, double r0, double volume, int n_k, const double *k_edges, int n_l, int n_p, const double *p,
                const double *wp, const double *pk, double *out_dev) {
  double *om = static_cast<double *>(ensure(c, c.th_om, size_t(n_l) * n_p * n_k * 8));
  theory_omega(c, r0, n_k, k_edges, n_l, 2, n_p, p, om);
  const std::vector<double> K = gaunt_coefficients(n_l);
  const double *Kd = upload(c, c.th_K, K.data(), K.size());
  const double *pd = upload(c, c.th_p, p, size_t(n_p)), *wd = upload(c, c.th_wp, wp, size_t(n_p));
  const double *pkd = upload(c, c.th_pk, pk, size_t(n_l) * n_p);
  double *fq = static_cast<double *>(ensure(c, c.th_J, size_t(n_l) * n_l * n_p * 8));  // J is no longer needed
  k_theory_q<<<blocks(int64_t(n_l) * n_l * n_p), 256, 0, c.stream>>>(pd, wd, pkd, Kd, n_p, n_l, fq);
  HIPSTER_HIP(hipGetLastError());
  const int64_t nout = int64_t(n_l) * n_k * n_l * n_k;
  k_theory_cov<<<blocks(nout), 256, 0, c.stream>>>(om, fq, n_p, n_k, n_l, 1.0 / volume, out_dev);
  HIPSTER_HIP(hipGetLastError());
}

void theory_c3(Ctx &c, double r0, double nbar, double volume, int n_k, const double *k_edges, int n_l, int n_p,
               const double *p, const double *wp, const double *pk, const double *wt, const double *pbin,
               const double *bk, double *out_dev) {
  double *om = static_cast<double *>(ensure(c, c.th_om, size_t(n_l) * n_p * n_k * 8));
  theory_omega(c, r0, n_k, k_edges, n_l, 2, n_p, p, om);
  const std::vector<double> K3 = gaunt3(n_l);
  const double *Kd = upload(c, c.th_K, K3.data(), K3.size());
  const double *pd = upload(c, c.th_p, p, size_t(n_p)), *wd = upload(c, c.th_wp, wp, size_t(n_p));
  const double *pkd = upload(c, c.th_pk, pk, size_t(n_l) * n_p);
  double *fq = static_cast<double *>(ensure(c, c.th_J, size_t(n_l) * n_l * n_p * 8));
  k_theory_q3<<<blocks(int64_t(n_l) * n_l * n_p), 256, 0, c.stream>>>(pd, wd, pkd, Kd, n_p, n_l, fq);
  HIPSTER_HIP(hipGetLastError());
  const int64_t nout = int64_t(n_l) * n_k * n_l * n_k;
  // k_theory_cov scales by 2 (2l+1)(2l'+1) x its last factor: 2/(n V) gives
  // 4/(n V); (-1)^l is 1 for the even multipoles
  k_theory_cov<<<blocks(nout), 256, 0, c.stream>>>(om, fq, n_p, n_k, n_l, 2.0 / (nbar * volume), out_dev);
  HIPSTER_HIP(hipGetLastError());
  const double *wtd = upload(c, c.th_wt, wt, size_t(n_k));
  const double *pbd = pbin ? upload(c, c.th_pb, pbin, size_t(n_l) * n_k) : nullptr;
  const double *bkd = bk ? upload(c, c.th_bk, bk, size_t(n_l) * n_k * n_k) : nullptr;
  k_theory_c3_add<<<blocks(nout), 256, 0, c.stream>>>(wtd, pbd, bkd, n_k, n_l, 4.0 / (nbar * volume), out_dev);
  HIPSTER_HIP(hipGetLastError());
}

void theory_ng(Ctx &c, double r0, double volume, int n_k, const double *k_edges, int n_l, int n_p, const double *p,
               const double *wp, const double *tbar, double *out_dev) {
  double *om = static_cast<double *>(ensure(c, c.th_om, size_t(n_l) * n_p * n_k * 8));
  theory_omega(c, r0, n_k, k_edges, n_l, 2, n_p, p, om);
  const double *pd = upload(c, c.th_p, p, size_t(n_p)), *wd = upload(c, c.th_wp, wp, size_t(n_p));
  const double *Td = upload(c, c.th_T, tbar, size_t(n_l) * n_l * n_p * n_p);
  const int64_t nx = int64_t(n_l) * n_l * n_p * n_k;
  double *X = static_cast<double *>(ensure(c, c.th_X, size_t(nx) * 8));
  k_theory_ng_x<<<blocks(nx), 256, 0, c.stream>>>(pd, wd, Td, om, n_p, n_k, n_l, X);
  HIPSTER_HIP(hipGetLastError());
  const int64_t nout = int64_t(n_l) * n_k * n_l * n_k;
  k_theory_ng_c<<<blocks(nout), 256, 0, c.stream>>>(pd, wd, om, X, n_p, n_k, n_l, 1.0 / volume, out_dev);
  HIPSTER_HIP(hipGetLastError());
}

}  // namespace hipster
