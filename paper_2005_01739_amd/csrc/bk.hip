// Bispectrum path (Sec. 4): per-primary spherical-harmonic coefficients
//   A^a_lm(x_p) = sum_j w_j jbar^a_l(r_pj) W(r_pj/R0) y_lm(xhat_pj)      (eq. AC-def)
//   C^ab_l(x_p) = sum_j w_j^2 jbar^a_l jbar^b_l W^2
// for data primaries (j != p) and random primaries (all data j), contracted
// per primary into G^ab_l += w_p (4 pi/(2l+1)) sum_m A^a_lm A^b_lm, with
// real orthonormal harmonics y_lm (the sum over m is basis independent).
// Data primaries also give S0^b = sum_{p != j} w_p w_j jbar^b_0 W, the pair sum
// of the analytic DDR^I term.
//
// Enumeration: one wave per home cell of the primary catalogue; for each of
// its primaries in sorted order, the 27 neighbour cells of the data grid are
// flattened into one candidate range that the wave sweeps 64 at a time,
// compacting the pairs inside R0 into a per-primary contiguous stream (r,
// unit vector, w_j).  A count pass sizes every primary's segment first, so
// the stream's order -- and every sum -- is deterministic.
//
// Sweep: one wave per primary.  Lanes take 64 (32 in the FP64 form) of its
// neighbours, evaluate the bin values g^a_l = W jbar^a_l and y_lm, and stage
// w_j g^a_l and y_lm in LDS; each lane then owns a fixed set of A, C, S0 and
// G outputs, which it accumulates in double precision.
#include <type_traits>

#include "common.h"
#include "specfun.h"

namespace hipster {

__device__ inline int bk_wrap(int v, int nc, int &shift) {
  shift = 0;
  if (v >= nc) {
    shift = 1;
    return v - nc;
  }
  if (v < 0) {
    shift = -1;
    return v + nc;
  }
  return v;
}

__device__ inline double bk_image(double d, int shift, double L) {
  return shift > 0 ? d - L : (shift < 0 ? d + L : d);
}

__device__ inline double bk_sq_norm(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  double a = dx * dx;
  double b = dy * dy;
  double c = dz * dz;
  return (a + b) + c;
}

template <bool WRITE>
__global__ __launch_bounds__(64) void k_bk_pairs(Sorted prim, Sorted sec, int nc, double L, double r02,
                                                 int self_set, int64_t p_lo, int64_t p_hi, int64_t c_lo,
                                                 int *__restrict__ pcnt, int *__restrict__ maxcnt,
                                                 const int64_t *__restrict__ poff, int64_t base, BkPairs out) {
  __shared__ int64_t nb_start[27];
  __shared__ int nb_pref[28];
  __shared__ int nb_shift[27];
  const int64_t cell = c_lo + blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t hs = prim.cell_start[cell], he = prim.cell_start[cell + 1];
  const int64_t i0 = hs > p_lo ? hs : p_lo, i1 = he < p_hi ? he : p_hi;
  if (i0 >= i1) return;
  const int cz = int(cell % nc), cy = int((cell / nc) % nc), cx = int(cell / (int64_t(nc) * nc));
  if (lane < 27) {
    int sx, sy, sz;
    const int nx = bk_wrap(cx + lane / 9 - 1, nc, sx), ny = bk_wrap(cy + (lane / 3) % 3 - 1, nc, sy),
              nz = bk_wrap(cz + lane % 3 - 1, nc, sz);
    const int64_t nb = (int64_t(nx) * nc + ny) * nc + nz;
    nb_start[lane] = sec.cell_start[nb];
    nb_pref[lane + 1] = int(sec.cell_start[nb + 1] - sec.cell_start[nb]);
    nb_shift[lane] = (sx + 1) * 9 + (sy + 1) * 3 + (sz + 1);
  }
  __syncthreads();
  if (lane == 0) {
    nb_pref[0] = 0;
    for (int s = 0; s < 27; ++s) nb_pref[s + 1] += nb_pref[s];
  }
  __syncthreads();
  const int total = nb_pref[27];
  for (int64_t i = i0; i < i1; ++i) {
    if (prim.m && !prim.m[i]) {
      if (!WRITE && lane == 0) pcnt[i] = 0;
      continue;
    }
    const double xi = prim.x[i], yi = prim.y[i], zi = prim.z[i];
    int written = 0;
    const int64_t wbase = WRITE ? poff[i] - base : 0;
    for (int q0 = 0; q0 < total; q0 += 64) {
      const int q = q0 + lane;
      bool hit = false;
      double dx = 0.0, dy = 0.0, dz = 0.0, r2 = 0.0;
      int64_t j = 0;
      if (q < total) {
        int lo = 0, hi = 27;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (nb_pref[mid] <= q) lo = mid;
          else hi = mid;
        }
        j = nb_start[lo] + (q - nb_pref[lo]);
        const int sh = nb_shift[lo];
        dx = bk_image(xi - sec.x[j], sh / 9 - 1, L);
        dy = bk_image(yi - sec.y[j], (sh / 3) % 3 - 1, L);
        dz = bk_image(zi - sec.z[j], sh % 3 - 1, L);
        r2 = bk_sq_norm(dx, dy, dz);
        hit = r2 < r02 && !(self_set && lo == 13 && j == i);
      }
      const unsigned long long bal = __ballot(hit);
      if (WRITE && hit) {
        const int pre = __popcll(bal & ((1ull << lane) - 1ull));
        const int64_t k = wbase + written + pre;
        const double r = sqrt(r2);
        const double inv = r > 0.0 ? 1.0 / r : 0.0;
        out.r[k] = r;
        out.ux[k] = r > 0.0 ? dx * inv : 0.0;
        out.uy[k] = r > 0.0 ? dy * inv : 0.0;
        out.uz[k] = r > 0.0 ? dz * inv : 1.0;
        out.wj[k] = sec.w[j];
      }
      written += __popcll(bal);
    }
    if (!WRITE && lane == 0) {
      pcnt[i] = written;
      atomicMax(maxcnt, written);
    }
  }
}

// Real orthonormal spherical harmonics y_lm of a unit vector, index l*l+l+m:
// y_l0 = N_l0 Q_l^0(z), y_lm = N_lm Q_l^m(z) Re (x+iy)^m, y_l-m = N_lm Q_l^m(z) Im (x+iy)^m,
// with Q_l^m = d^m P_l / dz^m by its three-term recurrence.
template <int LM>
__device__ inline void real_ylm(double x, double y, double z, double (&Y)[(LM + 1) * (LM + 1)]) {
  double C[LM + 1], S[LM + 1];
  C[0] = 1.0;
  S[0] = 0.0;
#pragma unroll
  for (int m = 1; m <= LM; ++m) {
    C[m] = C[m - 1] * x - S[m - 1] * y;
    S[m] = S[m - 1] * x + C[m - 1] * y;
  }
  double qmm = 1.0;
#pragma unroll
  for (int m = 0; m <= LM; ++m) {
    if (m > 0) qmm *= double(2 * m - 1);
    double q2 = 0.0, q1 = 0.0;
#pragma unroll
    for (int l = m; l <= LM; ++l) {
      double q;
      if (l == m) q = qmm;
      else if (l == m + 1) q = z * double(2 * m + 1) * qmm;
      else q = (double(2 * l - 1) * z * q1 - double(l + m - 1) * q2) / double(l - m);
      q2 = q1;
      q1 = q;
      const double nq = YLM_NORM[l][m] * q;
      if (m == 0) {
        Y[l * l + l] = nq;
      } else {
        Y[l * l + l + m] = nq * C[m];
        Y[l * l + l - m] = nq * S[m];
      }
    }
  }
}

constexpr int kMaxOwnA = (kMaxNkB * 49 + 63) / 64;              // A outputs per lane
constexpr int kMaxOwnC = (7 * kMaxNkB * (kMaxNkB + 1) / 2 + 63) / 64;  // C / G outputs per lane

template <int NL, bool FP64>
__global__ __launch_bounds__(64) void k_bk_sweep(BkPairs pairs, const int64_t *__restrict__ poff, int64_t base,
                                                 int64_t p_lo, int64_t p_hi, const double *__restrict__ pw,
                                                 double inv_r0, const double *__restrict__ edges,
                                                 const double *__restrict__ bin_coef, int NK, int do_s0,
                                                 double *__restrict__ partial, int rowlen) {
  using T = typename std::conditional<FP64, double, float>::type;
  constexpr int NLM = NL * NL;
  constexpr int BATCH = FP64 ? 32 : 64;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int NG = NL * NK;
  T *gw = reinterpret_cast<T *>(lds_raw);                 // [BATCH][NL*NK]
  T *yv = gw + BATCH * NG;                                // [BATCH][NLM]
  double *Ash = reinterpret_cast<double *>(yv + BATCH * NLM + ((BATCH * NLM) & 1));  // [NK][NLM]
  const int lane = threadIdx.x;
  const int NT = NK * (NK + 1) / 2;
  const int nA = NK * NLM, nC = NL * NT;

  // output ownership: lane owns A entries lane + 64 k, C/G entries lane + 64 k
  int oa_a[kMaxOwnA], oa_lm[kMaxOwnA], oa_l[kMaxOwnA];
#pragma unroll
  for (int k = 0; k < kMaxOwnA; ++k) {
    const int o = lane + 64 * k;
    const int a = o / NLM, lm = o - a * NLM;
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    oa_a[k] = a;
    oa_lm[k] = lm;
    oa_l[k] = l;
  }
  int oc_l[kMaxOwnC], oc_a[kMaxOwnC], oc_b[kMaxOwnC];
#pragma unroll
  for (int k = 0; k < kMaxOwnC; ++k) {
    const int o = lane + 64 * k;
    int l = 0, a = 0, b = 0;
    if (o < nC) {
      l = o / NT;
      int t = o - l * NT;
      while (t >= NK - a) {
        t -= NK - a;
        ++a;
      }
      b = a + t;
    }
    oc_l[k] = l;
    oc_a[k] = a;
    oc_b[k] = b;
  }
  double accC[kMaxOwnC], accG[kMaxOwnC];
#pragma unroll
  for (int k = 0; k < kMaxOwnC; ++k) accC[k] = accG[k] = 0.0;
  double accS0 = 0.0;

  for (int64_t p = p_lo + blockIdx.x; p < p_hi; p += gridDim.x) {
    const int64_t o0 = poff[p] - base, o1 = poff[p + 1] - base;
    if (o0 >= o1) continue;
    const double wp = pw[p];
    double accA[kMaxOwnA];
#pragma unroll
    for (int k = 0; k < kMaxOwnA; ++k) accA[k] = 0.0;
    for (int64_t b0 = o0; b0 < o1; b0 += BATCH) {
      const int nv = int((o1 - b0) < BATCH ? (o1 - b0) : BATCH);
      if (lane < BATCH) {
        T *g_row = gw + lane * NG;
        T *y_row = yv + lane * NLM;
        if (lane < nv) {
          const int64_t k = b0 + lane;
          const double r = pairs.r[k];
          const double wjW = pairs.wj[k] * window<double>(r * inv_r0);
          double Y[NLM];
          real_ylm<NL - 1>(pairs.ux[k], pairs.uy[k], pairs.uz[k], Y);
#pragma unroll
          for (int q = 0; q < NLM; ++q) y_row[q] = T(Y[q]);
          double prev[NL];
          double kprev3 = 0.0;
          for (int e = 0; e <= NK; ++e) {
            const double ke = edges[e], ke3 = ke * ke * ke;
            const double u = ke * r;
            Gv<double, NL> G;
            if constexpr (FP64) G = G_fp64<NL, 1>(u);
            else G = G_mixed<NL, 1>(u);
            if (e > 0) {
              const double cf = wjW * bin_coef[e - 1];
#pragma unroll
              for (int l = 0; l < NL; ++l) g_row[l * NK + e - 1] = T(cf * (ke3 * G.v[l] - kprev3 * prev[l]));
            }
#pragma unroll
            for (int l = 0; l < NL; ++l) prev[l] = G.v[l];
            kprev3 = ke3;
          }
        } else {
          for (int q = 0; q < NG; ++q) g_row[q] = T(0);
          for (int q = 0; q < NLM; ++q) y_row[q] = T(0);
        }
      }
      __syncthreads();
      // A^a_lm += sum_j (w_j g^a_l) y_lm
#pragma unroll
      for (int k = 0; k < kMaxOwnA; ++k) {
        if (lane + 64 * k < nA) {
          const T *gp = gw + oa_l[k] * NK + oa_a[k];
          const T *yp = yv + oa_lm[k];
          double s = 0.0;
          for (int q = 0; q < nv; ++q) s = fma(double(gp[q * NG]), double(yp[q * NLM]), s);
          accA[k] += s;
        }
      }
      // C^ab_l += w_p sum_j (w_j g^a_l)(w_j g^b_l)
#pragma unroll
      for (int k = 0; k < kMaxOwnC; ++k) {
        if (lane + 64 * k < nC) {
          const T *ga = gw + oc_l[k] * NK + oc_a[k];
          const T *gb = gw + oc_l[k] * NK + oc_b[k];
          double s = 0.0;
          for (int q = 0; q < nv; ++q) s = fma(double(ga[q * NG]), double(gb[q * NG]), s);
          accC[k] = fma(wp, s, accC[k]);
        }
      }
      if (do_s0 && lane < NK) {
        const T *g0 = gw + lane;
        double s = 0.0;
        for (int q = 0; q < nv; ++q) s += double(g0[q * NG]);
        accS0 = fma(wp, s, accS0);
      }
      __syncthreads();
    }
    // per-primary contraction G^ab_l += w_p (4 pi/(2l+1)) sum_m A^a_lm A^b_lm
#pragma unroll
    for (int k = 0; k < kMaxOwnA; ++k)
      if (lane + 64 * k < nA) Ash[oa_a[k] * NLM + oa_lm[k]] = accA[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMaxOwnC; ++k) {
      if (lane + 64 * k < nC) {
        const int l = oc_l[k];
        const double *xa = Ash + oc_a[k] * NLM + l * l;
        const double *xb = Ash + oc_b[k] * NLM + l * l;
        double s = 0.0;
        for (int m = 0; m < 2 * l + 1; ++m) s = fma(xa[m], xb[m], s);
        accG[k] = fma(wp * (4.0 * kPi / double(2 * l + 1)), s, accG[k]);
      }
    }
    __syncthreads();
  }
  double *row = partial + int64_t(blockIdx.x) * rowlen;
#pragma unroll
  for (int k = 0; k < kMaxOwnC; ++k) {
    const int o = lane + 64 * k;
    if (o < nC) {
      row[o] += accG[k];
      row[nC + o] += accC[k];
    }
  }
  if (lane < NK) row[2 * nC + lane] += accS0;
}

// --------------------------------------------------------------- launchers
void bk_pairs_count(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
                    int *pcnt, int *maxcnt) {
  const int64_t ncells = g.ncells();
  BkPairs none{};
  k_bk_pairs<false><<<dim3(unsigned(ncells)), dim3(64), 0, c.stream>>>(prim, sec, g.nc, g.L, r0 * r0, self_set ? 1 : 0,
                                                                        0, prim.n, 0, pcnt, maxcnt, nullptr, 0, none);
  HIPSTER_HIP(hipGetLastError());
}

void bk_pairs_write(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
                    int64_t p_lo, int64_t p_hi, int64_t c_lo, int64_t c_hi, const int64_t *poff, int64_t base,
                    BkPairs out) {
  if (c_hi <= c_lo) return;
  k_bk_pairs<true><<<dim3(unsigned(c_hi - c_lo)), dim3(64), 0, c.stream>>>(
      prim, sec, g.nc, g.L, r0 * r0, self_set ? 1 : 0, p_lo, p_hi, c_lo, nullptr, nullptr, poff, base, out);
  HIPSTER_HIP(hipGetLastError());
}

size_t bk_sweep_lds(int NL, int NK, bool fp64) {
  const int batch = fp64 ? 32 : 64;
  const size_t tsz = fp64 ? 8 : 4;
  const size_t nlm = size_t(NL) * NL;
  size_t bytes = size_t(batch) * (size_t(NL) * NK + nlm) * tsz;
  bytes += (batch * nlm & 1) ? tsz : 0;
  bytes = (bytes + 15) / 16 * 16;
  return bytes + size_t(NK) * nlm * 8;
}

template <int NL>
static void launch_bk(Ctx &c, const BkPairs &p, const int64_t *poff, int64_t base, int64_t p_lo, int64_t p_hi,
                      const double *pw, double inv_r0, const double *edges, const double *coef, int NK, int do_s0,
                      bool fp64, double *partial, int rowlen, int nwaves) {
  const size_t lds = bk_sweep_lds(NL, NK, fp64);
  if (fp64) {
    HIPSTER_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bk_sweep<NL, true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    k_bk_sweep<NL, true><<<dim3(unsigned(nwaves)), dim3(64), lds, c.stream>>>(
        p, poff, base, p_lo, p_hi, pw, inv_r0, edges, coef, NK, do_s0, partial, rowlen);
  } else {
    HIPSTER_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bk_sweep<NL, false>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    k_bk_sweep<NL, false><<<dim3(unsigned(nwaves)), dim3(64), lds, c.stream>>>(
        p, poff, base, p_lo, p_hi, pw, inv_r0, edges, coef, NK, do_s0, partial, rowlen);
  }
  HIPSTER_HIP(hipGetLastError());
}

void bk_sweep(Ctx &c, const BkPairs &p, const int64_t *poff, int64_t base, int64_t p_lo, int64_t p_hi,
              const double *pw, double r0, const double *edges, const double *coef, int NK, int ell_max, bool s0,
              bool fp64, double *partial, int rowlen, int nwaves) {
  const double inv = 1.0 / r0;
  switch (ell_max) {
    case 0: launch_bk<1>(c, p, poff, base, p_lo, p_hi, pw, inv, edges, coef, NK, s0, fp64, partial, rowlen, nwaves); break;
    case 1: launch_bk<2>(c, p, poff, base, p_lo, p_hi, pw, inv, edges, coef, NK, s0, fp64, partial, rowlen, nwaves); break;
    case 2: launch_bk<3>(c, p, poff, base, p_lo, p_hi, pw, inv, edges, coef, NK, s0, fp64, partial, rowlen, nwaves); break;
    case 3: launch_bk<4>(c, p, poff, base, p_lo, p_hi, pw, inv, edges, coef, NK, s0, fp64, partial, rowlen, nwaves); break;
    case 4: launch_bk<5>(c, p, poff, base, p_lo, p_hi, pw, inv, edges, coef, NK, s0, fp64, partial, rowlen, nwaves); break;
    case 5: launch_bk<6>(c, p, poff, base, p_lo, p_hi, pw, inv, edges, coef, NK, s0, fp64, partial, rowlen, nwaves); break;
    default: launch_bk<7>(c, p, poff, base, p_lo, p_hi, pw, inv, edges, coef, NK, s0, fp64, partial, rowlen, nwaves); break;
  }
}

// Chunk boundaries over primaries: chunk q starts at the first primary whose
// offset reaches q * cap; also returns the home cells spanned.
__global__ void k_chunk_bounds(const int64_t *__restrict__ poff, int64_t np, int64_t cap, int nchunks,
                               const int *__restrict__ scell, int64_t *__restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q > nchunks) return;
  int64_t p;
  if (q == nchunks) {
    p = np;
  } else {
    const int64_t target = int64_t(q) * cap;
    int64_t lo = 0, hi = np;  // first p in [0, np] with poff[p] >= target
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (poff[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    p = lo;
  }
  out[3 * q] = p;
  out[3 * q + 1] = p < np ? scell[p] : 0;
  out[3 * q + 2] = poff[p];
}

void chunk_bounds(Ctx &c, const int64_t *poff, int64_t np, int64_t cap, int nchunks, const int *scell,
                  int64_t *out_dev) {
  k_chunk_bounds<<<dim3(unsigned((nchunks + 1 + 63) / 64)), dim3(64), 0, c.stream>>>(poff, np, cap, nchunks, scell,
                                                                                     out_dev);
  HIPSTER_HIP(hipGetLastError());
}

}  // namespace hipster
