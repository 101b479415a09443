// Bispectrum path (Sec. 4): per-primary spherical-harmonic coefficients
//   A^a_lm(x_p) = sum_j w_j jbar^a_l(r_pj) W(r_pj/R0) y_lm(xhat_pj)      (eq. AC-def)
//   C^ab_l(x_p) = sum_j w_j^2 jbar^a_l jbar^b_l W^2
// for data primaries (j != p) and random primaries (all data j), contracted
// per primary into G^ab_l += w_p (4 pi/(2l+1)) sum_m A^a_lm A^b_lm, with
// real orthonormal harmonics y_lm (the sum over m is basis independent).
// Data primaries also give S0^b = sum_{p != j} w_p w_j jbar^b_0 W, the pair sum
// of the analytic DDR^I term.
//
// One fused kernel per primary catalogue: each wave takes primaries in turn,
// enumerates the data neighbours of each inside R0 from the 27 surrounding
// cells, and contracts them on the FP64 matrix cores (see k_bk_fused).  The
// candidate order is fixed, so every sum is deterministic.
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

// Real orthonormal spherical harmonics y_lm of a unit vector, index l*l+l+m:
// y_l0 = N_l0 Q_l^0(z), y_lm = N_lm Q_l^m(z) Re (x+iy)^m, y_l-m = N_lm Q_l^m(z) Im (x+iy)^m,
// with Q_l^m = d^m P_l / dz^m by its three-term recurrence.
template <int LM, typename Out>
__device__ inline void real_ylm(double x, double y, double z, Out Y) {
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

// ------------------------------------------------- fused enumerate + MFMA
// One wave per workgroup; waves take primaries p = p_lo + block, + grid, ...
// For each primary the wave scans the 27 neighbour cells 64 candidates at a
// time and appends the pairs inside R0 to an LDS hit buffer.  Every 64 hits
// form a batch, contracted on the FP64 matrix cores with
// v_mfma_f64_16x16x4f64 in 16 steps of 4 pairs:
//   A_l[a][m] += g_l[q][a] y_lm[q]            (A operand: bins x pairs)
//   C_l[a][b] += w_p g_l[q][a] g_l[q][b]      (both operands the same register)
// where g_l[q][a] = w_q W(r_q) jbar^a_l(r_q).  In step s lane L holds pair
// q = 4s + L/16 and bin a = L%16, the operand layout of the instruction, so
// each lane evaluates G_l at one bin edge and takes the next edge's value from
// lane L+1.  After the primary's last batch, G_l += w_p (4 pi/(2l+1)) A_l A_l^T
// through an LDS transpose of the A tile.  Operand layout (gfx950): A lane L
// -> A[L%16][L/16]; B lane L -> B[L/16][L%16]; result lane L, register v ->
// D[L/16 + 4v][L%16].
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ inline d4_t mfma_f64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kHitCap = 128;

// Minimum waves per SIMD the compiler must fit the fused kernel into (1 lets
// it use all 512 registers; 2 trades a few spills for twice the occupancy).
#ifndef HIPSTER_BK_WAVES_PER_EU
#define HIPSTER_BK_WAVES_PER_EU 1
#endif

size_t bk_fused_lds(int NL) {
  // y_lm staging [64][NL^2] and the A tile [NL][16][16] share the allocation
  const size_t a = size_t(64) * NL * NL, b = size_t(256) * NL;
  return (a > b ? a : b) * 8;
}

template <int NL, bool FP64>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(HIPSTER_BK_WAVES_PER_EU))) void k_bk_fused(Sorted prim, Sorted sec, int nc, double L, double r02, int self_set,
                                                 int64_t p_lo, int64_t p_hi, double inv_r0,
                                                 const double *__restrict__ edges, const double *__restrict__ coef,
                                                 int NK, double *__restrict__ partial, int rowlen,
                                                 unsigned long long *__restrict__ npairs) {
  constexpr int NLM = NL * NL;
  extern __shared__ __align__(16) double ylds[];  // [64][NLM]; reused as the A tile [NL][16][16]
  __shared__ double hb_r[kHitCap], hb_x[kHitCap], hb_y[kHitCap], hb_z[kHitCap], hb_w[kHitCap];
  __shared__ int64_t nb_start[27];
  __shared__ int nb_pref[28];
  __shared__ int nb_shift[27];
  const int lane = threadIdx.x, t4 = lane >> 4, col = lane & 15;
  // per-lane bin-edge constants: this lane evaluates edge `col`, bin `col`
  const bool has_edge = col <= NK;
  const double ke = edges[col <= NK ? col : NK];
  const double ke3 = ke * ke * ke;
  const bool has_bin = col < NK;
  const double kn = edges[col + 1 <= NK ? col + 1 : NK];
  const double kn3 = kn * kn * kn;
  const double cfb = has_bin ? coef[col] : 0.0;
  const bool extra_edge = (col == 15) && (NK == 16);  // the 17th edge
  d4_t accC[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) accC[l] = d4_t{0.0, 0.0, 0.0, 0.0};
  // the Gram sums live in this wave's own row of `partial` (zeroed by the
  // host), updated once per primary, to keep registers for the batch work
  double *row = partial + int64_t(blockIdx.x) * rowlen;
  double accS0 = 0.0;
  unsigned long long pcount = 0;
  int64_t cur_cell = -1;

  for (int64_t p = p_lo + blockIdx.x; p < p_hi; p += gridDim.x) {
    if (prim.m && !prim.m[p]) continue;
    const int64_t cell = prim.scell[p];
    if (cell != cur_cell) {
      __syncthreads();
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
        for (int q = 0; q < 27; ++q) nb_pref[q + 1] += nb_pref[q];
      }
      __syncthreads();
      cur_cell = cell;
    }
    const int total = nb_pref[27];
    const double xi = prim.x[p], yi = prim.y[p], zi = prim.z[p], wp = prim.w[p];
    d4_t accA[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) accA[l] = d4_t{0.0, 0.0, 0.0, 0.0};
    int nh = 0;

    auto batch = [&](int nv) {
      // y_lm of the lane's own pair into LDS (zeros past the batch)
      if (lane < nv) {
        real_ylm<NL - 1>(hb_x[lane], hb_y[lane], hb_z[lane], ylds + lane * NLM);
      } else {
#pragma unroll
        for (int q = 0; q < NLM; ++q) ylds[lane * NLM + q] = 0.0;
      }
      __syncthreads();
      for (int s = 0; s < 16 && 4 * s < nv; ++s) {
        const int q = 4 * s + t4;
        const bool valid = q < nv;
        const double rq = valid ? hb_r[q] : 0.0;
        const double wq = valid ? hb_w[q] : 0.0;
        Gv<double, NL> Ge;
        if (has_edge) {
          if constexpr (FP64) Ge = G_fp64<NL, 1>(ke * rq);
          else Ge = G_mixed<NL, 1>(ke * rq);
        } else {
#pragma unroll
          for (int l = 0; l < NL; ++l) Ge.v[l] = 0.0;
        }
        Gv<double, NL> Gn;
#pragma unroll
        for (int l = 0; l < NL; ++l) Gn.v[l] = __shfl(Ge.v[l], (lane & 48) | ((col + 1) & 15));
        if (extra_edge) {
          if constexpr (FP64) Gn = G_fp64<NL, 1>(kn * rq);
          else Gn = G_mixed<NL, 1>(kn * rq);
        }
        const double f = (valid && has_bin) ? wq * window<double>(rq * inv_r0) * cfb : 0.0;
        double g[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) g[l] = f * (kn3 * Gn.v[l] - ke3 * Ge.v[l]);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const double y = (col < 2 * l + 1) ? ylds[q * NLM + l * l + col] : 0.0;
          accA[l] = mfma_f64(g[l], y, accA[l]);
          accC[l] = mfma_f64(g[l] * wp, g[l], accC[l]);
        }
        accS0 = fma(wp, g[0], accS0);
      }
      __syncthreads();
    };

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
        hit = r2 < r02 && !(self_set && lo == 13 && j == p);
      }
      const unsigned long long bal = __ballot(hit);
      if (hit) {
        const int k = nh + __popcll(bal & ((1ull << lane) - 1ull));
        const double r = sqrt(r2);
        const double inv = r > 0.0 ? 1.0 / r : 0.0;
        hb_r[k] = r;
        hb_x[k] = r > 0.0 ? dx * inv : 0.0;
        hb_y[k] = r > 0.0 ? dy * inv : 0.0;
        hb_z[k] = r > 0.0 ? dz * inv : 1.0;
        hb_w[k] = sec.w[j];
      }
      const int added = __popcll(bal);
      nh += added;
      pcount += unsigned(added);
      if (nh >= 64) {
        __syncthreads();
        batch(64);
        // keep the overflow: entries [64, nh) move to the front
        const int rest = nh - 64;
        double vr = 0, vx = 0, vy = 0, vz = 0, vw = 0;
        if (lane < rest) {
          vr = hb_r[64 + lane];
          vx = hb_x[64 + lane];
          vy = hb_y[64 + lane];
          vz = hb_z[64 + lane];
          vw = hb_w[64 + lane];
        }
        __syncthreads();
        if (lane < rest) {
          hb_r[lane] = vr;
          hb_x[lane] = vx;
          hb_y[lane] = vy;
          hb_z[lane] = vz;
          hb_w[lane] = vw;
        }
        nh = rest;
      }
    }
    if (nh > 0) {
      __syncthreads();
      batch(nh);
    }
    // G_l += w_p (4 pi/(2l+1)) A_l A_l^T through an LDS transpose of A
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) ylds[l * 256 + (t4 + 4 * v) * 16 + col] = accA[l][v];
    __syncthreads();
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const double sc = wp * (4.0 * kPi / double(2 * l + 1));
      d4_t g4;
#pragma unroll
      for (int v = 0; v < 4; ++v) g4[v] = row[l * 256 + (t4 + 4 * v) * 16 + col];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const double x = ylds[l * 256 + col * 16 + 4 * s2 + t4];
        g4 = mfma_f64(x * sc, x, g4);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) row[l * 256 + (t4 + 4 * v) * 16 + col] = g4[v];
    }
    __syncthreads();
  }
  // per-wave partial row: [G tiles NL*256 (already there) | C tiles NL*256 | S0 16]
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = (t4 + 4 * v) * 16 + col;
      row[NL * 256 + l * 256 + e] += accC[l][v];
    }
  double s0 = accS0;
  s0 += __shfl_xor(s0, 16);
  s0 += __shfl_xor(s0, 32);
  if (lane < 16) row[2 * NL * 256 + lane] += s0;
  if (lane == 0 && pcount) atomicAdd(npairs, pcount);
}

template <int NL>
static void launch_fused(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
                         const double *edges, const double *coef, int NK, bool fp64, double *partial, int rowlen,
                         int nwaves, unsigned long long *npairs) {
  const size_t lds = bk_fused_lds(NL);
  if (prim.n == 0) return;
  if (fp64)
    k_bk_fused<NL, true><<<dim3(unsigned(nwaves)), dim3(64), lds, c.stream>>>(
        prim, sec, g.nc, g.L, r0 * r0, self_set ? 1 : 0, 0, prim.n, 1.0 / r0, edges, coef, NK, partial, rowlen, npairs);
  else
    k_bk_fused<NL, false><<<dim3(unsigned(nwaves)), dim3(64), lds, c.stream>>>(
        prim, sec, g.nc, g.L, r0 * r0, self_set ? 1 : 0, 0, prim.n, 1.0 / r0, edges, coef, NK, partial, rowlen, npairs);
  HIPSTER_HIP(hipGetLastError());
}

void bk_fused(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
              const double *edges, const double *coef, int NK, int ell_max, bool fp64, double *partial, int rowlen,
              int nwaves, unsigned long long *npairs) {
  switch (ell_max) {
    case 0: launch_fused<1>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, partial, rowlen, nwaves, npairs); break;
    case 1: launch_fused<2>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, partial, rowlen, nwaves, npairs); break;
    case 2: launch_fused<3>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, partial, rowlen, nwaves, npairs); break;
    case 3: launch_fused<4>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, partial, rowlen, nwaves, npairs); break;
    case 4: launch_fused<5>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, partial, rowlen, nwaves, npairs); break;
    case 5: launch_fused<6>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, partial, rowlen, nwaves, npairs); break;
    default: launch_fused<7>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, partial, rowlen, nwaves, npairs); break;
  }
}

}  // namespace hipster
