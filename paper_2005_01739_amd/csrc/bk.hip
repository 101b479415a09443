// Bispectrum path (Sec. 4): per-primary spherical-harmonic coefficients
//   A^a_lm(x_p) = sum_j w_j jbar^a_l(r_pj) W(r_pj/R0) y_lm(xhat_pj)      (eq. AC-def)
//   C^ab_l(x_p) = sum_j w_j^2 jbar^a_l jbar^b_l W^2
// for data primaries (j != p) and random primaries (all data j), contracted
// per primary into G^ab_l += w_p (4 pi/(2l+1)) sum_m A^a_lm A^b_lm, with
// real orthonormal harmonics y_lm (the sum over m is basis independent).
// Data primaries also give S0^b = sum_{p != j} w_p w_j jbar^b_0 W, the pair sum
// of the analytic DDR^I term.
//
// One fused kernel per primary catalogue: each wave takes runs of primaries,
// enumerates the data neighbours of each inside R0 from the 27 surrounding
// cells, and contracts them on the FP64 matrix cores (see k_bk_fused).  The
// candidate order and the primary-to-wave assignment are fixed, so every sum
// is deterministic.
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
      else q = (double(2 * l - 1) * z * q1 - double(l + m - 1) * q2) * (1.0 / double(l - m));
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
// One wave per workgroup.  Each wave takes runs of kPrimRun consecutive
// primaries (cell order) from its XCD's slab (see the loop below);
// consecutive primaries mostly share a home cell, whose 27 neighbour cells are
// merged into at most 27 contiguous runs of the sorted secondaries (cells
// adjacent along z are adjacent in memory).  The runs are scanned 64
// candidates at a time, the loads of the next 64 issued before the current
// ones are tested; pairs inside R0 go to an LDS hit buffer, and every kBatch
// hits form a batch: y_lm of each pair into LDS, then kBatch/4 steps of 4
// pairs contracted on v_mfma_f64_16x16x4f64:
//   A_l[a][m] += sum_q g_l[q][a] y_lm[q]            (l >= 1; A operand: bins x pairs)
//   C_l[a][b] += w_p sum_q g_l[q][a] g_l[q][b]      (both operands the same register)
// where g_l[q][a] = w_q W(r_q) jbar^a_l(r_q).  In step s lane L holds pair
// q = 4s + L/16 and bin a = L%16, the operand layout of the instruction, so
// each lane evaluates G_l at one bin edge and takes the next edge's value
// from lane L+1 (the 17th edge of a 16-bin set is evaluated per pair with the
// harmonics).  A_00 has a single column, so its sum Sigma_q g_0 is kept on
// the vector unit; it also gives S0 and the l = 0 Gram directly.  (FP64
// matrix and vector instructions do not execute concurrently on this chip --
// the co-execution counter reads zero -- so nothing is gained by
// interleaving them.)
//
// After a primary's last batch, G_l += w_p (4 pi/(2l+1)) A_l A_l^T through an
// LDS transpose of the A tile.  G, C and S0 stay in registers until the wave
// ends.  Operand layout (gfx950): A lane L -> A[L%16][L/16]; B lane L ->
// B[L/16][L%16]; result lane L, register v -> D[L/16 + 4v][L%16].
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ inline d4_t mfma_f64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kBatch = 64;           // pairs per contraction batch
constexpr int kHitCap = kBatch + 64; // < kBatch left over + at most 64 hits per scan step
constexpr int kPrimRun = 16;         // consecutive primaries per wave assignment
constexpr int kXcds = 8;             // accelerator complex dies of the MI355X (the grid is a multiple)

// Minimum waves per SIMD the compiler must fit the fused kernel into (1 lets
// it use all 512 registers; 2 trades spills for twice the occupancy).
#ifndef HIPSTER_BK_WAVES_PER_EU
#define HIPSTER_BK_WAVES_PER_EU 1
#endif
// Occupancy hint of the variant without the C sums (fewer accumulators).
#ifndef HIPSTER_BK_WAVES_PER_EU_NOC
#define HIPSTER_BK_WAVES_PER_EU_NOC 1
#endif

// The value held by lane L+1 of the same 16-lane row (lane 15 of a row gets
// 0): a DPP row shift, no LDS round trip.
__device__ inline double from_next_lane_in_row(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int nlo = __builtin_amdgcn_update_dpp(0, lo, 0x101, 0xf, 0xf, false);  // row_shl:1
  const int nhi = __builtin_amdgcn_update_dpp(0, hi, 0x101, 0xf, 0xf, false);
  return __hiloint2double(nhi, nlo);
}

// y_lm staging of one lane's pair: element idx of pair q at ylds[idx][q],
// rows padded to kBatch + 1 doubles so that lanes write distinct banks.
struct YRow {
  double *base;
  __device__ double &operator[](int idx) const { return base[idx * (64 + 1)]; }
};

__device__ inline int64_t uniform_i64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v))));
  const int hi = __builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v) >> 32)));
  return int64_t((uint64_t(uint32_t(hi)) << 32) | uint64_t(uint32_t(lo)));
}

constexpr int kSinCosTabBk = 64;      // sine/cosine table entries (LDS)
constexpr int kYStride = kBatch + 1;  // row stride of the y_lm staging
static_assert(kYStride == 64 + 1, "YRow assumes kBatch = 64");

size_t bk_fused_lds(int NL, int NK) {
  // y_lm [NL^2][kYStride], one row of zeros, then a region that holds the
  // top-edge values [NL][kBatch] (16 bins) during batches and the A tile
  // [NL][16][16] after them
  (void)NK;
  return (size_t(kYStride) * (NL * NL + 1) + size_t(256) * NL) * 8;
}

// G_l(u) of the mixed form for the closed-form lanes, with lanes below
// kUSmall replaced by the Taylor branch (a uniform branch, taken only when
// some lane needs it).
// WITH_C = false leaves the C sums out (their partial-row entries stay zero):
// the mixed form takes C from the pair histogram of the C-term sweep instead
// (k_ddr2_hist), which saves the NL matrix instructions per step that C costs
// here.
template <int NL, bool FP64, bool WITH_C>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WITH_C ? HIPSTER_BK_WAVES_PER_EU
                                                                             : HIPSTER_BK_WAVES_PER_EU_NOC))) void
k_bk_fused(
    Sorted prim, Sorted sec, int nc, double L, double r02, int self_set, int64_t p_lo, int64_t p_hi,
    double inv_r0, const double *__restrict__ edges, const double *__restrict__ coef, int NK,
    double *__restrict__ partial, int rowlen, unsigned long long *__restrict__ npairs) {
  constexpr int NLM = NL * NL;
  extern __shared__ __align__(16) double lds[];
  double *ylds = lds;                          // [NLM + 1][kYStride], row NLM all zeros
  double *gtop = lds + kYStride * (NLM + 1);   // [NL][kBatch]: k_NK^3 G_l(k_NK r_q), 16 bins
  double *atile = gtop;                        // [NL][16][16] between primaries
  // hit buffer; slot kHitCap is a neutral pair (weight 0) read by lanes
  // past the end of a batch, so that no operand load needs a condition
  __shared__ double hb_r[kHitCap + 1], hb_ir[kHitCap + 1], hb_f[kHitCap + 1], hb_x[kHitCap], hb_y[kHitCap],
      hb_z[kHitCap];
  __shared__ int64_t nb_beg[27], nb_end[27], run_beg[27], run_end[27];
  // sine/cosine table for the mixed form's closed branch (64 entries: the
  // LDS of four one-wave workgroups per CU has room for 1 KB more)
  __shared__ double2 sc_tab[FP64 ? 1 : kSinCosTabBk];
  if constexpr (!FP64) {
    stage_sincos_tab<kSinCosTabBk>(sc_tab);
    __syncthreads();
  }
  __shared__ int nb_sh[27], run_sh[27], n_runs_s;
  const int lane = threadIdx.x, t4 = lane >> 4, col = lane & 15;
  // per-lane edge constants: this lane evaluates edge `col`, bin `col`
  const bool has_bin = col < NK;
  const double ke = edges[col <= NK ? col : NK];
  const double ke3 = ke * ke * ke;
  const double ike = ke > 0.0 ? 1.0 / ke : 0.0;
  const double kn = edges[col + 1 <= NK ? col + 1 : NK];
  const double kn3 = kn * kn * kn;
  const double cfb = has_bin ? coef[col] : 0.0;
  const bool top16 = NK == kMaxNkB;             // the 17th edge is evaluated per pair
  const bool top_lane = top16 && col == kMaxNkB - 1;
  const double ktop = edges[NK], ktop3 = ktop * ktop * ktop, iktop = ktop > 0.0 ? 1.0 / ktop : 0.0;
  const int src = (lane & 48) | ((col + 1) & 15);
  constexpr double kY00 = 0.28209479177387814347;  // y_00 = 1/(2 sqrt(pi))

  d4_t accA[NL], accC[NL], accG[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    accC[l] = d4_t{0.0, 0.0, 0.0, 0.0};
    accG[l] = d4_t{0.0, 0.0, 0.0, 0.0};
  }
  double accS0 = 0.0;
  unsigned long long pcount = 0;
  int64_t cur_cell = -1;
  if (lane == 0) {
    hb_r[kHitCap] = 0.5 / inv_r0;
    hb_ir[kHitCap] = 2.0 * inv_r0;
    hb_f[kHitCap] = 0.0;
  }
  ylds[NLM * kYStride + lane] = 0.0;

  // XCD-aware assignment: workgroups are dealt to the 8 XCDs round-robin, so
  // the waves of XCD x (blockIdx % 8 == x) share one contiguous eighth of the
  // primaries (a slab of cells), whose neighbour data then stays in that
  // XCD's L2.  Within the slab, runs of kPrimRun go round-robin to its waves.
  const int xcd = int(blockIdx.x % kXcds), wx = int(blockIdx.x / kXcds), nwx = int(gridDim.x / kXcds);
  const int64_t np = p_hi - p_lo;
  const int64_t s_lo = p_lo + np * xcd / kXcds, s_hi = p_lo + np * (xcd + 1) / kXcds;
  for (int64_t c0 = s_lo + int64_t(wx) * kPrimRun; c0 < s_hi; c0 += int64_t(nwx) * kPrimRun) {
    const int64_t c1 = c0 + kPrimRun < s_hi ? c0 + kPrimRun : s_hi;
    for (int64_t p = c0; p < c1; ++p) {
      if (prim.m && !prim.m[p]) continue;
      const int64_t cell = prim.scell[p];
      if (cell != cur_cell) {
        // neighbour cells in (dx, dy, dz) order, then merged into runs
        const int cz = int(cell % nc), cy = int((cell / nc) % nc), cx = int(cell / (int64_t(nc) * nc));
        __syncthreads();
        if (lane < 27) {
          int sx, sy, sz;
          const int nx = bk_wrap(cx + lane / 9 - 1, nc, sx), ny = bk_wrap(cy + (lane / 3) % 3 - 1, nc, sy),
                    nz = bk_wrap(cz + lane % 3 - 1, nc, sz);
          const int64_t nb = (int64_t(nx) * nc + ny) * nc + nz;
          nb_beg[lane] = sec.cell_start[nb];
          nb_end[lane] = sec.cell_start[nb + 1];
          nb_sh[lane] = (sx + 1) * 9 + (sy + 1) * 3 + (sz + 1);
        }
        __syncthreads();
        if (lane == 0) {
          int nr = 0;
          for (int k = 0; k < 27; ++k) {
            if (nb_end[k] == nb_beg[k]) continue;
            if (nr > 0 && run_end[nr - 1] == nb_beg[k] && run_sh[nr - 1] == nb_sh[k]) {
              run_end[nr - 1] = nb_end[k];
            } else {
              run_beg[nr] = nb_beg[k];
              run_end[nr] = nb_end[k];
              run_sh[nr] = nb_sh[k];
              ++nr;
            }
          }
          n_runs_s = nr;
        }
        __syncthreads();
        cur_cell = cell;
      }
      const int n_runs = __builtin_amdgcn_readfirstlane(n_runs_s);
      const double xi = prim.x[p], yi = prim.y[p], zi = prim.z[p], wp = prim.w[p];
#pragma unroll
      for (int l = 0; l < NL; ++l) accA[l] = d4_t{0.0, 0.0, 0.0, 0.0};
      double a0 = 0.0;  // sum over this lane's pairs of g_0 for bin col
      int nh = 0;

      auto batch = [&](int nv) {
        // y_lm of pair `lane` (zeros past the batch), and for 16 bins the
        // value at the top edge
        if (lane < nv) {
          real_ylm<NL - 1>(hb_x[lane], hb_y[lane], hb_z[lane], YRow{ylds + lane});
        } else {
#pragma unroll
          for (int k = 0; k < NLM; ++k) ylds[k * kYStride + lane] = 0.0;
        }
        if (top16) {
          const bool v = lane < nv;
          const double rq = v ? hb_r[lane] : 0.0, irq = v ? hb_ir[lane] : 0.0;
          Gv<double, NL> T;
          if constexpr (FP64) T = G_fp64<NL, 1>(ktop * rq);
          else T = G_mixed_w<NL, 1, kSinCosTabBk>(ktop * rq, iktop * irq, sc_tab);
#pragma unroll
          for (int l = 0; l < NL; ++l) gtop[l * kBatch + lane] = ktop3 * T.v[l];
        }
        __syncthreads();
        // 4 pairs per step: lane (col, t4) evaluates G_l at edge col for pair
        // q = 4s + t4, takes edge col+1 from the next lane, and feeds bin col
        // of pair q to the matrix instructions.  Lanes past the batch read the
        // neutral slot, and columns outside an l block read the zero row, so
        // every load is unconditional.
        const int nsteps = (nv + 3) >> 2;
        for (int s = 0; s < nsteps; ++s) {
          const int q = 4 * s + t4;
          const int qe = q < nv ? q : kHitCap;
          const double rq = hb_r[qe], irq = hb_ir[qe];
          const double fb = hb_f[qe] * cfb;
          Gv<double, NL> Ge;
          if constexpr (FP64) Ge = G_fp64<NL, 1>(ke * rq);
          else Ge = G_mixed_w<NL, 1, kSinCosTabBk>(ke * rq, ike * irq, sc_tab);
#pragma unroll
          for (int l = 0; l < NL; ++l) {
            const double gn = from_next_lane_in_row(Ge.v[l]);
            const double hi = top_lane ? gtop[l * kBatch + q] : kn3 * gn;
            const double g = fb * (hi - ke3 * Ge.v[l]);
            if (l == 0) {
              a0 += g;
            } else {
              const int row = col < 2 * l + 1 ? l * l + col : NLM;
              const double y = ylds[row * kYStride + q];
              accA[l] = mfma_f64(g, y, accA[l]);
            }
            if constexpr (WITH_C) accC[l] = mfma_f64(g * wp, g, accC[l]);
          }
        }
        __syncthreads();
      };

      // scan: runs of candidates, 64 at a time, the next step's loads in flight
      int ri = 0;
      int64_t pos = n_runs > 0 ? uniform_i64(run_beg[0]) : 0;
      bool have = n_runs > 0;
      double cx = 0.0, cy = 0.0, cz = 0.0, cw = 0.0;
      int64_t cj = 0;
      bool cok = false;
      int csh = 13;
      auto fetch = [&](double &x, double &y, double &z, double &w, int64_t &j, bool &ok, int &sh) {
        const int64_t end = uniform_i64(run_end[ri]);
        sh = __builtin_amdgcn_readfirstlane(run_sh[ri]);
        j = pos + lane;
        ok = j < end;
        if (ok) {
          x = sec.x[j];
          y = sec.y[j];
          z = sec.z[j];
          w = sec.w[j];
        }
        pos += 64;
        if (pos >= end) {
          ++ri;
          if (ri < n_runs) pos = uniform_i64(run_beg[ri]);
        }
      };
      if (have) fetch(cx, cy, cz, cw, cj, cok, csh);
      while (have) {
        const bool have_next = ri < n_runs;
        double nx = 0.0, ny = 0.0, nz = 0.0, nw = 0.0;
        int64_t nj = 0;
        bool nok = false;
        int nsh = 13;
        if (have_next) fetch(nx, ny, nz, nw, nj, nok, nsh);
        bool hit = false;
        double dx = 0.0, dy = 0.0, dz = 0.0, r2 = 0.0;
        if (cok) {
          dx = bk_image(xi - cx, csh / 9 - 1, L);
          dy = bk_image(yi - cy, (csh / 3) % 3 - 1, L);
          dz = bk_image(zi - cz, csh % 3 - 1, L);
          r2 = bk_sq_norm(dx, dy, dz);
          hit = r2 < r02 && !(self_set && csh == 13 && cj == p);
        }
        const unsigned long long bal = __ballot(hit);
        if (hit) {
          const int k = nh + __popcll(bal & ((1ull << lane) - 1ull));
          const double r = sqrt(r2);
          const double inv = r > 0.0 ? 1.0 / r : 0.0;
          hb_r[k] = r;
          hb_ir[k] = inv;
          hb_f[k] = cw * window<double>(r * inv_r0);
          hb_x[k] = r > 0.0 ? dx * inv : 0.0;
          hb_y[k] = r > 0.0 ? dy * inv : 0.0;
          hb_z[k] = r > 0.0 ? dz * inv : 1.0;
        }
        const int added = __popcll(bal);
        nh += added;
        pcount += unsigned(added);
        // a step can leave up to kBatch - 1 + 64 hits: run batches until
        // fewer than kBatch remain, so the next step fits in the buffer
        while (nh >= kBatch) {
          __syncthreads();
          batch(kBatch);
          // keep the overflow: entries [kBatch, nh) move to the front
          const int rest = nh - kBatch;
          double vr = 0, vi = 0, vf = 0, vx = 0, vy = 0, vz = 0;
          if (lane < rest) {
            vr = hb_r[kBatch + lane];
            vi = hb_ir[kBatch + lane];
            vf = hb_f[kBatch + lane];
            vx = hb_x[kBatch + lane];
            vy = hb_y[kBatch + lane];
            vz = hb_z[kBatch + lane];
          }
          __syncthreads();
          if (lane < rest) {
            hb_r[lane] = vr;
            hb_ir[lane] = vi;
            hb_f[lane] = vf;
            hb_x[lane] = vx;
            hb_y[lane] = vy;
            hb_z[lane] = vz;
          }
          nh = rest;
        }
        cx = nx;
        cy = ny;
        cz = nz;
        cw = nw;
        cj = nj;
        cok = nok;
        csh = nsh;
        have = have_next;
      }
      if (nh > 0) {
        __syncthreads();
        batch(nh);
      }
      // l = 0: A_00[a] = y_00 S_a with S_a = sum_q g_0[q][a]; the Gram term
      // w_p 4 pi y_00^2 S_a S_b = w_p S_a S_b and the S0 sum w_p S_b follow
      double sa = a0;
      sa += __shfl_xor(sa, 16);
      sa += __shfl_xor(sa, 32);
      accS0 = fma(wp, sa, accS0);
      const double wsa = wp * sa;
#pragma unroll
      for (int v = 0; v < 4; ++v) accG[0][v] = fma(__shfl(sa, t4 + 4 * v), wsa, accG[0][v]);
      // l >= 1: G_l += w_p (4 pi/(2l+1)) A_l A_l^T through an LDS transpose of A
      if constexpr (NL > 1) {
#pragma unroll
        for (int l = 1; l < NL; ++l)
#pragma unroll
          for (int v = 0; v < 4; ++v) atile[l * 256 + (t4 + 4 * v) * 16 + col] = accA[l][v];
        __syncthreads();
#pragma unroll
        for (int l = 1; l < NL; ++l) {
          const double sc = wp * (4.0 * kPi / double(2 * l + 1));
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) {
            const double x = atile[l * 256 + col * 16 + 4 * s2 + t4];
            accG[l] = mfma_f64(x * sc, x, accG[l]);
          }
        }
        __syncthreads();
      }
    }
  }
  (void)kY00;
  // per-wave partial row: [G tiles NL*256 | C tiles NL*256 | S0 16], zeroed by the host
  double *row = partial + int64_t(blockIdx.x) * rowlen;
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = (t4 + 4 * v) * 16 + col;
      row[l * 256 + e] += accG[l][v];
      if constexpr (WITH_C) row[NL * 256 + l * 256 + e] += accC[l][v];
    }
  if (t4 == 0) row[2 * NL * 256 + col] += accS0;
  if (lane == 0 && pcount) atomicAdd(npairs, pcount);
}

template <int NL>
static void launch_fused(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
                         const double *edges, const double *coef, int NK, bool fp64, bool with_c, double *partial,
                         int rowlen, int nwaves, unsigned long long *npairs) {
  const size_t lds = bk_fused_lds(NL, NK);
  if (prim.n == 0) return;
  if (NK < 1 || NK > kMaxNkB) throw Error{HIPSTER_EUNSUPPORTED, "bispectrum: n_k outside [1, 16]"};
  if (nwaves < kXcds || nwaves % kXcds) throw Error{HIPSTER_EINVAL, "bispectrum: wave count must be a multiple of 8"};
  if (fp64 && !with_c) throw Error{HIPSTER_EINVAL, "bispectrum: the FP64 form sums C in the fused kernel"};
  if (fp64)
    k_bk_fused<NL, true, true><<<dim3(unsigned(nwaves)), dim3(64), lds, c.stream>>>(
        prim, sec, g.nc, g.L, r0 * r0, self_set ? 1 : 0, 0, prim.n, 1.0 / r0, edges, coef, NK, partial, rowlen, npairs);
  else if (with_c)
    k_bk_fused<NL, false, true><<<dim3(unsigned(nwaves)), dim3(64), lds, c.stream>>>(
        prim, sec, g.nc, g.L, r0 * r0, self_set ? 1 : 0, 0, prim.n, 1.0 / r0, edges, coef, NK, partial, rowlen, npairs);
  else
    k_bk_fused<NL, false, false><<<dim3(unsigned(nwaves)), dim3(64), lds, c.stream>>>(
        prim, sec, g.nc, g.L, r0 * r0, self_set ? 1 : 0, 0, prim.n, 1.0 / r0, edges, coef, NK, partial, rowlen, npairs);
  HIPSTER_HIP(hipGetLastError());
}

void bk_fused(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
              const double *edges, const double *coef, int NK, int ell_max, bool fp64, bool with_c, double *partial,
              int rowlen, int nwaves, unsigned long long *npairs) {
  switch (ell_max) {
    case 0: launch_fused<1>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, partial, rowlen, nwaves, npairs); break;
    case 1: launch_fused<2>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, partial, rowlen, nwaves, npairs); break;
    case 2: launch_fused<3>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, partial, rowlen, nwaves, npairs); break;
    case 3: launch_fused<4>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, partial, rowlen, nwaves, npairs); break;
    case 4: launch_fused<5>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, partial, rowlen, nwaves, npairs); break;
    case 5: launch_fused<6>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, partial, rowlen, nwaves, npairs); break;
    default: launch_fused<7>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, partial, rowlen, nwaves, npairs); break;
  }
}

}  // namespace hipster
