// Bispectrum path (Sec. 4): per-primary spherical-harmonic coefficients
//   A^a_lm(x_p) = sum_j w_j jbar^a_l(r_pj) W(r_pj/R0) y_lm(xhat_pj)      (eq. AC-def)
//   C^ab_l(x_p) = sum_j w_j^2 jbar^a_l jbar^b_l W^2
// for data primaries (j != p) and random primaries (all data j), contracted
// into G^ab_l = sum_p w_p (4 pi/(2l+1)) sum_m A^a_lm A^b_lm, with real
// orthonormal harmonics y_lm (the sum over m does not depend on the basis).
// Data primaries also give S0^b = sum_{p != j} w_p w_j jbar^b_0 W, the pair sum
// of the analytic DDR^I term.
//
// Work unit: a quad, up to four primaries of one home cell.  A wave takes a
// quad, one primary per 16-lane row, so each candidate secondary loaded from
// the 27 neighbour cells is tested against four primaries.  Hits go to one
// ring buffer per row; batches of up to 8 pairs per row are staged (lane =
// (row, pair): geometry, y_lm times w_q W, the top bin edge) and then swept in
// steps of one pair per row.  (Eight, not sixteen: the staging's LDS is what
// limits the waves per CU.)  In a step lane (col, row) evaluates
// k_e^3 G_l(k_e r) at bin edge e = 16 g + col for its row's pair and adds it
// times every y_lm into FP64 accumulators of its row's primary.  The y_lm of
// the step's pair reach all lanes of a row as 64-bit DPP broadcasts
// (row_newbcast) fused into the multiply-adds (fmac_dpp.h).  The mixed form
// sums per edge and takes each bin's sum A^{16g+col}_lm once per quad as the
// difference of adjacent lanes' edge sums (the top edge of the group summed
// from the staged values); the FP64 form, which also forms the C sums from
// each pair's bin values, takes the next edge's value from lane col + 1 by
// DPP in every step.
//
// Up to 16 bins: after each quad, G_l += A_l A_l^T on the FP64 matrix cores,
// the four primaries of the quad forming the instruction's K = 4 dimension,
// into accumulators that stay in registers until the wave ends.  More bins:
// one pass over the quads per group of 16 bins, A written to a buffer, then
// the Gram as a separate matrix-core contraction (k_bk_gram).
//
// Quads go to waves by a fixed rule and every sum is taken in a fixed order,
// so results are bitwise reproducible.
#include <type_traits>

// the special functions' Horner steps as plain fma (see fma3)
#define HIPSTER_PLAIN_FMA
#include "common.h"
#include "fmac_dpp.h"
#include "specfun.h"

namespace hipster {

// f times the real orthonormal spherical harmonics y_lm of a unit vector,
// index l*l+l+m: y_l0 = N_l0 Q_l^0(z), y_lm = N_lm Q_l^m(z) Re (x+iy)^m,
// y_l-m = N_lm Q_l^m(z) Im (x+iy)^m, with Q_l^m = d^m P_l / dz^m.  The factor f
// seeds the powers of (x+iy), and p_l = N_lm Q_l^m runs the three-term
// recurrence of Q_l^m with the normalisation ratios folded into its
// (compile-time) coefficients.
template <int LM, typename Out>
__device__ inline void real_ylm(double x, double y, double z, double f, Out Y) {
  double C[LM + 1], S[LM + 1];
  C[0] = f;
  S[0] = 0.0;
#pragma unroll
  for (int m = 1; m <= LM; ++m) {
    C[m] = C[m - 1] * x - S[m - 1] * y;
    S[m] = S[m - 1] * x + C[m - 1] * y;
  }
  double dfact = 1.0;  // (2m - 1)!!
#pragma unroll
  for (int m = 0; m <= LM; ++m) {
    if (m > 0) dfact *= double(2 * m - 1);
    double p2 = 0.0, p1 = 0.0;
#pragma unroll
    for (int l = m; l <= LM; ++l) {
      double p;
      if (l == m) {
        p = YLM_NORM[l][m] * dfact;
      } else if (l == m + 1) {
        p = (YLM_NORM[l][m] * double(2 * m + 1) * dfact) * z;
      } else {
        // Q_l = [(2l-1) z Q_{l-1} - (l+m-1) Q_{l-2}] / (l-m), in terms of p
        const double a = double(2 * l - 1) / double(l - m) * (YLM_NORM[l][m] / YLM_NORM[l - 1][m]);
        const double b = double(l + m - 1) / double(l - m) * (YLM_NORM[l][m] / YLM_NORM[l - 2][m]);
        p = fma(a * z, p1, -b * p2);
      }
      p2 = p1;
      p1 = p;
      if (m == 0) {
        Y[l * l + l] = p * f;
      } else {
        Y[l * l + l + m] = p * C[m];
        Y[l * l + l - m] = p * S[m];
      }
    }
  }
}

typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ inline d4_t mfma_f64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The value held by lane L+1 of the same 16-lane row (lane 15 of a row gets
// 0): a DPP row shift, no LDS round trip.
__device__ inline double from_next_lane_in_row(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int nlo = __builtin_amdgcn_update_dpp(0, lo, 0x101, 0xf, 0xf, false);  // row_shl:1
  const int nhi = __builtin_amdgcn_update_dpp(0, hi, 0x101, 0xf, 0xf, false);
  return __hiloint2double(nhi, nlo);
}

__device__ inline int64_t uniform_i64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v))));
  const int hi = __builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v) >> 32)));
  return int64_t((uint64_t(uint32_t(hi)) << 32) | uint64_t(uint32_t(lo)));
}

__device__ inline double uniform_f64(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

__device__ inline double bk_sq_norm(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  double a = dx * dx;
  double b = dy * dy;
  double c = dz * dz;
  return (a + b) + c;
}

// Orders the wave's LDS accesses: every lane's earlier LDS writes are visible
// to every lane's later LDS reads (one wave per workgroup).
__device__ inline void wave_sync() { __syncthreads(); }

constexpr int kXcds = 8;             // accelerator complex dies of the MI355X (the grid is a multiple)
constexpr int kQuadRun = 4;          // consecutive quads per wave assignment
// hit rings per row (powers of two): far and near class.  A row's hits come
// in bursts (a primary near one face of the home cell finds most of its
// neighbours in the cells on that side), so the far ring holds about a
// quad's imbalance between rows before a batch must run with idle rows.
constexpr int kHitCapF = 256;
constexpr int kHitCapN = 128;
template <int CL>
constexpr int hit_cap() { return CL == 0 ? kHitCapF : kHitCapN; }
// entry i of class CL's ring of row r in the flat ring array
template <int CL>
__device__ __forceinline__ int ring_at(int r, int i) {
  return CL == 0 ? r * kHitCapF + i : 4 * kHitCapF + r * kHitCapN + i;
}
constexpr int kRowBatch = 8;         // pairs per row per batch
constexpr int kSlots = 4 * kRowBatch;  // staged pairs per batch, slot = kRowBatch row + i
constexpr int kYStride = kSlots + 1;   // y staging row stride (odd)
// sine/cosine table entries (LDS).  At l_max = 5 the y staging of 36
// harmonics leaves room within 20 KiB per wave, the LDS share of two waves
// per SIMD, only for the 64-entry table (two more terms in its polynomials).
template <int NL>
constexpr int bk_tab() { return NL == 6 ? 64 : 256; }

// Writes w_q W y_lm of one slot into the y staging as real_ylm produces it:
// element idx goes to base[idx * kYStride].
template <typename YT>
struct YStore {
  YT *base;
  struct Ref {
    YT *p;
    __device__ void operator=(double v) const { *p = YT(v); }
  };
  __device__ Ref operator[](int idx) const { return Ref{base + idx * kYStride}; }
};

// Four primaries of one home cell (sorted indices; -1 = none, never first).
struct BkQuad {
  int p[4];
};

// One set of primaries against one box's secondaries.
struct BkJob {
  Sorted prim, sec;
  int nc;
  double L, r02, inv_r0;
  int self_set;
  const double *edges;  // n_k + 1
  const double *coef;   // n_k: 3 / (k_{a+1}^3 - k_a^3)
  int n_k;
  unsigned long long *npairs;  // ordered pairs inside R0 (added to)
};

// A queued task: quads [q0, q1) of job `job`; its sums go to row `slot`.
struct BkTask {
  int64_t q0, q1;
  int job, slot;
};

// Arguments of one sweep launch.  A single job: quads [q_lo, q_hi) of
// `job`, waves assigned by a fixed rule, per-wave rows.  Queued (many boxes):
// waves take tasks from `counter` until n_tasks are taken.
struct BkArgs {
  BkJob job;
  const BkQuad *quads;
  int64_t q_lo, q_hi;  // quads of this launch
  int group;            // bins 16 group .. 16 group + 15 of this pass
  double *partial;      // per-wave rows
  int rowlen;
  double *abuf;         // more than 16 bins: A of slot 4 (q - q_lo) + row, [NL^2][ld]
  double *wbuf;         // and w_p of that slot
  int ld;               // 16 * groups
  const BkJob *jobs;    // queued launch
  const BkTask *tasks;
  int n_tasks;
  int *counter;         // next task (zero before the launch)
  double *slots;        // one row per task
};

// Per-wave row layout.  Up to 16 bins: [G tiles NL*256 | C tiles NL*256 | S0 64];
// more: [S0 64 per group].  S0 entries are (row, bin) = 16 row + bin; their sum
// over rows is the S0 sum times 1/y_00.
__host__ __device__ inline int bk_rowlen(int NL, int groups) { return groups == 1 ? 2 * NL * 256 + 64 : 64 * groups; }

// y staging element: double in both forms (single-precision staging of
// w_q W y_lm left B errors at ~1 unit of 2^-24 of its scale on small boxes)
template <bool FP64>
using YStage = double;

template <int NL, bool FP64>
size_t bk_lds_bytes() {
  return size_t(NL * NL) * kYStride * sizeof(YStage<FP64>);
}

// G_l(u), l = 0 .. NL-1: the mixed form (double-precision table sine/cosine,
// single-precision sine-integral auxiliaries; Taylor series below u = 2) or
// the FP64 form.
template <int NL, bool FP64>
__device__ inline Gv<double, NL> G_any(double u, double wd, const double2 *tab) {
  if constexpr (FP64) return G_fp64<NL, 1>(u);
  else return G_mixed_w<NL, 1, bk_tab<NL>(), false>(u, wd, tab);
}

// fmac_block for l = L .. NL-1 (compile-time recursion).
template <int L, int NL, int NA, int NY>
__device__ __forceinline__ void fmac_all(double (&acc)[NA], const double (&yr)[NY], const double (&gl)[NL]) {
  if constexpr (L < NL) {
    fmac_block<L>(acc, yr, gl[L]);
    fmac_all<L + 1>(acc, yr, gl);
  }
}

// acc[l*l+m] = E^{e+1}_lm - E^e_lm for l = L .. NL-1, E^{e+1} from the next
// lane of the row, or on lane 15 (last) from the top-edge sums t (harmonic k
// on lane k % 16 of t[k / 16]).
template <int L, int NL, int NA, int NY>
__device__ __forceinline__ void edge_diff(double (&acc)[NA], const double (&t)[NY], bool last) {
  if constexpr (L < NL) {
    double tk[NA];
#pragma unroll
    for (int m = 0; m < 2 * L + 1; ++m) tk[L * L + m] = 0.0;
    fmac_block<L>(tk, t, 1.0);
#pragma unroll
    for (int m = 0; m < 2 * L + 1; ++m) {
      const int k = L * L + m;
      const double nx = from_next_lane_in_row(acc[k]);
      acc[k] = (last ? tk[k] : nx) - acc[k];
    }
    edge_diff<L + 1, NL>(acc, t, last);
  }
}

// Waves per SIMD the compiler must fit the sweep into (registers); more
// waves hide the latency of the candidate and staging loads.
#ifndef HIPSTER_BK_WAVES
#define HIPSTER_BK_WAVES 2
#endif

// Anisotropic combinations (l1 <= l2 < NL, m = 0 .. l1) in (l1, l2, m) order.
__host__ __device__ constexpr int aniso_count(int NL) {
  int c = 0;
  for (int l1 = 0; l1 < NL; ++l1) c += (NL - l1) * (l1 + 1);
  return c;
}

// NOTOP: the launch's group of bins is not full (no top edge), so the
// steps carry no top-edge sums.
template <int NL, bool FP64, bool WITH_C, bool GRAM, bool QUEUE, bool ANISO = false, bool NOTOP = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NL <= 6 ? HIPSTER_BK_WAVES : 1))) void k_bk_quad(
    BkArgs A) {
  static_assert(GRAM || !QUEUE, "the queued sweep keeps its Gram tiles in registers");
  static_assert(!ANISO || (GRAM && !FP64 && !WITH_C && !QUEUE), "the anisotropic sweep is single-box, mixed form");
  constexpr int NLM = NL * NL;
  constexpr int NY = (NLM + 15) / 16;
  using YT = YStage<FP64>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  YT *ylds = reinterpret_cast<YT *>(lds_raw);  // [NLM][kYStride]: w_q W y_lm of slot kRowBatch row + i
  __shared__ double s_r[kSlots], s_ir[kSlots], s_f[WITH_C ? kSlots : 1], s_gt[NL][kSlots];
  // hit rings per class (0: far, every edge of the group at u >= U_BIG;
  // 1: near) and row; an entry is (secondary index << 5) | image shift code
  __shared__ unsigned hl[4 * (kHitCapF + kHitCapN)];
  // the home cell's neighbour runs: [begin, end) of the sorted secondaries
  // (fewer than 2^27) and image shift code
  __shared__ int run_beg[27], run_end[27], run_sh[27], n_runs_s;
  // the quad's four primaries (x, y, z and index per row), read per scan step
  // from LDS rather than held in scalar registers; a row without a primary
  // has coordinates far outside any box, so that its tests never hit
  __shared__ double q_xyz[4][3];
  __shared__ int q_idx[4];
  __shared__ double2 sc_tab[FP64 ? 1 : bk_tab<NL>()];
  if constexpr (!FP64) stage_sincos_tab<bk_tab<NL>()>(sc_tab);
  for (int i = threadIdx.x; i < NL * kSlots; i += 64) (&s_gt[0][0])[i] = 0.0;

  const int lane = threadIdx.x, row = lane >> 4, col = lane & 15;
  const int64_t e0 = int64_t(16) * A.group;
  // the job's constants; a queued launch reloads them when its task's job changes
  BkJob J = A.job;
  double ke, ke3, ike, kn3, cfb, top_w, ktop, ktop3, iktop, r_neutral, ir_neutral, L, rfar, rfar2, r02v;
  bool top;
  auto set_job = [&]() {
    const int NK = J.n_k;
    // this lane's edge e = 16 g + col (clamped) and bin e (if it exists)
    const int e = int(e0) + col;
    ke = J.edges[e <= NK ? e : NK];
    ke3 = ke * ke * ke;
    ike = ke > 0.0 ? 1.0 / ke : 0.0;
    const double kn = J.edges[e + 1 <= NK ? e + 1 : NK];
    kn3 = kn * kn * kn;
    cfb = e < NK ? J.coef[e] : 0.0;
    // a full group of 16 bins takes its top edge 16 g + 16 from the staging
    top = e0 + 16 <= NK;
    top_w = top && col == 15 ? 1.0 : 0.0;
    ktop = top ? J.edges[e0 + 16] : 0.0;
    ktop3 = ktop * ktop * ktop;
    iktop = ktop > 0.0 ? 1.0 / ktop : 0.0;
    r_neutral = 0.5 / J.inv_r0;
    ir_neutral = 2.0 * J.inv_r0;
    L = J.L;
    // pairs at r^2 >= rfar2 put every edge of the group on the large-argument
    // side (no Taylor or sine-integral series); rfar2 = inf leaves all near
    const double k_lo = J.edges[e0];
    rfar = k_lo > 0.0 ? HIPSTER_U_BIG / k_lo : 0.0;
    rfar2 = (FP64 || !(k_lo > 0.0)) ? __builtin_inf() : rfar * rfar * (1.0 + 1e-12);
    // R0^2 for the scan's tests, kept in vector registers: the scalar ones
    // are short there
    r02v = J.r02;
    asm volatile("" : "+v"(r02v));
  };
  set_job();
  // Without the C sums (mixed form) each lane sums its own edge's values,
  // E^e_lm = sum_pairs k_e^3 G_l(k_e r) w_q W y_lm, and the bin sums are taken
  // once per quad as differences of adjacent lanes' sums; the top edge of a
  // full group is summed from the staged values (tacc, harmonic k = col + 16 i
  // of this row, multipole lk[i]).  The C sums need each pair's bin values,
  // so the FP64 form differences per pair.
  constexpr bool PER_EDGE = !WITH_C;
  int lk[NY];
#pragma unroll
  for (int i = 0; i < NY; ++i) {
    const int k = col + 16 * i;
    int l = 0;
#pragma unroll
    for (int t = 1; t < NL; ++t) l += k >= t * t ? 1 : 0;
    lk[i] = l;
  }
  // C sums (FP64 form) and the Gram tiles stay in matrix-core accumulators
  // for the wave's whole life and reach its row once, at the end (a
  // per-quad update of the 16 x 16 tiles in memory cost 10 KiB of writes per
  // quad at l_max = 4, every one of them leaving L2)
  d4_t accC[NL], accG[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) accC[l] = accG[l] = d4_t{0.0, 0.0, 0.0, 0.0};
  double s0acc = 0.0;
  double tl[ANISO ? NL : 1];  // anisotropic: sum_p w_p A^a_{l0}, per multipole
#pragma unroll
  for (int l = 0; l < (ANISO ? NL : 1); ++l) tl[l] = 0.0;
  unsigned long long pcount = 0;
  int64_t cur_cell = -1;
  wave_sync();

  // XCD-aware assignment: workgroups are dealt to the 8 XCDs round-robin, so
  // the waves of XCD x (blockIdx % 8 == x) share one contiguous eighth of the
  // quads (a slab of cells), whose neighbour data then stays in that XCD's
  // L2.  Within the slab, runs of kQuadRun quads go round-robin to its waves.
  auto quad = [&](int64_t qi) {
    {
      const BkQuad qd = A.quads[qi];
      int qp[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) qp[r] = __builtin_amdgcn_readfirstlane(qd.p[r]);
      const int64_t cell = J.prim.scell[qp[0]];
      if (cell != cur_cell) {
        // neighbour cells in (dx, dy, dz) order, merged into runs of the
        // sorted secondaries (cells adjacent along z are adjacent in memory)
        const int nc = J.nc;
        const int cz = int(cell % nc), cy = int((cell / nc) % nc), cx = int(cell / (int64_t(nc) * nc));
        int nbb = 0, nbe = 0, nbs = 0;
        if (lane < 27) {
          int sx = 0, sy = 0, sz = 0;
          int nx = cx + lane / 9 - 1, ny = cy + (lane / 3) % 3 - 1, nz = cz + lane % 3 - 1;
          if (nx >= nc) { nx -= nc; sx = 1; } else if (nx < 0) { nx += nc; sx = -1; }
          if (ny >= nc) { ny -= nc; sy = 1; } else if (ny < 0) { ny += nc; sy = -1; }
          if (nz >= nc) { nz -= nc; sz = 1; } else if (nz < 0) { nz += nc; sz = -1; }
          const int64_t nb = (int64_t(nx) * nc + ny) * nc + nz;
          nbb = int(J.sec.cell_start[nb]);
          nbe = int(J.sec.cell_start[nb + 1]);
          nbs = (sx + 1) * 9 + (sy + 1) * 3 + (sz + 1);
        }
        // merged in lane order (uniform), each run written when the next opens
        int nr = 0, rb = 0, re = 0, rs = 0;
        for (int k = 0; k < 27; ++k) {
          const int b = __builtin_amdgcn_readlane(nbb, k), e = __builtin_amdgcn_readlane(nbe, k);
          const int sc = __builtin_amdgcn_readlane(nbs, k);
          if (e == b) continue;
          if (nr > 0 && re == b && rs == sc) {
            re = e;
            continue;
          }
          if (nr > 0 && lane == 0) {
            run_beg[nr - 1] = rb;
            run_end[nr - 1] = re;
            run_sh[nr - 1] = rs;
          }
          rb = b;
          re = e;
          rs = sc;
          ++nr;
        }
        if (lane == 0) {
          if (nr > 0) {
            run_beg[nr - 1] = rb;
            run_end[nr - 1] = re;
            run_sh[nr - 1] = rs;
          }
          n_runs_s = nr;
        }
        wave_sync();
        cur_cell = cell;
      }
      const int n_runs = __builtin_amdgcn_readfirstlane(n_runs_s);
      // the four primaries (uniform), and this row's
      if (lane < 16) {
        const int r = lane / 4, d = lane % 4;
        const int pp = qp[r] >= 0 ? qp[r] : qp[0];
        if (d == 3) q_idx[r] = qp[r];
        else if (qp[r] < 0) q_xyz[r][d] = 1e300;
        else q_xyz[r][d] = d == 0 ? J.prim.x[pp] : (d == 1 ? J.prim.y[pp] : J.prim.z[pp]);
      }
      wave_sync();
      const int my_p = row == 0 ? qp[0] : row == 1 ? qp[1] : row == 2 ? qp[2] : qp[3];
      const bool my_valid = my_p >= 0;
      const int my_pp = my_valid ? my_p : qp[0];
      const double px = J.prim.x[my_pp], py = J.prim.y[my_pp], pz = J.prim.z[my_pp];
      const double wp = my_valid ? J.prim.w[my_pp] : 0.0;

      double acc[NLM], tacc[NY];
#pragma unroll
      for (int k = 0; k < NLM; ++k) acc[k] = 0.0;
#pragma unroll
      for (int i = 0; i < NY; ++i) tacc[i] = 0.0;
      // per class and row: hit count and ring head (uniform)
      int hn[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, hh[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};

      // one batch of class CL: up to kRowBatch pairs of each row
      auto batch = [&](auto cls) {
        constexpr int CL = decltype(cls)::value;
        int cnt[4];
        int cmax = 0;
        unsigned cpack = 0, hpack = 0;  // per-row count and head, 8 bits each
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cnt[r] = hn[CL][r] < kRowBatch ? hn[CL][r] : kRowBatch;
          cmax = cnt[r] > cmax ? cnt[r] : cmax;
          cpack |= unsigned(cnt[r]) << (8 * r);
          hpack |= unsigned(hh[CL][r]) << (8 * r);
        }
        const int my_cnt = int((cpack >> (8 * row)) & 255u);
        const int my_head = int((hpack >> (8 * row)) & 255u);
        // staging, lane (row, i = col < kRowBatch) = slot kRowBatch row + i
        if (col < kRowBatch) {
          const int slot = kRowBatch * row + col;
          double r = r_neutral, ir = ir_neutral, f = 0.0, ux = 0.0, uy = 0.0, uz = 1.0;
          if (col < my_cnt) {
            const int idx = (my_head + col) & (hit_cap<CL>() - 1);
            const unsigned ent = hl[ring_at<CL>(row, idx)];
            const int j = int(ent >> 5), sh = int(ent & 31u);
            const double ox = double(sh / 9 - 1) * L, oy = double((sh / 3) % 3 - 1) * L, oz = double(sh % 3 - 1) * L;
            const double dx = (px - J.sec.x[j]) - ox;
            const double dy = (py - J.sec.y[j]) - oy;
            const double dz = (pz - J.sec.z[j]) - oz;
            const double r2 = bk_sq_norm(dx, dy, dz);
            r = sqrt(r2);
            ir = r > 0.0 ? 1.0 / r : 0.0;
            f = J.sec.w[j] * window<double>(r * J.inv_r0);
            if (r > 0.0) {
              ux = dx * ir;
              uy = dy * ir;
              uz = dz * ir;
            }
          } else if (CL == 0) {
            r = rfar < r_neutral ? r_neutral : rfar;  // an idle slot of a far batch stays far
            ir = 1.0 / r;
          }
          // far class: k_e^3 G_l(k_e r) = Dt_l(k_e r) / r^3, the 1/r^3 goes with
          // the harmonics and the steps difference Dt values
          constexpr bool DT = !FP64 && CL == 0;
          const double fy = DT ? f * (ir * ir * ir) : f;
          real_ylm<NL - 1>(ux, uy, uz, fy, YStore<YT>{ylds + slot});
          s_r[slot] = r;
          s_ir[slot] = ir;
          if constexpr (WITH_C) s_f[slot] = f;
          if (!NOTOP && top) {
            if constexpr (DT) {
              const Gv<double, NL> T = Dt_far<NL, 1, false, bk_tab<NL>()>(ktop * r, iktop * ir, sc_tab);
#pragma unroll
              for (int l = 0; l < NL; ++l) s_gt[l][slot] = T.v[l];
            } else {
              const Gv<double, NL> T = G_any<NL, FP64>(ktop * r, iktop * ir, sc_tab);
#pragma unroll
              for (int l = 0; l < NL; ++l) s_gt[l][slot] = ktop3 * T.v[l];
            }
          }
        }
        wave_sync();
        // steps: one pair per row.  Two operand sets alternate, so the next
        // step's LDS operands are read while the current step computes
        // without register copies.
        auto ld_step = [&](int s, double &rq, double &irq, double (&yr)[NY]) {
          const int slot = kRowBatch * row + s;
          rq = s_r[slot];
          irq = s_ir[slot];
#pragma unroll
          for (int i = 0; i < NY; ++i) {
            // lanes past the last harmonic read a valid row; no multiply-add
            // broadcasts their value
            const int k = col + 16 * i < NLM ? col + 16 * i : NLM - 1;
            yr[i] = double(ylds[k * kYStride + slot]);
          }
        };
        auto step = [&](int s, double rq, double irq, const double (&yr)[NY]) {
          const int slot = kRowBatch * row + s;
          const double u = ke * rq, wd = ike * irq;
          // gl = [k^3 G_l(k r)] between this lane's edge and the next, without
          // the bin's 3 / (k_{a+1}^3 - k_a^3) (applied to A after the quad):
          // far class from Dt values (the 1/r^3 is in the harmonics)
          constexpr bool DT = !FP64 && CL == 0;
          Gv<double, NL> Ge;
          if constexpr (FP64) Ge = G_any<NL, true>(u, wd, sc_tab);
          else if constexpr (DT) Ge = Dt_far<NL, 1, false, bk_tab<NL>()>(u, wd, sc_tab);
          else Ge = G_any<NL, false>(u, wd, sc_tab);
          double gl[NL];
#pragma unroll
          for (int l = 0; l < NL; ++l) {
            if constexpr (PER_EDGE) {
              gl[l] = DT ? Ge.v[l] : ke3 * Ge.v[l];
            } else {
              // lane 15 of a row receives 0 from the shift and adds the top
              // edge (s_gt is zero unless the group is full)
              const double gn = from_next_lane_in_row(Ge.v[l]);
              const double hi = fma(s_gt[l][slot], top_w, DT ? gn : kn3 * gn);
              gl[l] = DT ? hi - Ge.v[l] : fma(-ke3, Ge.v[l], hi);
            }
          }
          // acc[l*l+m] += (w_q W y_lm)(pair) * jbar^a_l(pair)
          fmac_all<0>(acc, yr, gl);
          if constexpr (PER_EDGE) {
            // the top edge of a full group: harmonic k = col + 16 i of this
            // row's pair (yr[i]) times its staged value.  Lanes past the last
            // harmonic sum a value no broadcast reads; without a full group
            // the sum is unused (its bin factor is zero) and s_gt is finite.
            if constexpr (!NOTOP) {
#pragma unroll
              for (int i = 0; i < NY; ++i) tacc[i] = fma((&s_gt[0][0])[lk[i] * kSlots + slot], yr[i], tacc[i]);
            }
          }
          if constexpr (WITH_C) {
            const double fq = s_f[slot] * cfb;
#pragma unroll
            for (int l = 0; l < NL; ++l) {
              const double gq = gl[l] * fq;
              accC[l] = mfma_f64(gq, wp * gq, accC[l]);
            }
          }
        };
        double rq0, irq0, yr0[NY], rq1, irq1, yr1[NY];
        ld_step(0, rq0, irq0, yr0);
        for (int s = 0; s < cmax; s += 2) {
          const bool two = s + 1 < cmax;
          ld_step(two ? s + 1 : s, rq1, irq1, yr1);
          step(s, rq0, irq0, yr0);
          if (!two) break;
          ld_step(s + 2 < cmax ? s + 2 : s + 1, rq0, irq0, yr0);
          step(s + 1, rq1, irq1, yr1);
        }
        wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          hh[CL][r] = (hh[CL][r] + cnt[r]) & (hit_cap<CL>() - 1);
          hn[CL][r] -= cnt[r];
        }
      };
      using Far = std::integral_constant<int, 0>;
      using Near = std::integral_constant<int, 1>;

      // scan: runs of candidates, 64 at a time.  The next chunk's load is
      // issued after the current chunk's tests, so that it is in flight during
      // the batches (a wait for the current chunk would otherwise also wait
      // for it: loads complete in order)
      int ri = 0;
      int64_t pos = n_runs > 0 ? __builtin_amdgcn_readfirstlane(run_beg[0]) : 0;
      bool have = n_runs > 0;
      double cx = 0.0, cy = 0.0, cz = 0.0;
      int cj = 0;
      bool cok = false;
      int csh = 13;
      auto fetch = [&](double &x, double &y, double &z, int &j, bool &ok, int &sh) {
        const int64_t end = __builtin_amdgcn_readfirstlane(run_end[ri]);
        sh = __builtin_amdgcn_readfirstlane(run_sh[ri]);
        const int64_t jj = pos + lane;
        ok = jj < end;
        j = int(jj);
        if (ok) {
          x = J.sec.x[jj];
          y = J.sec.y[jj];
          z = J.sec.z[jj];
        }
        pos += 64;
        if (pos >= end) {
          ++ri;
          if (ri < n_runs) pos = __builtin_amdgcn_readfirstlane(run_beg[ri]);
        }
      };
      if (have) fetch(cx, cy, cz, cj, cok, csh);
      while (have) {
        const bool have_next = ri < n_runs;
        // the run's periodic image offset, from its shift code (uniform)
        const double ox = double(csh / 9 - 1) * L, oy = double((csh / 3) % 3 - 1) * L, oz = double(csh % 3 - 1) * L;
        const bool self_run = J.self_set && csh == 13;
        const unsigned ent = (unsigned(cj) << 5) | unsigned(csh);
        // the lane masks are formed as ballots of single compares (each is
        // the compare's own mask) joined by scalar operations; a ballot of a
        // compound predicate goes through a vector register
        const unsigned long long okm = __builtin_amdgcn_ballot_w64(cok);
        // the row tests, in one form for a run of the home image (no offset to
        // subtract: most runs) and one for a shifted image
        auto rows = [&](auto shifted) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // a row without a primary (only in the last quad of a cell) finds
          // r2 = inf
          double dx = q_xyz[r][0] - cx, dy = q_xyz[r][1] - cy, dz = q_xyz[r][2] - cz;
          if constexpr (decltype(shifted)::value) {
            dx -= ox;
            dy -= oy;
            dz -= oz;
          }
          const double r2 = bk_sq_norm(dx, dy, dz);
          const bool in = r2 < r02v, far = r2 >= rfar2, other = cj != q_idx[r];
          unsigned long long mh = __builtin_amdgcn_ballot_w64(in) & okm;
          if (self_run) mh &= __builtin_amdgcn_ballot_w64(other);
          const unsigned long long mf = __builtin_amdgcn_ballot_w64(far);
          const unsigned long long balf = mh & mf, baln = mh & ~mf;
          const bool hit = cok && in && (!self_run || other);
          // each class appends to its ring at the row's (uniform) end plus the
          // lane's rank among the class's hits
          if (hit && far) {
            const int pre = int(__builtin_amdgcn_mbcnt_hi(unsigned(balf >> 32), __builtin_amdgcn_mbcnt_lo(unsigned(balf), 0u)));
            hl[ring_at<0>(r, (hh[0][r] + hn[0][r] + pre) & (kHitCapF - 1))] = ent;
          }
          if (hit && !far) {
            const int pre = int(__builtin_amdgcn_mbcnt_hi(unsigned(baln >> 32), __builtin_amdgcn_mbcnt_lo(unsigned(baln), 0u)));
            hl[ring_at<1>(r, (hh[1][r] + hn[1][r] + pre) & (kHitCapN - 1))] = ent;
          }
          hn[0][r] += __popcll(balf);
          hn[1][r] += __popcll(baln);
          pcount += unsigned(__popcll(balf) + __popcll(baln));
        }
        };
        if (csh == 13) rows(std::false_type{});
        else rows(std::true_type{});
        double nx = 0.0, ny = 0.0, nz = 0.0;
        int nj = 0;
        bool nok = false;
        int nsh = 13;
        if (have_next) fetch(nx, ny, nz, nj, nok, nsh);
        // a batch of a class when every row has a full batch of it, or before a
        // row could overflow in the next step (each step adds at most 64 hits
        // per row and class)
        for (;;) {
          const int mn = min(min(hn[0][0], hn[0][1]), min(hn[0][2], hn[0][3]));
          const int mx = max(max(hn[0][0], hn[0][1]), max(hn[0][2], hn[0][3]));
          if (!(mn >= kRowBatch || mx > kHitCapF - 64)) break;
          wave_sync();
          batch(Far{});
        }
        for (;;) {
          const int mn = min(min(hn[1][0], hn[1][1]), min(hn[1][2], hn[1][3]));
          const int mx = max(max(hn[1][0], hn[1][1]), max(hn[1][2], hn[1][3]));
          if (!(mn >= kRowBatch || mx > kHitCapN - 64)) break;
          wave_sync();
          batch(Near{});
        }
        cx = nx;
        cy = ny;
        cz = nz;
        cj = nj;
        cok = nok;
        csh = nsh;
        have = have_next;
      }
      wave_sync();
      while (max(max(hn[0][0], hn[0][1]), max(hn[0][2], hn[0][3])) > 0) batch(Far{});
      while (max(max(hn[1][0], hn[1][1]), max(hn[1][2], hn[1][3])) > 0) batch(Near{});

      if constexpr (PER_EDGE) {
        // bin e = E^{e+1} - E^e; lane 15 of a row takes E^{e+1} from tacc,
        // each harmonic broadcast from the lane that holds it, one multipole
        // at a time (at most 2 l + 1 broadcasts live beside acc)
        edge_diff<0, NL>(acc, tacc, col == 15);
      }
      // the quad's contribution; the bin's 3 / (k_{a+1}^3 - k_a^3) first
#pragma unroll
      for (int k = 0; k < NLM; ++k) acc[k] *= cfb;
      if constexpr (ANISO) {
        // G^{ab}_{l1 l2 m} += w_p sum_{mu = +-m} A^a_{l1 mu} A^b_{l2 mu}, added to
        // the wave's row after every quad (too many tiles for registers)
        double *const wrow = A.partial + int64_t(blockIdx.x) * A.rowlen;
        int cidx = 0;
#pragma unroll
        for (int l1 = 0; l1 < NL; ++l1)
#pragma unroll
          for (int l2 = l1; l2 < NL; ++l2)
#pragma unroll
            for (int m = 0; m <= l1; ++m, ++cidx) {
              d4_t g = mfma_f64(acc[l1 * l1 + l1 + m], wp * acc[l2 * l2 + l2 + m], d4_t{0.0, 0.0, 0.0, 0.0});
              if (m > 0) g = mfma_f64(acc[l1 * l1 + l1 - m], wp * acc[l2 * l2 + l2 - m], g);
#pragma unroll
              for (int v = 0; v < 4; ++v) wrow[cidx * 256 + (row + 4 * v) * 16 + col] += g[v];
              // one tile's read-modify-write at a time: hoisting every tile's
              // loads would need all of their registers at once
              __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
        for (int l = 0; l < NL; ++l) tl[l] = fma(wp, acc[l * l + l], tl[l]);
      } else if constexpr (GRAM) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const double wsc = wp * (4.0 * kPi / double(2 * l + 1));
#pragma unroll
          for (int m = 0; m < 2 * l + 1; ++m) accG[l] = mfma_f64(acc[l * l + m], wsc * acc[l * l + m], accG[l]);
        }
      } else {
        const int64_t slot = (qi - A.q_lo) * 4 + row;
        double *ap = A.abuf + slot * NLM * A.ld + e0 + col;
#pragma unroll
        for (int k = 0; k < NLM; ++k) ap[int64_t(k) * A.ld] = acc[k];
        if (col == 0) A.wbuf[slot] = wp;
      }
      s0acc = fma(wp, acc[0], s0acc);
    }
  };

  if constexpr (!QUEUE) {
    const int xcd = int(blockIdx.x % kXcds), wx = int(blockIdx.x / kXcds), nwx = int(gridDim.x / kXcds);
    const int64_t nq = A.q_hi - A.q_lo;
    const int64_t s_lo = A.q_lo + nq * xcd / kXcds, s_hi = A.q_lo + nq * (xcd + 1) / kXcds;
    for (int64_t c0 = s_lo + int64_t(wx) * kQuadRun; c0 < s_hi; c0 += int64_t(nwx) * kQuadRun) {
      const int64_t c1 = c0 + kQuadRun < s_hi ? c0 + kQuadRun : s_hi;
      for (int64_t qi = c0; qi < c1; ++qi) quad(qi);
    }
    double *out = A.partial + int64_t(blockIdx.x) * A.rowlen;
    if constexpr (ANISO) {
#pragma unroll
      for (int l = 0; l < NL; ++l) out[aniso_count(NL) * 256 + l * 64 + lane] += tl[l];
    } else if constexpr (GRAM) {
#pragma unroll
      for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[l * 256 + (row + 4 * v) * 16 + col] += accG[l][v];
      if constexpr (WITH_C) {
#pragma unroll
        for (int l = 0; l < NL; ++l)
#pragma unroll
          for (int v = 0; v < 4; ++v) out[NL * 256 + l * 256 + (row + 4 * v) * 16 + col] += accC[l][v];
      }
      out[2 * NL * 256 + lane] += s0acc;
    } else {
      out[64 * A.group + lane] += s0acc;
    }
    if (lane == 0 && pcount && A.group == 0) atomicAdd(J.npairs, pcount);
  } else {
    // tasks in queue order until none is left; each task's sums go to its
    // own row, so the per-job merge is in a fixed order whichever wave ran it
    int cur_job = -1;
    for (;;) {
      int t = 0;
      if (lane == 0) t = atomicAdd(A.counter, 1);
      t = __builtin_amdgcn_readfirstlane(t);
      if (t >= A.n_tasks) break;
      const BkTask T = A.tasks[t];
      const int job = __builtin_amdgcn_readfirstlane(T.job);
      if (job != cur_job) {
        J = A.jobs[job];
        set_job();
        cur_job = job;
        cur_cell = -1;
      }
      const int64_t q0 = uniform_i64(T.q0), q1 = uniform_i64(T.q1);
      for (int64_t qi = q0; qi < q1; ++qi) quad(qi);
      double *out = A.slots + int64_t(__builtin_amdgcn_readfirstlane(T.slot)) * A.rowlen;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
#pragma unroll
        for (int v = 0; v < 4; ++v) out[l * 256 + (row + 4 * v) * 16 + col] = accG[l][v];
        accG[l] = d4_t{0.0, 0.0, 0.0, 0.0};
      }
      if constexpr (WITH_C) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
#pragma unroll
          for (int v = 0; v < 4; ++v) out[NL * 256 + l * 256 + (row + 4 * v) * 16 + col] = accC[l][v];
          accC[l] = d4_t{0.0, 0.0, 0.0, 0.0};
        }
      }
      out[2 * NL * 256 + lane] = s0acc;
      s0acc = 0.0;
      if (lane == 0 && pcount) atomicAdd(J.npairs, pcount);
      pcount = 0;
    }
  }
}

// Gram of the A buffer: one wave per (tile, chunk of slots), tile = (l, ga,
// gb), ga <= gb; the K dimension runs over (slot, m), four at a time.
// gpart[chunk][tile][256] += the tile's sum over the chunk (one wave per
// entry per launch, launches in stream order: deterministic).
struct GramTile {
  int l, ga, gb, pad;
};

__global__ __launch_bounds__(64) void k_bk_gram(const double *__restrict__ abuf, const double *__restrict__ wbuf,
                                                int64_t nslots, int NLM, int ld, const GramTile *__restrict__ tiles,
                                                int ntiles, int nchunks, double *__restrict__ gpart) {
  const int t = int(blockIdx.x % unsigned(ntiles)), ch = int(blockIdx.x / unsigned(ntiles));
  const int lane = threadIdx.x, row = lane >> 4, col = lane & 15;
  const GramTile T = tiles[t];
  const int nm = 2 * T.l + 1;
  const double sc = 4.0 * kPi / double(nm);
  const int64_t s_lo = nslots * ch / nchunks, s_hi = nslots * (ch + 1) / nchunks;
  const int64_t k_lo = s_lo * nm, k_hi = s_hi * nm;
  d4_t acc = d4_t{0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = k_lo; k0 < k_hi; k0 += 4) {
    const int64_t K = k0 + row;
    double a = 0.0, b = 0.0;
    if (K < k_hi) {
      const int64_t slot = K / nm;
      const int m = int(K - slot * nm);
      const double *base = abuf + (slot * NLM + T.l * T.l + m) * ld;
      a = base[16 * T.ga + col];
      b = wbuf[slot] * sc * base[16 * T.gb + col];
    }
    acc = mfma_f64(a, b, acc);
  }
  double *o = gpart + (int64_t(ch) * ntiles + t) * 256;
#pragma unroll
  for (int v = 0; v < 4; ++v) o[(row + 4 * v) * 16 + col] += acc[v];
}

// ------------------------------------------------------------------ quads
// Quads of a catalogue: per cell, its (selected) primaries four at a time, in
// the order `perm` gives (by neighbour count inside the cell), so that the
// four rows of a quad carry about the same number of pairs.
__global__ __launch_bounds__(256) void k_quad_count(const int64_t *__restrict__ cell_start,
                                                    const uint8_t *__restrict__ mask, int64_t ncells,
                                                    int64_t *__restrict__ qcount) {
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= ncells) return;
  const int64_t b = cell_start[c], e = cell_start[c + 1];
  int64_t n = e - b;
  if (mask) {
    n = 0;
    for (int64_t p = b; p < e; ++p) n += mask[p] ? 1 : 0;
  }
  qcount[c] = (n + 3) / 4;
}

__global__ __launch_bounds__(256) void k_quad_fill(const int64_t *__restrict__ cell_start,
                                                   const uint8_t *__restrict__ mask, const int *__restrict__ perm,
                                                   int64_t ncells, const int64_t *__restrict__ qoff,
                                                   BkQuad *__restrict__ quads) {
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= ncells) return;
  const int64_t b = cell_start[c], e = cell_start[c + 1];
  int64_t o = qoff[c];
  BkQuad q{{-1, -1, -1, -1}};
  int k = 0;
  for (int64_t i = b; i < e; ++i) {
    const int p = perm[i];
    if (mask && !mask[p]) continue;
    q.p[k++] = p;
    if (k == 4) {
      quads[o++] = q;
      q = BkQuad{{-1, -1, -1, -1}};
      k = 0;
    }
  }
  if (k) quads[o] = q;
}

// ------------------------------------------------------------------- host
// Elapsed time of the sweep launches alone, from two HIP events on the stream
// (read after the stream has been synchronised; 0 if an event is missing).
struct LaunchClock {
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  explicit LaunchClock(Ctx &c) : s(c.stream) {
    if (hipEventCreate(&a) != hipSuccess) a = nullptr;
    if (hipEventCreate(&b) != hipSuccess) b = nullptr;
  }
  void start() {
    if (a) HIPSTER_HIP(hipEventRecord(a, s));
  }
  void stop() {
    if (b) HIPSTER_HIP(hipEventRecord(b, s));
  }
  double ms() const {
    float t = 0.0f;
    return a && b && hipEventElapsedTime(&t, a, b) == hipSuccess ? double(t) : 0.0;
  }
  ~LaunchClock() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  LaunchClock(const LaunchClock &) = delete;
  LaunchClock &operator=(const LaunchClock &) = delete;
};

template <int NL, bool FP64, bool WITH_C, bool GRAM, bool QUEUE = false, bool NOTOP = false>
static void launch_quad(Ctx &c, const BkArgs &a, int nwaves) {
  const size_t lds = bk_lds_bytes<NL, FP64>();
  k_bk_quad<NL, FP64, WITH_C, GRAM, QUEUE, false, NOTOP><<<dim3(unsigned(nwaves)), dim3(64), lds, c.stream>>>(a);
  HIPSTER_HIP(hipGetLastError());
}

template <int NL, bool FP64, bool WITH_C, bool GRAM, bool QUEUE = false, bool NOTOP = false>
static int quad_waves(Ctx &c) {
  int per_cu = 0;
  const size_t lds = bk_lds_bytes<NL, FP64>();
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bk_quad<NL, FP64, WITH_C, GRAM, QUEUE, false, NOTOP>, 64,
                                                   lds) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  hipDeviceProp_t prop{};
  int cus = 256;
  if (hipGetDeviceProperties(&prop, c.device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  int n = cus * per_cu;
  return std::max(kXcds, n / kXcds * kXcds);
}

static BkJob bk_job(const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
                    const double *edges, const double *coef, int NK, unsigned long long *npairs) {
  BkJob j{};
  j.prim = prim;
  j.sec = sec;
  j.nc = g.nc;
  j.L = g.L;
  j.r02 = r0 * r0;
  j.inv_r0 = 1.0 / r0;
  j.self_set = self_set ? 1 : 0;
  j.edges = edges;
  j.coef = coef;
  j.n_k = NK;
  j.npairs = npairs;
  return j;
}

template <int NL>
static void bk_sweep_nl(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
                        const double *edges, const double *coef, int NK, bool fp64, bool with_c,
                        unsigned long long *npairs, BkSums &out) {
  const int groups = (NK + 15) / 16;
  if (fp64 && groups > 1)
    throw Error{HIPSTER_EUNSUPPORTED, "bispectrum: the FP64 form takes at most 16 bins (its C sums are per pair)"};
  if (with_c && !fp64) throw Error{HIPSTER_EINVAL, "bispectrum: the mixed form takes C from the pair histogram"};
  if (sec.n >= (int64_t(1) << 27))
    throw Error{HIPSTER_EUNSUPPORTED, "bispectrum: at most 2^27 - 1 data points (27-bit hit indices)"};
  out.NL = NL;
  out.NK = NK;
  out.G.assign(size_t(NL) * NK * NK, 0.0);
  out.C.assign(size_t(NL) * NK * NK, 0.0);
  out.S0.assign(size_t(NK), 0.0);
  if (prim.n == 0) return;
  // quads
  const int64_t ncells = g.ncells();
  int64_t *qcount = static_cast<int64_t *>(ensure(c, c.bq_count, size_t(ncells + 1) * 8));
  int64_t *qoff = static_cast<int64_t *>(ensure(c, c.bq_off, size_t(ncells + 1) * 8));
  const unsigned cb = unsigned((ncells + 255) / 256);
  k_quad_count<<<dim3(cb), dim3(256), 0, c.stream>>>(prim.cell_start, prim.m, ncells, qcount);
  HIPSTER_HIP(hipGetLastError());
  scan_i64(c, qcount, qoff, ncells, c.bq_scan);
  int64_t nq = 0;
  HIPSTER_HIP(hipMemcpyAsync(&nq, qoff + ncells, 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  if (nq == 0) return;
  BkQuad *quads = static_cast<BkQuad *>(ensure(c, c.bq_quads, size_t(nq) * sizeof(BkQuad)));
  const int *perm = order_by_neighbours(c, prim, sec, g, r0, self_set);
  k_quad_fill<<<dim3(cb), dim3(256), 0, c.stream>>>(prim.cell_start, prim.m, perm, ncells, qoff, quads);
  HIPSTER_HIP(hipGetLastError());

  BkArgs a{};
  a.job = bk_job(prim, sec, g, r0, self_set, edges, coef, NK, npairs);
  a.quads = quads;
  a.rowlen = bk_rowlen(NL, groups);
  a.ld = 16 * groups;

  if (groups == 1) {
    // the mixed form's steps leave out the top-edge sums when the bins do
    // not fill the group
    const bool full = NK == 16;
    const int nwaves = fp64   ? quad_waves<NL, true, true, true>(c)
                       : full ? quad_waves<NL, false, false, true>(c)
                              : quad_waves<NL, false, false, true, false, true>(c);
    double *part = static_cast<double *>(ensure(c, c.bk_partial, size_t(nwaves) * a.rowlen * 8));
    HIPSTER_HIP(hipMemsetAsync(part, 0, size_t(nwaves) * a.rowlen * 8, c.stream));
    a.partial = part;
    a.q_lo = 0;
    a.q_hi = nq;
    a.group = 0;
    LaunchClock clk(c);
    clk.start();
    if (fp64) launch_quad<NL, true, true, true>(c, a, nwaves);
    else if (full) launch_quad<NL, false, false, true>(c, a, nwaves);
    else launch_quad<NL, false, false, true, false, true>(c, a, nwaves);
    clk.stop();
    double *merged = static_cast<double *>(ensure(c, c.merged, size_t(a.rowlen) * 8));
    merge_partials(c, part, nwaves, a.rowlen, merged);
    std::vector<double> M(size_t(a.rowlen));
    HIPSTER_HIP(hipMemcpyAsync(M.data(), merged, size_t(a.rowlen) * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
    out.ms_kernel = clk.ms();
    // tiles are 16 x 16 per l; the Gram sums are symmetric up to rounding, so
    // the upper triangle is mirrored to make the output exactly symmetric
    for (int l = 0; l < NL; ++l)
      for (int x = 0; x < NK; ++x)
        for (int y = 0; y < NK; ++y) {
          const int t = l * 256 + std::min(x, y) * 16 + std::max(x, y);
          const size_t o = (size_t(l) * NK + x) * NK + y;
          out.G[o] = M[size_t(t)];
          out.C[o] = M[size_t(NL * 256 + t)];
        }
    for (int b = 0; b < NK; ++b) {
      double s = 0.0;
      for (int r = 0; r < 4; ++r) s += M[size_t(2 * NL * 256 + 16 * r + b)];
      out.S0[size_t(b)] = s;
    }
    out.launches = 1;
    return;
  }

  // more than 16 bins: A through a buffer, one pass per bin group
  constexpr int NLM = NL * NL;
  const int ld = 16 * groups;
  const int64_t bytes_per_quad = int64_t(4) * NLM * ld * 8;
  const int64_t budget = int64_t(1) << 30;
  const int64_t qchunk = std::max<int64_t>(1, std::min<int64_t>(nq, budget / bytes_per_quad));
  const int nwaves = quad_waves<NL, false, false, false>(c);
  double *part = static_cast<double *>(ensure(c, c.bk_partial, size_t(nwaves) * a.rowlen * 8));
  HIPSTER_HIP(hipMemsetAsync(part, 0, size_t(nwaves) * a.rowlen * 8, c.stream));
  a.partial = part;
  a.abuf = static_cast<double *>(ensure(c, c.bk_abuf, size_t(qchunk) * size_t(bytes_per_quad)));
  a.wbuf = static_cast<double *>(ensure(c, c.bk_wbuf, size_t(qchunk) * 4 * 8));
  std::vector<GramTile> tl;
  for (int l = 0; l < NL; ++l)
    for (int ga = 0; ga < groups; ++ga)
      for (int gb = ga; gb < groups; ++gb) tl.push_back(GramTile{l, ga, gb, 0});
  const int ntiles = int(tl.size());
  GramTile *tiles = static_cast<GramTile *>(ensure(c, c.bk_tiles, tl.size() * sizeof(GramTile)));
  HIPSTER_HIP(hipMemcpyAsync(tiles, tl.data(), tl.size() * sizeof(GramTile), hipMemcpyHostToDevice, c.stream));
  const int nchunks = std::max(1, std::min(256, 4096 / ntiles));
  double *gpart = static_cast<double *>(ensure(c, c.bk_gpart, size_t(nchunks) * ntiles * 256 * 8));
  HIPSTER_HIP(hipMemsetAsync(gpart, 0, size_t(nchunks) * ntiles * 256 * 8, c.stream));
  uint64_t launches = 0;
  LaunchClock clk(c);
  clk.start();
  for (int64_t q0 = 0; q0 < nq; q0 += qchunk) {
    a.q_lo = q0;
    a.q_hi = std::min(nq, q0 + qchunk);
    for (int gi = 0; gi < groups; ++gi) {
      a.group = gi;
      // the last group, when not full, without the top-edge sums
      if (16 * (gi + 1) <= NK) launch_quad<NL, false, false, false>(c, a, nwaves);
      else launch_quad<NL, false, false, false, false, true>(c, a, nwaves);
      ++launches;
    }
    k_bk_gram<<<dim3(unsigned(ntiles * nchunks)), dim3(64), 0, c.stream>>>(a.abuf, a.wbuf, (a.q_hi - a.q_lo) * 4, NLM,
                                                                           ld, tiles, ntiles, nchunks, gpart);
    HIPSTER_HIP(hipGetLastError());
  }
  clk.stop();
  double *merged = static_cast<double *>(ensure(c, c.merged, size_t(std::max(a.rowlen, ntiles * 256)) * 8));
  double *gmerged = static_cast<double *>(ensure(c, c.bk_gmerged, size_t(ntiles) * 256 * 8));
  merge_partials(c, part, nwaves, a.rowlen, merged);
  merge_partials(c, gpart, nchunks, ntiles * 256, gmerged);
  std::vector<double> M(size_t(a.rowlen)), GM(size_t(ntiles) * 256);
  HIPSTER_HIP(hipMemcpyAsync(M.data(), merged, size_t(a.rowlen) * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(GM.data(), gmerged, GM.size() * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  out.ms_kernel = clk.ms();
  std::vector<int> tindex(size_t(NL) * groups * groups, -1);
  for (int t = 0; t < ntiles; ++t) tindex[(size_t(tl[t].l) * groups + tl[t].ga) * groups + tl[t].gb] = t;
  for (int l = 0; l < NL; ++l)
    for (int x = 0; x < NK; ++x)
      for (int y = 0; y < NK; ++y) {
        const int lo = std::min(x, y), hi = std::max(x, y);
        const int t = tindex[(size_t(l) * groups + lo / 16) * groups + hi / 16];
        out.G[(size_t(l) * NK + x) * NK + y] = GM[size_t(t) * 256 + (lo % 16) * 16 + hi % 16];
      }
  for (int b = 0; b < NK; ++b) {
    double s = 0.0;
    for (int r = 0; r < 4; ++r) s += M[size_t(64 * (b / 16) + 16 * r + b % 16)];
    out.S0[size_t(b)] = s;
  }
  out.launches = launches;
}

template <int NL>
static void bk_sweep_queue_nl(Ctx &c, const std::vector<BkQueueJob> &jobs, bool fp64, std::vector<BkSums> &out) {
  const int nj = int(jobs.size());
  out.assign(size_t(nj), BkSums{});
  for (int j = 0; j < nj; ++j) {
    const BkQueueJob &J = jobs[size_t(j)];
    if (J.NK < 1 || J.NK > 16) throw Error{HIPSTER_EUNSUPPORTED, "queued bispectrum: n_k must lie in [1, 16]"};
    if (J.sec.n >= (int64_t(1) << 27))
      throw Error{HIPSTER_EUNSUPPORTED, "bispectrum: at most 2^27 - 1 data points (27-bit hit indices)"};
    out[size_t(j)].NL = NL;
    out[size_t(j)].NK = J.NK;
    out[size_t(j)].G.assign(size_t(NL) * J.NK * J.NK, 0.0);
    out[size_t(j)].C.assign(size_t(NL) * J.NK * J.NK, 0.0);
    out[size_t(j)].S0.assign(size_t(J.NK), 0.0);
  }
  if (nj == 0) return;
  // quads of every job: per-job counts and offsets side by side, one readback
  std::vector<int64_t> cbase(size_t(nj) + 1, 0);
  for (int j = 0; j < nj; ++j) cbase[size_t(j) + 1] = cbase[size_t(j)] + jobs[size_t(j)].g.ncells() + 1;
  int64_t *qcount = static_cast<int64_t *>(ensure(c, c.bq_count, size_t(cbase[size_t(nj)]) * 8));
  int64_t *qoff = static_cast<int64_t *>(ensure(c, c.bq_off, size_t(cbase[size_t(nj)]) * 8));
  std::vector<int64_t> nq(size_t(nj), 0);
  for (int j = 0; j < nj; ++j) {
    const BkQueueJob &J = jobs[size_t(j)];
    const int64_t ncells = J.g.ncells();
    if (J.prim.n == 0) continue;
    const unsigned cb = unsigned((ncells + 255) / 256);
    k_quad_count<<<dim3(cb), dim3(256), 0, c.stream>>>(J.prim.cell_start, J.prim.m, ncells, qcount + cbase[size_t(j)]);
    HIPSTER_HIP(hipGetLastError());
    scan_i64(c, qcount + cbase[size_t(j)], qoff + cbase[size_t(j)], ncells, c.bq_scan);
    HIPSTER_HIP(hipMemcpyAsync(&nq[size_t(j)], qoff + cbase[size_t(j)] + ncells, 8, hipMemcpyDeviceToHost, c.stream));
  }
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  std::vector<int64_t> qbase(size_t(nj) + 1, 0);
  for (int j = 0; j < nj; ++j) qbase[size_t(j) + 1] = qbase[size_t(j)] + nq[size_t(j)];
  const int64_t total = qbase[size_t(nj)];
  if (total == 0) return;
  BkQuad *quads = static_cast<BkQuad *>(ensure(c, c.bq_quads, size_t(total) * sizeof(BkQuad)));
  for (int j = 0; j < nj; ++j) {
    const BkQueueJob &J = jobs[size_t(j)];
    if (nq[size_t(j)] == 0) continue;
    const int64_t ncells = J.g.ncells();
    const unsigned cb = unsigned((ncells + 255) / 256);
    const int *perm = order_by_neighbours(c, J.prim, J.sec, J.g, J.r0, J.self_set);
    k_quad_fill<<<dim3(cb), dim3(256), 0, c.stream>>>(J.prim.cell_start, J.prim.m, perm, ncells,
                                                      qoff + cbase[size_t(j)], quads + qbase[size_t(j)]);
    HIPSTER_HIP(hipGetLastError());
  }
  // tasks of about equal expected work (pairs), some eight per wave; jobs in
  // order of expected pairs per quad (dearest first), each job's tasks
  // consecutive.  A box's pairs per quad can differ from another's by 1e4.
  // the mixed form's steps leave out the top-edge sums when no job's bins
  // fill the group
  bool any_full = false;
  for (const BkQueueJob &J : jobs) any_full = any_full || J.NK == 16;
  const int nwaves = fp64       ? quad_waves<NL, true, true, true, true>(c)
                     : any_full ? quad_waves<NL, false, false, true, true>(c)
                                : quad_waves<NL, false, false, true, true, true>(c);
  double work = 0.0;
  for (int j = 0; j < nj; ++j) work += double(nq[size_t(j)]) * (4.0 * jobs[size_t(j)].cost + 1.0);
  const double per_task = std::max(1.0, work / (8.0 * nwaves));
  std::vector<int> order(static_cast<size_t>(nj));
  for (int j = 0; j < nj; ++j) order[size_t(j)] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return jobs[size_t(a)].cost > jobs[size_t(b)].cost; });
  std::vector<BkTask> tasks;
  std::vector<int> tfirst(size_t(nj), 0), tcount(size_t(nj), 0);
  for (int j : order) {
    tfirst[size_t(j)] = int(tasks.size());
    const int64_t tq = std::max<int64_t>(
        1, std::min<int64_t>(4096, int64_t(per_task / (4.0 * jobs[size_t(j)].cost + 1.0))));
    for (int64_t q0 = qbase[size_t(j)]; q0 < qbase[size_t(j) + 1]; q0 += tq) {
      const int slot = int(tasks.size());
      tasks.push_back(BkTask{q0, std::min(qbase[size_t(j) + 1], q0 + tq), j, slot});
    }
    tcount[size_t(j)] = int(tasks.size()) - tfirst[size_t(j)];
  }
  std::vector<BkJob> hj(static_cast<size_t>(nj));
  for (int j = 0; j < nj; ++j) {
    const BkQueueJob &J = jobs[size_t(j)];
    hj[size_t(j)] = bk_job(J.prim, J.sec, J.g, J.r0, J.self_set, J.edges, J.coef, J.NK, J.npairs);
  }
  const int rowlen = bk_rowlen(NL, 1);
  BkJob *djobs = static_cast<BkJob *>(ensure(c, c.bq_jobs, hj.size() * sizeof(BkJob)));
  BkTask *dtasks = static_cast<BkTask *>(ensure(c, c.bq_tasks, tasks.size() * sizeof(BkTask)));
  double *slots = static_cast<double *>(ensure(c, c.bq_slots, tasks.size() * size_t(rowlen) * 8));
  int *counter = static_cast<int *>(ensure(c, c.bq_counter, 16));
  HIPSTER_HIP(hipMemcpyAsync(djobs, hj.data(), hj.size() * sizeof(BkJob), hipMemcpyHostToDevice, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(dtasks, tasks.data(), tasks.size() * sizeof(BkTask), hipMemcpyHostToDevice, c.stream));
  HIPSTER_HIP(hipMemsetAsync(counter, 0, 4, c.stream));
  BkArgs a{};
  a.job = hj[size_t(order[0])];
  a.quads = quads;
  a.group = 0;
  a.rowlen = rowlen;
  a.ld = 16;
  a.jobs = djobs;
  a.tasks = dtasks;
  a.n_tasks = int(tasks.size());
  a.counter = counter;
  a.slots = slots;
  if (fp64) launch_quad<NL, true, true, true, true>(c, a, nwaves);
  else if (any_full) launch_quad<NL, false, false, true, true>(c, a, nwaves);
  else launch_quad<NL, false, false, true, true, true>(c, a, nwaves);
  // per job: its task rows in task order
  double *merged = static_cast<double *>(ensure(c, c.bk_gmerged, size_t(nj) * rowlen * 8));
  for (int j = 0; j < nj; ++j) {
    if (tcount[size_t(j)] == 0) {
      HIPSTER_HIP(hipMemsetAsync(merged + size_t(j) * rowlen, 0, size_t(rowlen) * 8, c.stream));
      continue;
    }
    merge_partials(c, slots + size_t(tfirst[size_t(j)]) * rowlen, tcount[size_t(j)], rowlen,
                   merged + size_t(j) * rowlen);
  }
  std::vector<double> M(size_t(nj) * rowlen);
  HIPSTER_HIP(hipMemcpyAsync(M.data(), merged, M.size() * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  for (int j = 0; j < nj; ++j) {
    const int NK = jobs[size_t(j)].NK;
    const double *Mj = M.data() + size_t(j) * rowlen;
    BkSums &o = out[size_t(j)];
    for (int l = 0; l < NL; ++l)
      for (int x = 0; x < NK; ++x)
        for (int y = 0; y < NK; ++y) {
          const int t = l * 256 + std::min(x, y) * 16 + std::max(x, y);
          const size_t oi = (size_t(l) * NK + x) * NK + y;
          o.G[oi] = Mj[size_t(t)];
          o.C[oi] = fp64 ? Mj[size_t(NL * 256 + t)] : 0.0;
        }
    for (int b = 0; b < NK; ++b) {
      double s0 = 0.0;
      for (int r = 0; r < 4; ++r) s0 += Mj[size_t(2 * NL * 256 + 16 * r + b)];
      o.S0[size_t(b)] = s0;
    }
    o.launches = 1;
  }
}

void bk_sweep_queue(Ctx &c, const std::vector<BkQueueJob> &jobs, int ell_max, bool fp64, std::vector<BkSums> &out) {
  switch (ell_max) {
    case 0: bk_sweep_queue_nl<1>(c, jobs, fp64, out); break;
    case 1: bk_sweep_queue_nl<2>(c, jobs, fp64, out); break;
    case 2: bk_sweep_queue_nl<3>(c, jobs, fp64, out); break;
    case 3: bk_sweep_queue_nl<4>(c, jobs, fp64, out); break;
    case 4: bk_sweep_queue_nl<5>(c, jobs, fp64, out); break;
    case 5: bk_sweep_queue_nl<6>(c, jobs, fp64, out); break;
    case 6: bk_sweep_queue_nl<7>(c, jobs, fp64, out); break;
    default: throw Error{HIPSTER_EDOMAIN, "ell_max must lie in [0, 6]"};
  }
}

template <int NL>
static void bk_aniso_nl(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
                        const double *edges, const double *coef, int NK, unsigned long long *npairs,
                        std::vector<double> &G, std::vector<double> &T, double &ms_kernel) {
  constexpr int NC = aniso_count(NL);
  if (NK < 1 || NK > 16) throw Error{HIPSTER_EUNSUPPORTED, "anisotropic bispectrum: n_k must lie in [1, 16]"};
  if (sec.n >= (int64_t(1) << 27))
    throw Error{HIPSTER_EUNSUPPORTED, "bispectrum: at most 2^27 - 1 data points (27-bit hit indices)"};
  G.assign(size_t(NC) * NK * NK, 0.0);
  T.assign(size_t(NL) * NK, 0.0);
  if (prim.n == 0) return;
  const int64_t ncells = g.ncells();
  int64_t *qcount = static_cast<int64_t *>(ensure(c, c.bq_count, size_t(ncells + 1) * 8));
  int64_t *qoff = static_cast<int64_t *>(ensure(c, c.bq_off, size_t(ncells + 1) * 8));
  const unsigned cb = unsigned((ncells + 255) / 256);
  k_quad_count<<<dim3(cb), dim3(256), 0, c.stream>>>(prim.cell_start, prim.m, ncells, qcount);
  HIPSTER_HIP(hipGetLastError());
  scan_i64(c, qcount, qoff, ncells, c.bq_scan);
  int64_t nq = 0;
  HIPSTER_HIP(hipMemcpyAsync(&nq, qoff + ncells, 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  if (nq == 0) return;
  BkQuad *quads = static_cast<BkQuad *>(ensure(c, c.bq_quads, size_t(nq) * sizeof(BkQuad)));
  const int *perm = order_by_neighbours(c, prim, sec, g, r0, self_set);
  k_quad_fill<<<dim3(cb), dim3(256), 0, c.stream>>>(prim.cell_start, prim.m, perm, ncells, qoff, quads);
  HIPSTER_HIP(hipGetLastError());
  BkArgs a{};
  a.job = bk_job(prim, sec, g, r0, self_set, edges, coef, NK, npairs);
  a.quads = quads;
  a.q_lo = 0;
  a.q_hi = nq;
  a.group = 0;
  a.rowlen = NC * 256 + NL * 64;
  a.ld = 16;
  int per_cu = 0;
  const size_t lds = bk_lds_bytes<NL, false>();
  // without a full group of bins the steps carry no top-edge sums
  void (*const kern)(BkArgs) = NK == 16 ? k_bk_quad<NL, false, false, true, false, true>
                                        : k_bk_quad<NL, false, false, true, false, true, true>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  hipDeviceProp_t prop{};
  int cus = 256;
  if (hipGetDeviceProperties(&prop, c.device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  const int nwaves = std::max(kXcds, cus * per_cu / kXcds * kXcds);
  double *part = static_cast<double *>(ensure(c, c.bk_partial, size_t(nwaves) * a.rowlen * 8));
  HIPSTER_HIP(hipMemsetAsync(part, 0, size_t(nwaves) * a.rowlen * 8, c.stream));
  a.partial = part;
  LaunchClock clk(c);
  clk.start();
  hipLaunchKernelGGL(kern, dim3(unsigned(nwaves)), dim3(64), lds, c.stream, a);
  HIPSTER_HIP(hipGetLastError());
  clk.stop();
  double *merged = static_cast<double *>(ensure(c, c.merged, size_t(a.rowlen) * 8));
  merge_partials(c, part, nwaves, a.rowlen, merged);
  std::vector<double> M(size_t(a.rowlen));
  HIPSTER_HIP(hipMemcpyAsync(M.data(), merged, size_t(a.rowlen) * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  ms_kernel += clk.ms();
  // tile c: D[a][b] = sum_p w_p sum_mu A^a_{l1 mu} A^b_{l2 mu} at c 256 + 16 a + b
  for (int ci = 0; ci < NC; ++ci)
    for (int x = 0; x < NK; ++x)
      for (int y = 0; y < NK; ++y) G[(size_t(ci) * NK + x) * NK + y] = M[size_t(ci * 256 + x * 16 + y)];
  for (int l = 0; l < NL; ++l)
    for (int b = 0; b < NK; ++b) {
      double t = 0.0;
      for (int r = 0; r < 4; ++r) t += M[size_t(NC * 256 + l * 64 + 16 * r + b)];
      T[size_t(l) * NK + b] = t;
    }
}

void bk_aniso_sweep(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
                    const double *edges, const double *coef, int NK, int ell_max, unsigned long long *npairs,
                    std::vector<double> &G, std::vector<double> &T, double &ms_kernel) {
  switch (ell_max) {
    case 0: bk_aniso_nl<1>(c, prim, sec, g, r0, self_set, edges, coef, NK, npairs, G, T, ms_kernel); break;
    case 1: bk_aniso_nl<2>(c, prim, sec, g, r0, self_set, edges, coef, NK, npairs, G, T, ms_kernel); break;
    case 2: bk_aniso_nl<3>(c, prim, sec, g, r0, self_set, edges, coef, NK, npairs, G, T, ms_kernel); break;
    case 3: bk_aniso_nl<4>(c, prim, sec, g, r0, self_set, edges, coef, NK, npairs, G, T, ms_kernel); break;
    case 4: bk_aniso_nl<5>(c, prim, sec, g, r0, self_set, edges, coef, NK, npairs, G, T, ms_kernel); break;
    default: throw Error{HIPSTER_EUNSUPPORTED, "anisotropic bispectrum: ell_max must lie in [0, 4]"};
  }
}

void bk_sweep(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
              const double *edges, const double *coef, int NK, int ell_max, bool fp64, bool with_c,
              unsigned long long *npairs, BkSums &out) {
  if (NK < 1 || NK > kMaxNkB)
    throw Error{HIPSTER_EUNSUPPORTED, "bispectrum: n_k outside [1, " + std::to_string(kMaxNkB) + "]"};
  switch (ell_max) {
    case 0: bk_sweep_nl<1>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, npairs, out); break;
    case 1: bk_sweep_nl<2>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, npairs, out); break;
    case 2: bk_sweep_nl<3>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, npairs, out); break;
    case 3: bk_sweep_nl<4>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, npairs, out); break;
    case 4: bk_sweep_nl<5>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, npairs, out); break;
    case 5: bk_sweep_nl<6>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, npairs, out); break;
    default: bk_sweep_nl<7>(c, prim, sec, g, r0, self_set, edges, coef, NK, fp64, with_c, npairs, out); break;
  }
}

}  // namespace hipster
