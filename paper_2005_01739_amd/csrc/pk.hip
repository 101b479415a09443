// Power-spectrum pair-weight sweep (the dominant cost; Sec. 9 of the paper
// names the Bessel weights the limiting step).
//
// For each unordered pair (r, mu, w_i w_j m_ij) and each bin edge k_e the
// single-box sweep adds c_l k_e^3 G_l(k_e r) to a per-lane double accumulator,
// with c_l = w_i w_j m_ij W(r/R0) L_l(mu).  The bin values follow on the host as
// S^a_l = 3 (2l+1) (-i)^l [E'_l(a+1) - E'_l(a)] / (k_{a+1}^3 - k_a^3),
// E'_l(e) = sum over pairs of c_l k_e^3 G_l(k_e r) (Sec. 3, binned estimator
// with eq. jla-def).  Since k^3 G_l(k r) = Dt_l(k r) / r^3, pairs of the far
// bucket (r >= U_BIG / k_0, so every edge is on the large-argument side) go
// through a kernel of their own that accumulates (c_l / r^3) Dt_l(k_e r) with
// no per-edge rescaling; pairs of the near bucket (and every pair in the FP64
// form) take the general kernel, which evaluates G_l and scales it by k_e^3.
// Edges are processed in chunks so the accumulators stay in registers; the
// pair stream is re-read once per chunk.  Each wave reduces its lanes with
// cross-lane shuffles and adds its sums to its own row of `partial` (the far
// kernel runs after the general one on the same stream, with the same rows);
// rows are merged in a fixed order, so results are bitwise reproducible.
#include <type_traits>

#include "common.h"
#include "specfun.h"

namespace hipster {

constexpr int kSweepBlock = 256;
constexpr int kChunk = 8;  // batched sweep

// Edges per chunk of the single-box sweep.  A larger chunk reads the pair
// stream fewer times and spreads each pair's set-up (window, Legendre, 1/r)
// over more edges, at the cost of registers.  The far kernel evaluates all CH
// edges of a chunk without branches (past the last edge it repeats the last
// edge and discards the result), so the host picks its CH per edge count from
// the compiled sizes below to keep that padding small.
constexpr int kChunksMixed3[3] = {21, 16, 11};  // far path, up to three multipoles
constexpr int kChunksMixed4[3] = {14, 11, 8};   // far path, four multipoles
constexpr int kChunkNear = 11;                  // general path, mixed form (near bucket)
constexpr int kChunkFp64 = 8;                   // general path, FP64 form

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Minimum waves per SIMD for the sweep (a build-time tuning knob).
#ifndef HIPSTER_PK_WAVES_PER_EU
#define HIPSTER_PK_WAVES_PER_EU 2
#endif

// Per-pair set-up shared by both buckets: c_l = w W(r/R0) L_l(mu).
template <int NE>
__device__ inline void pair_coeffs(double r, double mu, double ww, double inv_r0, double (&cf)[NE]) {
  const double wt = ww * window<double>(r * inv_r0);
  double L[NE];
  legendre_even<double, NE>(mu, L);
#pragma unroll
  for (int i = 0; i < NE; ++i) cf[i] = wt * L[i];
}

// ek holds the edge table written by the host: k_e, 1/k_e, k_e^3 (doubles,
// n_edges each).
//
// General path: pairs [0, npairs) of its stream, any r, G_l(k_e r) k_e^3 from
// the full special functions (the FP64 form, and the near bucket of the mixed
// form).  Balanced chunks of at most CH edges.
template <int NE, bool FP64, int CH>
__global__ __launch_bounds__(kSweepBlock) __attribute__((amdgpu_waves_per_eu(HIPSTER_PK_WAVES_PER_EU))) void k_pk_sweep(
    const double *__restrict__ pr, const double *__restrict__ pmu, const double *__restrict__ pww, int64_t npairs,
    double inv_r0, const double *__restrict__ ek, int n_edges, double *__restrict__ partial) {
  const double *k_e = ek, *inv_k = ek + n_edges, *k3 = ek + 2 * n_edges;
  __shared__ double2 tab[FP64 ? 1 : kSinCosTab];
  if constexpr (!FP64) {
    stage_sincos_tab<kSinCosTab>(tab);
    __syncthreads();
  }
  const int64_t gtid = int64_t(blockIdx.x) * kSweepBlock + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * kSweepBlock;
  const int wave = int(gtid >> 6), lane = threadIdx.x & 63;
  const int nchunk = (n_edges + CH - 1) / CH, per = (n_edges + nchunk - 1) / nchunk;
  for (int e0 = 0; e0 < n_edges; e0 += per) {
    const int e_end = e0 + per < n_edges ? e0 + per : n_edges;
    double acc[NE][CH];
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) acc[i][cc] = 0.0;
    for (int64_t p = gtid; p < npairs; p += stride) {
      const double r = pr[p];
      double cf[NE];
      pair_coeffs<NE>(r, pmu[p], pww[p], inv_r0, cf);
      const double inv_r = r > 0.0 ? 1.0 / r : 0.0;
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) {
        const int e = e0 + cc;
        if (e < e_end) {
          const double u = k_e[e] * r;
          Gv<double, NE> G;
          // the Taylor branch inline (measured faster), except with four
          // multipoles, where it would spill
          if constexpr (FP64) G = G_fp64<NE, 2, true>(u);
          else G = G_mixed_w<NE, 2, kSinCosTab, (NE <= 3)>(u, inv_k[e] * inv_r, tab);
          const double s3 = k3[e];
#pragma unroll
          for (int i = 0; i < NE; ++i) acc[i][cc] = fma(cf[i], G.v[i] * s3, acc[i][cc]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) {
        const double v = wave_sum(acc[i][cc]);
        const int e = e0 + cc;
        if (lane == 0 && e < e_end) partial[(int64_t(wave) * NE + i) * n_edges + e] += v;
      }
  }
}

// Far path (mixed form): pairs with r >= U_BIG / k_0, k_0 > 0, so every edge
// is on the large-argument side; accumulates (c_l / r^3) Dt_l(k_e r).  Chunk j
// covers edges [j CH, (j+1) CH) and evaluates all CH of them without branches
// (past the last edge it repeats the last edge and discards the result).  The
// sine/cosine table and the edges' (k, 1/k) are staged in LDS; the next pair's
// values are loaded one iteration ahead (the last iteration reloads its own
// pair) and each edge's (k, 1/k) one edge ahead.
template <int NE, int CH, bool FP64>
__global__ __launch_bounds__(kSweepBlock) __attribute__((amdgpu_waves_per_eu(HIPSTER_PK_WAVES_PER_EU))) void k_pk_far(
    const double *__restrict__ pr, const double *__restrict__ pmu, const double *__restrict__ pww, int64_t npairs,
    double inv_r0, const double *__restrict__ ek, int n_edges, double *__restrict__ partial) {
  __shared__ double2 tab[kSinCosTab];
  __shared__ double2 ekk[kMaxNk + 1];
  stage_sincos_tab<kSinCosTab>(tab);
  for (int i = threadIdx.x; i < n_edges; i += kSweepBlock) ekk[i] = make_double2(ek[i], ek[n_edges + i]);
  __syncthreads();
  const int64_t gtid = int64_t(blockIdx.x) * kSweepBlock + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * kSweepBlock;
  const int wave = int(gtid >> 6), lane = threadIdx.x & 63;
  for (int e0 = 0; e0 < n_edges; e0 += CH) {
    const int e_end = e0 + CH < n_edges ? e0 + CH : n_edges;
    double acc[NE][CH];
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) acc[i][cc] = 0.0;
    int64_t p = gtid;
    double r_n = 0.0, mu_n = 0.0, ww_n = 0.0;
    if (p < npairs) r_n = pr[p], mu_n = pmu[p], ww_n = pww[p];
    for (; p < npairs; p += stride) {
      const double r = r_n, mu = mu_n, ww = ww_n;
      const int64_t q = p + stride < npairs ? p + stride : p;
      r_n = pr[q], mu_n = pmu[q], ww_n = pww[q];
      double cf[NE];
      pair_coeffs<NE>(r, mu, ww, inv_r0, cf);
      const double inv_r = 1.0 / r;
      const double ir3 = inv_r * inv_r * inv_r;
#pragma unroll
      for (int i = 0; i < NE; ++i) cf[i] *= ir3;
      double2 kk = ekk[e0];
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) {
        const double2 kc = kk;
        const int en = e0 + cc + 1 < e_end ? e0 + cc + 1 : e_end - 1;
        kk = ekk[en];
        const Gv<double, NE> D = Dt_far<NE, 2, FP64>(kc.x * r, kc.y * inv_r, tab);
#pragma unroll
        for (int i = 0; i < NE; ++i) acc[i][cc] = fma(cf[i], D.v[i], acc[i][cc]);
      }
    }
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) {
        const double v = wave_sum(acc[i][cc]);
        const int e = e0 + cc;
        if (lane == 0 && e < e_end) partial[(int64_t(wave) * NE + i) * n_edges + e] += v;
      }
  }
}

int pk_sweep_waves(Ctx &c) {
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c.device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  return cus * 16;  // 4 blocks of 4 waves per CU
}

// Chunk size of the far path for n_edges edges from the compiled sizes: the
// fewest padded edge evaluations plus about three edges' worth of set-up per
// pair and chunk.
static int pick_chunk(const int (&sizes)[3], int n_edges) {
  int best = sizes[0];
  long best_cost = -1;
  for (int ch : sizes) {
    const long nchunk = (n_edges + ch - 1) / ch, cost = nchunk * (ch + 3);
    if (best_cost < 0 || cost < best_cost) best = ch, best_cost = cost;
  }
  return best;
}

template <int NE>
static void launch_general(Ctx &c, const PkPairs &p, int64_t npairs, bool fp64, double inv_r0, const double *ek,
                           int n_edges, double *partial, int nwaves) {
  const dim3 grid(unsigned(nwaves / 4)), block(kSweepBlock);
  const double *mu = static_cast<const double *>(p.mu), *ww = static_cast<const double *>(p.ww);
  if (fp64)
    k_pk_sweep<NE, true, kChunkFp64><<<grid, block, 0, c.stream>>>(p.r, mu, ww, npairs, inv_r0, ek, n_edges, partial);
  else
    k_pk_sweep<NE, false, kChunkNear><<<grid, block, 0, c.stream>>>(p.r, mu, ww, npairs, inv_r0, ek, n_edges, partial);
  HIPSTER_HIP(hipGetLastError());
}

template <int NE, int CH>
static void launch_far_ch(Ctx &c, const PkPairs &p, int64_t npairs, bool fp64, double inv_r0, const double *ek,
                          int n_edges, double *partial, int nwaves) {
  const double *mu = static_cast<const double *>(p.mu), *ww = static_cast<const double *>(p.ww);
  const dim3 grid(unsigned(nwaves / 4)), block(kSweepBlock);
  if (fp64)
    k_pk_far<NE, CH, true><<<grid, block, 0, c.stream>>>(p.r, mu, ww, npairs, inv_r0, ek, n_edges, partial);
  else
    k_pk_far<NE, CH, false><<<grid, block, 0, c.stream>>>(p.r, mu, ww, npairs, inv_r0, ek, n_edges, partial);
  HIPSTER_HIP(hipGetLastError());
}

template <int NE>
static void launch_far_any(Ctx &c, int ch, const PkPairs &p, int64_t npairs, bool fp64, double inv_r0,
                           const double *ek, int n_edges, double *partial, int nwaves) {
  constexpr bool four = NE >= 4;
  constexpr int c0 = four ? kChunksMixed4[0] : kChunksMixed3[0];
  constexpr int c1 = four ? kChunksMixed4[1] : kChunksMixed3[1];
  if (ch == c0) launch_far_ch<NE, c0>(c, p, npairs, fp64, inv_r0, ek, n_edges, partial, nwaves);
  else if (ch == c1) launch_far_ch<NE, c1>(c, p, npairs, fp64, inv_r0, ek, n_edges, partial, nwaves);
  else launch_far_ch<NE, (four ? kChunksMixed4[2] : kChunksMixed3[2])>(c, p, npairs, fp64, inv_r0, ek, n_edges,
                                                                        partial, nwaves);
}

// Edge-chunk size of the far kernel, measured.  The first sweep of a shape
// (multipoles, edges, form) with at least kTunePairs pairs times each
// compiled size on the first kTunePairs pairs into a scratch row set (two
// runs each, the faster counted) and keeps the fastest in the context, and
// in the file named by HIPSTER_TUNE_CACHE if set (one line per shape, keyed
// by the device).  Smaller sweeps, and sweeps in workspace mode (which
// creates no events), use the cost model of pick_chunk.  The
// chunk size does not change any sum (each edge adds the same pairs in the
// same order), so the choice affects time only.
constexpr int64_t kTunePairs = int64_t(1) << 22;

template <int NE>
static int tuned_chunk(Ctx &c, const PkPairs &p, int64_t npairs, bool fp64, double inv_r0, const double *ek,
                       int n_edges, int nwaves) {
  constexpr bool four = NE >= 4;
  const int(&sizes)[3] = four ? kChunksMixed4 : kChunksMixed3;
  const std::string key = tune_key(c, "pk_far", {NE, n_edges, fp64 ? 1 : 0});
  const int known = tune_lookup(c, key);
  if (known > 0) return known;
  if (npairs < kTunePairs || c.arena) return pick_chunk(sizes, n_edges);
  const size_t rows = size_t(nwaves) * NE * n_edges;
  double *scratch = static_cast<double *>(ensure(c, c.tune_scratch, rows * 8));
  hipEvent_t e0, e1;
  HIPSTER_HIP(hipEventCreate(&e0));
  HIPSTER_HIP(hipEventCreate(&e1));
  int best = pick_chunk(sizes, n_edges);
  float best_ms = -1.0f;
  for (int ch : sizes) {
    float ms_min = -1.0f;
    for (int rep = 0; rep < 2; ++rep) {
      HIPSTER_HIP(hipMemsetAsync(scratch, 0, rows * 8, c.stream));
      HIPSTER_HIP(hipEventRecord(e0, c.stream));
      launch_far_any<NE>(c, ch, p, kTunePairs, fp64, inv_r0, ek, n_edges, scratch, nwaves);
      HIPSTER_HIP(hipEventRecord(e1, c.stream));
      HIPSTER_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPSTER_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms_min < 0.0f || ms < ms_min) ms_min = ms;
    }
    if (best_ms < 0.0f || ms_min < best_ms) best = ch, best_ms = ms_min;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tune_store(c, key, best);
  return best;
}

template <int NE>
static void launch_far(Ctx &c, const PkPairs &p, int64_t npairs, bool fp64, double inv_r0, const double *ek,
                       int n_edges, double *partial, int nwaves) {
  const int ch = tuned_chunk<NE>(c, p, npairs, fp64, inv_r0, ek, n_edges, nwaves);
  launch_far_any<NE>(c, ch, p, npairs, fp64, inv_r0, ek, n_edges, partial, nwaves);
}

void pk_sweep_general(Ctx &c, const PkPairs &p, int64_t npairs, int n_ell, bool fp64, double r0, const double *ek,
                      int n_edges, double *partial, int nwaves) {
  if (npairs <= 0) return;
  if (n_edges < 1 || n_edges > kMaxNk + 1) throw Error{HIPSTER_EINVAL, "sweep: edge count out of range"};
  const double inv = 1.0 / r0;
  switch (n_ell) {
    case 1: launch_general<1>(c, p, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
    case 2: launch_general<2>(c, p, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
    case 3: launch_general<3>(c, p, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
    default: launch_general<4>(c, p, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
  }
}

void pk_sweep_far(Ctx &c, const PkPairs &p, int64_t npairs, int n_ell, bool fp64, double r0, const double *ek,
                  int n_edges, double *partial, int nwaves) {
  if (npairs <= 0) return;
  if (n_edges < 1 || n_edges > kMaxNk + 1) throw Error{HIPSTER_EINVAL, "sweep: edge count out of range"};
  const double inv = 1.0 / r0;
  switch (n_ell) {
    case 1: launch_far<1>(c, p, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
    case 2: launch_far<2>(c, p, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
    case 3: launch_far<3>(c, p, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
    default: launch_far<4>(c, p, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
  }
}

// out[col] = sum over rows of partial[row][col], summed in a fixed order.
__global__ __launch_bounds__(256) void k_merge(const double *__restrict__ partial, int rows, int cols,
                                               double *__restrict__ out) {
  __shared__ double sh[256];
  const int col = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int r = t; r < rows; r += 256) s += partial[int64_t(r) * cols + col];
  sh[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) out[col] = sh[0];
}

void merge_partials(Ctx &c, const double *partial, int rows, int cols, double *out) {
  k_merge<<<dim3(unsigned(cols)), dim3(256), 0, c.stream>>>(partial, rows, cols, out);
  HIPSTER_HIP(hipGetLastError());
}

}  // namespace hipster

namespace hipster {

// ------------------------------------------------- batched work-queue sweep
// Many boxes' pair streams concatenated into one; the stream is cut into
// tasks (box, [begin, end)) of at most kTaskPairs pairs, ordered largest box
// first.  A persistent grid of waves pulls tasks from an atomic counter until
// the queue is empty (every wave reaches that exit), and each task writes its
// own row of edge sums, so the merge per box is in task order and the result
// does not depend on which wave took which task.
template <int NE, bool FP64>
__global__ __launch_bounds__(kSweepBlock) void k_pk_tasks(const double *__restrict__ pr, const double *__restrict__ pmu,
                                                          const double *__restrict__ pww,
                                                          const PkTask *__restrict__ tasks, int ntasks,
                                                          int *__restrict__ counter, const double *__restrict__ edges_all,
                                                          const BoxSweep *__restrict__ boxes, int cols,
                                                          double *__restrict__ rows) {
  const int lane = threadIdx.x & 63;
  __shared__ double2 tab[FP64 ? 1 : kSinCosTab];
  if constexpr (!FP64) {
    stage_sincos_tab<kSinCosTab>(tab);
    __syncthreads();
  }
  for (;;) {
    int t = 0;
    if (lane == 0) t = atomicAdd(counter, 1);
    t = __shfl(t, 0);
    if (t >= ntasks) break;
    const PkTask task = tasks[t];
    const BoxSweep bx = boxes[task.box];
    const double *edges = edges_all + bx.edge_off;
    const int n_edges = bx.n_edges;
    double *row = rows + int64_t(t) * cols;
    const int nchunk = (n_edges + kChunk - 1) / kChunk, per = (n_edges + nchunk - 1) / nchunk;
    for (int e0 = 0; e0 < n_edges; e0 += per) {
      const int e_end = e0 + per < n_edges ? e0 + per : n_edges;
      double acc[NE][kChunk];
#pragma unroll
      for (int i = 0; i < NE; ++i)
#pragma unroll
        for (int cc = 0; cc < kChunk; ++cc) acc[i][cc] = 0.0;
      for (int64_t p = task.begin + lane; p < task.end; p += 64) {
        const double r = pr[p];
        const double wt = pww[p] * window<double>(r * bx.inv_r0);
        double L[NE];
        legendre_even<double, NE>(pmu[p], L);
        double cf[NE];
#pragma unroll
        for (int i = 0; i < NE; ++i) cf[i] = wt * L[i];
#pragma unroll
        for (int cc = 0; cc < kChunk; ++cc) {
          const int e = e0 + cc;
          if (e < e_end) {
            const double u = edges[e] * r;
            Gv<double, NE> G;
            if constexpr (FP64) G = G_fp64<NE, 2, true>(u);
            else G = G_mixed<NE, 2, false>(u, tab);  // inline Taylor would cost this kernel an occupancy level
#pragma unroll
            for (int i = 0; i < NE; ++i) acc[i][cc] = fma(cf[i], G.v[i], acc[i][cc]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < NE; ++i)
#pragma unroll
        for (int cc = 0; cc < kChunk; ++cc) {
          const double v = wave_sum(acc[i][cc]);
          const int e = e0 + cc;
          if (lane == 0 && e < e_end) row[i * n_edges + e] = v;
        }
    }
  }
}

template <int NE>
static void launch_tasks(Ctx &c, const PkPairs &p, const PkTask *tasks, int ntasks, int *counter, const double *edges,
                         const BoxSweep *boxes, int cols, double *rows, bool fp64, int nwaves) {
  const dim3 grid(unsigned(nwaves / 4)), block(kSweepBlock);
  const double *mu = static_cast<const double *>(p.mu), *ww = static_cast<const double *>(p.ww);
  if (fp64)
    k_pk_tasks<NE, true><<<grid, block, 0, c.stream>>>(p.r, mu, ww, tasks, ntasks, counter, edges, boxes, cols, rows);
  else
    k_pk_tasks<NE, false><<<grid, block, 0, c.stream>>>(p.r, mu, ww, tasks, ntasks, counter, edges, boxes, cols, rows);
  HIPSTER_HIP(hipGetLastError());
}

void pk_sweep_tasks(Ctx &c, const PkPairs &p, const PkTask *tasks, int ntasks, int *counter, const double *edges,
                    const BoxSweep *boxes, int cols, double *rows, int n_ell, bool fp64, int nwaves) {
  switch (n_ell) {
    case 1: launch_tasks<1>(c, p, tasks, ntasks, counter, edges, boxes, cols, rows, fp64, nwaves); break;
    case 2: launch_tasks<2>(c, p, tasks, ntasks, counter, edges, boxes, cols, rows, fp64, nwaves); break;
    case 3: launch_tasks<3>(c, p, tasks, ntasks, counter, edges, boxes, cols, rows, fp64, nwaves); break;
    default: launch_tasks<4>(c, p, tasks, ntasks, counter, edges, boxes, cols, rows, fp64, nwaves); break;
  }
}

// out[b][col] += sum of rows[t][col] over the tasks t of box b, in task order;
// box b's rows are the consecutive range [range[2b], range[2b+1]).
__global__ __launch_bounds__(256) void k_merge_boxes(const double *__restrict__ rows, int cols,
                                                     const int *__restrict__ range, double *__restrict__ out) {
  const int b = blockIdx.y;
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= cols) return;
  double s = 0.0;
  for (int t = range[2 * b]; t < range[2 * b + 1]; ++t) s += rows[int64_t(t) * cols + col];
  out[int64_t(b) * cols + col] += s;
}

void merge_boxes(Ctx &c, const double *rows, int cols, const int *first, int nboxes, double *out) {
  k_merge_boxes<<<dim3(unsigned((cols + 255) / 256), unsigned(nboxes)), dim3(256), 0, c.stream>>>(rows, cols, first, out);
  HIPSTER_HIP(hipGetLastError());
}

}  // namespace hipster

namespace hipster {

// ------------------------------------------------------------- L1 mass
// sum over the stream's pairs of |ww| W(r/R0) (2l+1) |L_l(mu)| |jbar^a_l(r)|,
// l = 0, 2, .., in double precision (G_fp64 per edge), bins in chunks of 8
// with one pass over the pairs per chunk; wave sums added to the wave's row.
template <int NE>
__global__ __launch_bounds__(256) void k_pk_l1(const double *__restrict__ pr, const double *__restrict__ pmu,
                                               const double *__restrict__ pww, int64_t n, double inv_r0,
                                               const double *__restrict__ ek, int n_edges,
                                               double *__restrict__ rows) {
  constexpr int kB = 8;
  const int n_k = n_edges - 1;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const double *k = ek, *k3 = ek + 2 * n_edges;
  for (int a0 = 0; a0 < n_k; a0 += kB) {
    double acc[NE][kB];
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int b = 0; b < kB; ++b) acc[i][b] = 0.0;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride) {
      const double r = pr[p];
      const double wt = fabs(pww[p]) * window<double>(r * inv_r0);
      double L[NE];
      legendre_even<double, NE>(pmu[p], L);
      Gv<double, NE> prev = G_fp64<NE, 2>(k[a0] * r);
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        const int a = a0 + b;
        if (a < n_k) {
          const Gv<double, NE> cur = G_fp64<NE, 2>(k[a + 1] * r);
          const double cf = 3.0 / (k3[a + 1] - k3[a]);
#pragma unroll
          for (int i = 0; i < NE; ++i)
            acc[i][b] += wt * double(4 * i + 1) * fabs(L[i]) * fabs(cf * (k3[a + 1] * cur.v[i] - k3[a] * prev.v[i]));
          prev = cur;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        const double v = wave_sum(acc[i][b]);
        if (lane == 0 && a0 + b < n_k) rows[(wave * NE + i) * n_k + a0 + b] += v;
      }
  }
}

void pk_l1_sweep(Ctx &c, const PkPairs &p, int64_t npairs, int n_ell, double r0, const double *edges, int n_edges,
                 double *rows, int nwaves) {
  if (npairs <= 0) return;
  const dim3 grid(unsigned(nwaves / 4)), block(256);
  const double *mu = static_cast<const double *>(p.mu), *ww = static_cast<const double *>(p.ww);
  switch (n_ell) {
    case 1: k_pk_l1<1><<<grid, block, 0, c.stream>>>(p.r, mu, ww, npairs, 1.0 / r0, edges, n_edges, rows); break;
    case 2: k_pk_l1<2><<<grid, block, 0, c.stream>>>(p.r, mu, ww, npairs, 1.0 / r0, edges, n_edges, rows); break;
    case 3: k_pk_l1<3><<<grid, block, 0, c.stream>>>(p.r, mu, ww, npairs, 1.0 / r0, edges, n_edges, rows); break;
    default: k_pk_l1<4><<<grid, block, 0, c.stream>>>(p.r, mu, ww, npairs, 1.0 / r0, edges, n_edges, rows); break;
  }
  HIPSTER_HIP(hipGetLastError());
}

}  // namespace hipster
