// Power-spectrum pair-weight sweep (the dominant cost; Sec. 9 of the paper
// names the Bessel weights the limiting step).
//
// For each unordered pair (r, mu, w_i w_j m_ij) and each bin edge k_e the
// single-box sweep adds c_l k_e^3 G_l(k_e r) to a per-lane double accumulator,
// with c_l = w_i w_j m_ij W(r/R0) L_l(mu).  The bin values follow on the host as
// S^a_l = 3 (2l+1) (-i)^l [E'_l(a+1) - E'_l(a)] / (k_{a+1}^3 - k_a^3),
// E'_l(e) = sum over pairs of c_l k_e^3 G_l(k_e r) (Sec. 3, binned estimator
// with eq. jla-def).  Since k^3 G_l(k r) = Dt_l(k r) / r^3, pairs of the far
// bucket (r >= U_BIG / k_0, so every edge is on the large-argument side)
// accumulate (c_l / r^3) Dt_l(k_e r) with no per-edge rescaling; pairs of the
// near bucket evaluate G_l and scale it by k_e^3.  Edges are processed in
// balanced chunks (SweepChunk edges at most) so the accumulators stay in
// registers; the pair stream is re-read once per chunk.  Each wave reduces its lanes with cross-lane shuffles and
// adds its sums to its own row of `partial`; rows are merged in a fixed order,
// so results are bitwise reproducible.
#include <type_traits>

#include "common.h"
#include "specfun.h"

namespace hipster {

constexpr int kSweepBlock = 256;
constexpr int kChunk = 8;  // batched sweep; single-box sweep: SweepChunk below

// Edges per chunk of the single-box sweep.  A larger chunk reads the pair
// stream fewer times and spreads each pair's set-up (window, Legendre, 1/r)
// over more edges, at the cost of registers: the mixed form has room for 21
// edges of up to three multipoles (two chunks for 41 edges, measured 12%
// faster than 8) and 14 of four; the FP64 form's longer special functions keep
// it at 8 (larger chunks measured slower).
template <bool FP64, int NE>
constexpr int SweepChunk = FP64 ? 8 : (NE <= 3 ? 21 : 14);

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
// n_edges each) followed by U_BIG / k_e as floats.  Pairs [0, n_near) take the
// general path; pairs [n_near, npairs) take the far path (the mixed form only;
// the host passes n_near = npairs otherwise).
template <int NE, bool FP64>
__global__ __launch_bounds__(kSweepBlock) __attribute__((amdgpu_waves_per_eu(HIPSTER_PK_WAVES_PER_EU))) void k_pk_sweep(
    const double *__restrict__ pr, const double *__restrict__ pmu, const double *__restrict__ pww, int64_t n_near,
    int64_t npairs, double inv_r0, const double *__restrict__ ek, int n_edges, double *__restrict__ partial) {
  __shared__ double2 tab[256];
  if (!FP64) {
    for (int i = threadIdx.x; i < 256; i += kSweepBlock) tab[i] = make_double2(SINCOS_TAB[i][0], SINCOS_TAB[i][1]);
    __syncthreads();
  }
  const double *k_e = ek, *inv_k = ek + n_edges, *k3 = ek + 2 * n_edges;
  const float *t_e = reinterpret_cast<const float *>(ek + 3 * n_edges);
  const int64_t gtid = int64_t(blockIdx.x) * kSweepBlock + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * kSweepBlock;
  const int wave = int(gtid >> 6), lane = threadIdx.x & 63;
  // balanced chunks of at most CH edges
  constexpr int CH = SweepChunk<FP64, NE>;
  const int nchunk = (n_edges + CH - 1) / CH, per = (n_edges + nchunk - 1) / nchunk;
  for (int e0 = 0; e0 < n_edges; e0 += per) {
    const int e_end = e0 + per < n_edges ? e0 + per : n_edges;
    double acc[NE][CH];
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) acc[i][cc] = 0.0;
    // near bucket (and every pair in the FP64 form): G_l(k_e r) k_e^3
    for (int64_t p = gtid; p < n_near; p += stride) {
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
          if constexpr (FP64) G = G_fp64<NE, 2>(u);
          else G = G_mixed_w<NE, 2>(u, inv_k[e] * inv_r);
          const double s3 = k3[e];
#pragma unroll
          for (int i = 0; i < NE; ++i) acc[i][cc] = fma(cf[i], G.v[i] * s3, acc[i][cc]);
        }
      }
    }
    if constexpr (!FP64) {
      // far bucket: (c_l / r^3) Dt_l(k_e r), every edge on the large-argument side
      for (int64_t p = n_near + gtid; p < npairs; p += stride) {
        const double r = pr[p];
        double cf[NE];
        pair_coeffs<NE>(r, pmu[p], pww[p], inv_r0, cf);
        const double inv_r = 1.0 / r;
        const double ir3 = inv_r * inv_r * inv_r;
#pragma unroll
        for (int i = 0; i < NE; ++i) cf[i] *= ir3;
        const float inv_rf = float(inv_r);
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) {
          const int e = e0 + cc;
          if (e < e_end) {
            const Gv<double, NE> D = Dt_far_mixed<NE, 2>(k_e[e] * r, inv_k[e] * inv_r, t_e[e] * inv_rf, tab);
#pragma unroll
            for (int i = 0; i < NE; ++i) acc[i][cc] = fma(cf[i], D.v[i], acc[i][cc]);
          }
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

int pk_sweep_waves(Ctx &c) {
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c.device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  return cus * 16;  // 4 blocks of 4 waves per CU
}

template <int NE>
static void launch_sweep(Ctx &c, const PkPairs &p, int64_t n_near, int64_t npairs, bool fp64, double inv_r0,
                         const double *ek, int n_edges, double *partial, int nwaves) {
  const dim3 grid(unsigned(nwaves / 4)), block(kSweepBlock);
  const double *mu = static_cast<const double *>(p.mu), *ww = static_cast<const double *>(p.ww);
  if (fp64)
    k_pk_sweep<NE, true><<<grid, block, 0, c.stream>>>(p.r, mu, ww, npairs, npairs, inv_r0, ek, n_edges, partial);
  else
    k_pk_sweep<NE, false><<<grid, block, 0, c.stream>>>(p.r, mu, ww, n_near, npairs, inv_r0, ek, n_edges, partial);
  HIPSTER_HIP(hipGetLastError());
}

int pk_sweep(Ctx &c, const PkPairs &p, int64_t n_near, int64_t npairs, int n_ell, bool fp64, double r0,
             const double *ek, int n_edges, double *partial, int nwaves) {
  if (n_near < 0 || n_near > npairs) throw Error{HIPSTER_EINVAL, "sweep: near-bucket size out of range"};
  const double inv = 1.0 / r0;
  switch (n_ell) {
    case 1: launch_sweep<1>(c, p, n_near, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
    case 2: launch_sweep<2>(c, p, n_near, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
    case 3: launch_sweep<3>(c, p, n_near, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
    default: launch_sweep<4>(c, p, n_near, npairs, fp64, inv, ek, n_edges, partial, nwaves); break;
  }
  return nwaves;
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
            if constexpr (FP64) G = G_fp64<NE, 2>(u);
            else G = G_mixed<NE, 2>(u);
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
