// Device-built cell list: every point is assigned to a cubic cell of side
// L / n_c > R0 (of the periodic box, or of a survey's bounding cube), points
// are sorted by cell with a stable radix sort (ties in original index order,
// so the layout -- and every sum over it -- is deterministic), and the
// coordinates are gathered into coalesced structure-of-arrays in double
// precision.  Memory-bound; a few passes over ~40 bytes per point.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace hipster {

static int cells_per_axis(double L, double r0) {
  int nc = int(floor(L / r0));
  // Keep the cell side clear of R0 by a margin far above the rounding of the
  // cell assignment, so a pair inside R0 always lies in neighbouring cells.
  while (nc > 1 && L / nc < r0 * (1.0 + 1e-6)) --nc;
  if (nc < 1) nc = 1;
  if (nc > kMaxCellsPerAxis) nc = kMaxCellsPerAxis;
  return nc;
}

Grid make_grid(double L, double r0) {
  const int nc = cells_per_axis(L, r0);
  return Grid{nc, L, double(nc) / L};
}

Grid make_survey_grid(const double lo[3], const double hi[3], double r0) {
  double ext = 0.0;
  for (int d = 0; d < 3; ++d) ext = fmax(ext, hi[d] - lo[d]);
  // the cube [lo, lo + L) must hold the largest coordinate strictly inside
  const double L = ext * (1.0 + 1e-9) + 1e-9 * fmax(1.0, r0);
  const int nc = cells_per_axis(L, r0);
  Grid g{nc, L, double(nc) / L};
  g.ox = lo[0];
  g.oy = lo[1];
  g.oz = lo[2];
  g.periodic = false;
  return g;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bbox(const T *__restrict__ pos, int64_t n, double *__restrict__ out,
                                              int *__restrict__ bad) {
  __shared__ double sh[6][256];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  bool finite = true;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    for (int d = 0; d < 3; ++d) {
      const double x = double(pos[3 * i + d]);
      finite = finite && isfinite(x);
      v[d] = fmin(v[d], x);
      v[3 + d] = fmax(v[3 + d], x);
    }
  if (!finite) atomicOr(bad, 1);
  for (int d = 0; d < 6; ++d) sh[d][threadIdx.x] = v[d];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o)
      for (int d = 0; d < 6; ++d)
        sh[d][threadIdx.x] = d < 3 ? fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + o])
                                   : fmax(sh[d][threadIdx.x], sh[d][threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int d = 0; d < 6; ++d) out[blockIdx.x * 6 + d] = sh[d][0];
}

void bounding_box(Ctx &c, const void *pos, int64_t n, int dtype, double lo[3], double hi[3]) {
  if (n <= 0) return;
  const int nb = int(std::min<int64_t>(1024, (n + 255) / 256));
  double *out = static_cast<double *>(ensure(c, c.bbox, size_t(nb) * 6 * 8 + 64));
  int *bad = reinterpret_cast<int *>(out + size_t(nb) * 6);
  HIPSTER_HIP(hipMemsetAsync(bad, 0, sizeof(int), c.stream));
  if (dtype == HIPSTER_F32)
    k_bbox<float><<<dim3(unsigned(nb)), 256, 0, c.stream>>>(static_cast<const float *>(pos), n, out, bad);
  else
    k_bbox<double><<<dim3(unsigned(nb)), 256, 0, c.stream>>>(static_cast<const double *>(pos), n, out, bad);
  HIPSTER_HIP(hipGetLastError());
  std::vector<double> h(size_t(nb) * 6 + 8);
  HIPSTER_HIP(hipMemcpyAsync(h.data(), out, (size_t(nb) * 6 + 1) * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  int hbad = 0;
  memcpy(&hbad, h.data() + size_t(nb) * 6, sizeof(int));
  if (hbad) throw Error{HIPSTER_EOUTOFBOX, "a coordinate is not finite"};
  for (int b = 0; b < nb; ++b)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], h[size_t(b) * 6 + d]);
      hi[d] = fmax(hi[d], h[size_t(b) * 6 + 3 + d]);
    }
}

// Cell of each point of [o, o + L)^3; a point outside (or not finite) sets
// *bad.  The sorted coordinates keep the input values, so pair separations
// are differences of the inputs, as in the definition.
template <typename T>
__global__ void k_assign(const T *__restrict__ pos, int64_t n, double L, int nc, double scale, double ox, double oy,
                         double oz, int *__restrict__ cell, int *__restrict__ count, int *__restrict__ bad) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = double(pos[3 * i]) - ox, y = double(pos[3 * i + 1]) - oy, z = double(pos[3 * i + 2]) - oz;
  bool ok = (x >= 0.0) && (x < L) && (y >= 0.0) && (y < L) && (z >= 0.0) && (z < L);
  if (!ok) {
    atomicOr(bad, 1);
    cell[i] = -1;
    return;
  }
  int cx = min(int(x * scale), nc - 1), cy = min(int(y * scale), nc - 1), cz = min(int(z * scale), nc - 1);
  int c = (cx * nc + cy) * nc + cz;
  cell[i] = c;
  atomicAdd(&count[c], 1);
}

__global__ void k_widen(const int *__restrict__ in, int64_t *__restrict__ out, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

__global__ void k_iota(int *__restrict__ v, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) v[i] = int(i);
}

template <typename T>
__global__ void k_gather(const T *__restrict__ pos, const T *__restrict__ w, const uint8_t *__restrict__ mask,
                         const int *__restrict__ idx, int64_t n, double *__restrict__ x, double *__restrict__ y,
                         double *__restrict__ z, double *__restrict__ ws, uint8_t *__restrict__ ms) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int i = idx[k];
  x[k] = double(pos[3 * int64_t(i)]);
  y[k] = double(pos[3 * int64_t(i) + 1]);
  z[k] = double(pos[3 * int64_t(i) + 2]);
  ws[k] = w ? double(w[i]) : 1.0;
  if (ms) ms[k] = mask[i] ? 1 : 0;
}

// Philox4x64-10 (Salmon, Moraes, Dror and Shaw 2011, "Parallel random numbers:
// as easy as 1, 2, 3"): ten rounds of two 64 x 64 -> 128-bit products of the
// counter words with the round multipliers, the high halves mixed into the
// other words with the key, the key bumped by the Weyl constants between
// rounds.
__device__ inline void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, c[0]), lo0 = kM0 * c[0];
    const uint64_t hi1 = __umul64hi(kM1, c[2]), lo1 = kM1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ __launch_bounds__(256) void k_random_points(uint64_t seed, int64_t n, double L, double *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  uint64_t c[4] = {uint64_t(i) + 1, 0, 0, 0};
  philox4x64_10(c, seed, 0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double x = L * (double(c[d] >> 11) * 0x1.0p-53);
    if (x >= L) x = 0.0;
    out[3 * i + d] = x;
  }
}

void random_points(Ctx &c, uint64_t seed, int64_t n, double L, double *out) {
  if (n <= 0) return;
  k_random_points<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, c.stream>>>(seed, n, L, out);
  HIPSTER_HIP(hipGetLastError());
}

void widen_i32(Ctx &c, const int *in, int64_t *out, int64_t n) {
  if (n <= 0) return;
  k_widen<<<dim3(unsigned((n + 255) / 256)), 256, 0, c.stream>>>(in, out, n);
  HIPSTER_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- scan
constexpr int kScanBlock = 256, kScanItems = 4, kScanTile = kScanBlock * kScanItems;

__global__ __launch_bounds__(256) void k_scan_tile(const int64_t *__restrict__ in, int64_t *__restrict__ out,
                                                   int64_t *__restrict__ sums, int64_t n) {
  __shared__ int64_t sh[kScanBlock];
  const int t = threadIdx.x;
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(t) * kScanItems;
  int64_t v[kScanItems], tot = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    tot += v[k];
  }
  sh[t] = tot;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int64_t add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t run = sh[t] - tot;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (t == kScanBlock - 1) sums[blockIdx.x] = sh[t];
}

__global__ void k_scan_add(int64_t *__restrict__ out, const int64_t *__restrict__ offs, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i / kScanTile];
}

__global__ void k_scan_total(const int64_t *__restrict__ in, int64_t *__restrict__ out, int64_t n) {
  out[n] = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

static void scan_rec(Ctx &c, const int64_t *in, int64_t *out, int64_t n, int64_t *tmp) {
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) return;
  int64_t *sums = tmp, *sums_scan = tmp + nb;
  k_scan_tile<<<dim3(unsigned(nb)), dim3(kScanBlock), 0, c.stream>>>(in, out, sums, n);
  if (nb > 1) {
    scan_rec(c, sums, sums_scan, nb, tmp + 2 * nb);
    k_scan_add<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, c.stream>>>(out, sums_scan, n);
  }
}

void scan_i64(Ctx &c, const int64_t *in, int64_t *out, int64_t n, DevBuf &tmpb) {
  int64_t need = 0, m = n;
  while (m > 1) {
    m = (m + kScanTile - 1) / kScanTile;
    need += 2 * m + 2;
  }
  int64_t *tmp = static_cast<int64_t *>(ensure(c, tmpb, size_t(need + 8) * sizeof(int64_t)));
  scan_rec(c, in, out, n, tmp);
  k_scan_total<<<1, 1, 0, c.stream>>>(in, out, n);
  HIPSTER_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- driver
template <typename T>
static Sorted build_cells_t(Ctx &c, CellScratch &s, const Grid &g, const T *pos, const T *w,
                            const uint8_t *mask_dev, int64_t n) {
  const int64_t ncells = g.ncells();
  int *cell = static_cast<int *>(ensure(c, s.cell, size_t(n) * sizeof(int)));
  int *count = static_cast<int *>(ensure(c, s.count, size_t(ncells) * sizeof(int)));
  int64_t *start = static_cast<int64_t *>(ensure(c, s.start, size_t(2 * ncells + 2) * sizeof(int64_t)));
  int64_t *wide = start + ncells + 1;
  int *iota = static_cast<int *>(ensure(c, s.cursor, size_t(n) * sizeof(int)));
  int *idx = static_cast<int *>(ensure(c, s.idx, size_t(n) * sizeof(int)));
  double *x = static_cast<double *>(ensure(c, s.x, size_t(n) * sizeof(double)));
  double *y = static_cast<double *>(ensure(c, s.y, size_t(n) * sizeof(double)));
  double *z = static_cast<double *>(ensure(c, s.z, size_t(n) * sizeof(double)));
  double *ws = static_cast<double *>(ensure(c, s.w, size_t(n) * sizeof(double)));
  uint8_t *ms = mask_dev ? static_cast<uint8_t *>(ensure(c, s.m, size_t(n))) : nullptr;
  int *scell = static_cast<int *>(ensure(c, s.scell, size_t(n) * sizeof(int)));
  int *bad = static_cast<int *>(ensure(c, s.bad, sizeof(int) * 4));

  HIPSTER_HIP(hipMemsetAsync(count, 0, size_t(ncells) * sizeof(int), c.stream));
  if (n == 0) {
    HIPSTER_HIP(hipMemsetAsync(start, 0, size_t(ncells + 1) * sizeof(int64_t), c.stream));
    Sorted out;
    out.n = 0;
    out.x = x;
    out.y = y;
    out.z = z;
    out.w = ws;
    out.m = ms;
    out.cell_start = start;
    out.scell = scell;
    return out;
  }
  HIPSTER_HIP(hipMemsetAsync(bad, 0, sizeof(int), c.stream));
  const unsigned nbp = unsigned((n + 255) / 256), nbc = unsigned((ncells + 255) / 256);
  k_assign<T><<<nbp, 256, 0, c.stream>>>(pos, n, g.L, g.nc, g.scale, g.ox, g.oy, g.oz, cell, count, bad);
  int hbad = 0;
  HIPSTER_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  if (hbad) throw Error{HIPSTER_EOUTOFBOX, g.periodic ? "a coordinate is not finite or outside [0, L)"
                                                     : "a coordinate is not finite or outside the survey grid"};
  k_widen<<<nbc, 256, 0, c.stream>>>(count, wide, ncells);
  scan_i64(c, wide, start, ncells, s.scan_tmp);
  // (cell, index) pairs in cell order, each cell's points in input order: a
  // stable LSD radix sort of the cell ids with the point indices as values
  // (deterministic, O(n) whatever the points per cell); the sorted keys are
  // the per-point cell ids of the sorted arrays
  k_iota<<<nbp, 256, 0, c.stream>>>(iota, n);
  int bits = 1;
  while (bits < 31 && (int64_t(1) << bits) < ncells) ++bits;
  size_t tmp_bytes = 0;
  HIPSTER_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, cell, scell, iota, idx, int(n), 0, bits,
                                                 c.stream));
  void *tmp = ensure(c, s.sort_tmp, std::max<size_t>(tmp_bytes, 16));
  HIPSTER_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, cell, scell, iota, idx, int(n), 0, bits,
                                                 c.stream));
  k_gather<T><<<nbp, 256, 0, c.stream>>>(pos, w, mask_dev, idx, n, x, y, z, ws, ms);
  HIPSTER_HIP(hipGetLastError());
  Sorted out;
  out.n = n;
  out.x = x;
  out.y = y;
  out.z = z;
  out.w = ws;
  out.m = ms;
  out.cell_start = start;
  out.scell = scell;
  return out;
}

// Neighbour count of each selected sorted primary: the secondaries within R0
// in the 27 cells around its home cell, tested in single precision (the
// count only orders the primaries inside a cell, so a pair at the boundary
// may go either way without harm).  One wave per 64 consecutive primaries:
// the wave takes the distinct home cells of its lanes one at a time and
// stages that cell's candidates through LDS, 64 at a time; the lanes of the
// cell test every staged candidate.
__global__ __launch_bounds__(64) void k_nb_count(Sorted prim, Sorted sec, int nc, double L, float r02, int self_set,
                                                 int *__restrict__ cnt) {
  __shared__ float4 cand[64];
  const int lane = threadIdx.x;
  const int64_t p = int64_t(blockIdx.x) * 64 + lane;
  const bool valid = p < prim.n && (prim.m == nullptr || prim.m[p] != 0);
  const int my_cell = valid ? prim.scell[p] : -1;
  float px = 0.0f, py = 0.0f, pz = 0.0f;
  if (valid) {
    px = float(prim.x[p]);
    py = float(prim.y[p]);
    pz = float(prim.z[p]);
  }
  int count = 0;
  bool done = !valid;
  for (;;) {
    const unsigned long long pend = __ballot(!done);
    if (pend == 0) break;
    const int first = __ffsll((long long)pend) - 1;
    const int cell = __builtin_amdgcn_readfirstlane(__shfl(my_cell, first));
    const bool mine = !done && my_cell == cell;
    const int cz = cell % nc, cy = (cell / nc) % nc, cx = cell / (nc * nc);
    for (int k = 0; k < 27; ++k) {
      int nx = cx + k / 9 - 1, ny = cy + (k / 3) % 3 - 1, nz = cz + k % 3 - 1;
      double ox = 0.0, oy = 0.0, oz = 0.0;
      if (nx >= nc) { nx -= nc; ox = L; } else if (nx < 0) { nx += nc; ox = -L; }
      if (ny >= nc) { ny -= nc; oy = L; } else if (ny < 0) { ny += nc; oy = -L; }
      if (nz >= nc) { nz -= nc; oz = L; } else if (nz < 0) { nz += nc; oz = -L; }
      const int64_t nb = (int64_t(nx) * nc + ny) * nc + nz;
      const int64_t b = sec.cell_start[nb], e = sec.cell_start[nb + 1];
      for (int64_t j0 = b; j0 < e; j0 += 64) {
        const int64_t j = j0 + lane;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (j < e) v = make_float4(float(sec.x[j] + ox), float(sec.y[j] + oy), float(sec.z[j] + oz), 0.0f);
        __syncthreads();
        cand[lane] = v;
        __syncthreads();
        if (mine) {
          const int n = int(e - j0 < 64 ? e - j0 : 64);
          for (int i = 0; i < n; ++i) {
            const float4 q = cand[i];
            const float dx = px - q.x, dy = py - q.y, dz = pz - q.z;
            count += dx * dx + dy * dy + dz * dz < r02 ? 1 : 0;
          }
        }
      }
    }
    if (mine) done = true;
  }
  if (valid) cnt[p] = self_set && count > 0 ? count - 1 : count;
}

// Sort key (home cell, neighbour count): selected primaries by count, the
// others after them in their cell.
constexpr int kNbCountBits = 20;
__global__ __launch_bounds__(256) void k_nb_key(const int *__restrict__ scell, const uint8_t *__restrict__ m,
                                                const int *__restrict__ cnt, int64_t n, uint64_t *__restrict__ key,
                                                int *__restrict__ iota) {
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= n) return;
  const int top = (1 << kNbCountBits) - 1;
  int v = top;
  if (m == nullptr || m[p] != 0) v = cnt[p] < 0 ? 0 : (cnt[p] < top - 1 ? cnt[p] : top - 1);
  key[p] = (uint64_t(unsigned(scell[p])) << kNbCountBits) | uint64_t(unsigned(v));
  iota[p] = int(p);
}

const int *order_by_neighbours(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0,
                               bool self_set) {
  const int64_t n = prim.n;
  if (n == 0) return nullptr;
  if (n >= (int64_t(1) << 31)) throw Error{HIPSTER_EUNSUPPORTED, "bispectrum: at most 2^31 - 1 primaries"};
  int *cnt = static_cast<int *>(ensure(c, c.bo_cnt, size_t(n) * sizeof(int)));
  uint64_t *key = static_cast<uint64_t *>(ensure(c, c.bo_key, size_t(n) * sizeof(uint64_t)));
  uint64_t *key2 = static_cast<uint64_t *>(ensure(c, c.bo_key2, size_t(n) * sizeof(uint64_t)));
  int *iota = static_cast<int *>(ensure(c, c.bo_iota, size_t(n) * sizeof(int)));
  int *perm = static_cast<int *>(ensure(c, c.bo_perm, size_t(n) * sizeof(int)));
  k_nb_count<<<dim3(unsigned((n + 63) / 64)), dim3(64), 0, c.stream>>>(prim, sec, g.nc, g.L, float(r0 * r0),
                                                                       self_set ? 1 : 0, cnt);
  HIPSTER_HIP(hipGetLastError());
  k_nb_key<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, c.stream>>>(prim.scell, prim.m, cnt, n, key, iota);
  HIPSTER_HIP(hipGetLastError());
  int cbits = 1;
  while (cbits < 40 && (int64_t(1) << cbits) < g.ncells()) ++cbits;
  const int bits = cbits + kNbCountBits;
  size_t tmp_bytes = 0;
  HIPSTER_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key, key2, iota, perm, int(n), 0, bits,
                                                 c.stream));
  void *tmp = ensure(c, c.bo_tmp, std::max<size_t>(tmp_bytes, 16));
  HIPSTER_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, key2, iota, perm, int(n), 0, bits, c.stream));
  return perm;
}

Sorted build_cells(Ctx &c, CellScratch &s, const Grid &g, const void *pos, const void *w,
                   const uint8_t *mask_dev, int64_t n, int dtype) {
  if (dtype == HIPSTER_F32)
    return build_cells_t<float>(c, s, g, static_cast<const float *>(pos), static_cast<const float *>(w), mask_dev, n);
  return build_cells_t<double>(c, s, g, static_cast<const double *>(pos), static_cast<const double *>(w), mask_dev, n);
}

}  // namespace hipster
