// Pair enumeration for the power spectrum: every unordered pair {i, j} inside
// R0 of a periodic box (or of a survey catalogue, or every pair between a
// survey's data and randoms, without periodicity) is found once by a half stencil of 14 cells (the home
// cell with i < j, and 13 forward neighbours with all i, j), each neighbour
// carrying its periodic image shift.  Pairs are compacted wave-by-wave
// (ballot + popcount) into a coalesced stream (r, mu, w_i w_j m_ij) in double
// precision, written in a deterministic order: a count pass sizes the output
// of each work unit (a home cell's tile of up to 64 points, one workgroup
// each, so a dense cell spreads over many workgroups), an exclusive scan gives
// offsets, and a write pass repeats the same tests.  The home tile and each
// neighbour are staged through LDS in tiles of 64 points, and a tile pair's
// candidates are packed 64 per step.
//
// Pairs are written in two buckets: r < r_split first, then the rest.  With
// r_split = u_switch / k_min no pair of the second bucket ever takes the
// small-argument (Taylor) branch of the pair weight, so the sweep's waves over
// that bucket -- most of the pairs -- never diverge into it.
//
// The separation is the paper's pair vector x_i - x_j at the periodic image
// inside R0 (Sec. 2 pair counts; Sec. 3 periodic box); its squared length is
// (dx^2 + dy^2) + dz^2 in double precision without contraction, the predicate
// that defines the integer pair count.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "specfun.h"

namespace hipster {

// Half stencil: (0,0,0) first, then the 13 offsets lexicographically after it.
__device__ inline void half_stencil(int s, int &ox, int &oy, int &oz) {
  if (s == 0) {
    ox = oy = oz = 0;
    return;
  }
  int t = s + 13;  // index in the 27-cell cube ordered (ox, oy, oz) in -1..1
  ox = t / 9 - 1;
  oy = (t / 3) % 3 - 1;
  oz = t % 3 - 1;
}

__device__ inline int wrap_axis(int v, int nc, int &shift) {
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

__device__ inline double sq_norm_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  double a = dx * dx;
  double b = dy * dy;
  double c = dz * dz;
  return (a + b) + c;
}

constexpr int kPairTile = 64;  // points of a cell staged in LDS at a time

// Enumeration modes: the periodic box (half stencil, image shifts, a fixed
// line-of-sight axis); a survey catalogue with itself (half stencil, no
// periodicity, midpoint line of sight); a survey catalogue against another
// (all 27 neighbours, every pair once).
enum PairMode { kPeriodic = 0, kSurveySelf = 1, kSurveyCross = 2 };

// One workgroup (one wave) per work unit: a home cell's tile of up to
// kPairTile points against the home cell and its stencil neighbours.  Units
// are ordered by home cell, then tile, so the stream order is the same for
// any number of units per launch, and a dense cell is spread over as many
// workgroups as it has tiles.
//
// Only ~1 candidate in 6 lies inside R0.  A single-precision prefilter, whose
// bound lim2f covers the rounding of the coordinates to float with a wide
// margin, passes candidates into a per-wave LDS queue (ballot + prefix
// count); the exact double-precision predicate, the bucket and the stream
// writes then run on 64 queued candidates at a time with every lane busy.
// The queue keeps candidate order, so the count and write passes see the
// same sequence.
template <bool WRITE, int MODE, bool MASKED>
__global__ __launch_bounds__(64) void k_pk_pairs(Sorted a, Sorted b, int nc, double L, double r02, float lim2f,
                                                 double rs2, int los, double scale, const int *__restrict__ unit_cell,
                                                 const int *__restrict__ unit_tile, int64_t u0,
                                                 int64_t *__restrict__ cnt_a, int64_t *__restrict__ cnt_b,
                                                 unsigned long long *__restrict__ ordered,
                                                 const int64_t *__restrict__ off_a, const int64_t *__restrict__ off_b,
                                                 int64_t base_a, int64_t base_b, int64_t n_a,
                                                 double *__restrict__ out_r, double *__restrict__ out_mu,
                                                 double *__restrict__ out_ww) {
  // home-cell and neighbour-cell tiles of kPairTile points in LDS; the
  // candidates of a tile pair are packed 64 to a step
  __shared__ double hx[kPairTile], hy[kPairTile], hz[kPairTile], hw[kPairTile];
  __shared__ double jx[kPairTile], jy[kPairTile], jz[kPairTile], jw[kPairTile];
  __shared__ int hm[kPairTile], jm[kPairTile];
  __shared__ float hxf[kPairTile], hyf[kPairTile], hzf[kPairTile], jxf[kPairTile], jyf[kPairTile], jzf[kPairTile];
  __shared__ int q_ii[128], q_jj[128];  // prefilter-passed candidates, in order
  constexpr int kStencil = MODE == kSurveyCross ? 27 : 14;
  const int64_t unit = u0 + blockIdx.x;
  const int64_t cell = unit_cell[unit];
  const int lane = threadIdx.x;
  const int cz = int(cell % nc), cy = int((cell / nc) % nc), cx = int(cell / (int64_t(nc) * nc));
  const int64_t hs = a.cell_start[cell];
  const int ni = int(a.cell_start[cell + 1] - hs);
  int64_t written_a = 0, written_b = 0;
  unsigned long long ord = 0;       // per lane, with masks
  unsigned long long ord_w = 0;     // per wave, without masks
  const int64_t wbase_a = WRITE ? off_a[unit] - base_a : 0;
  const int64_t wbase_b = WRITE ? n_a + off_b[unit] - base_b : 0;
  {
    const int i0 = unit_tile[unit] * kPairTile;
    const int ti = ni - i0 < kPairTile ? ni - i0 : kPairTile;
    if (lane < ti) {
      const int64_t i = hs + i0 + lane;
      hx[lane] = a.x[i];
      hy[lane] = a.y[i];
      hz[lane] = a.z[i];
      hw[lane] = a.w[i];
      hxf[lane] = float(a.x[i]);
      hyf[lane] = float(a.y[i]);
      hzf[lane] = float(a.z[i]);
      if (MASKED) hm[lane] = a.m ? int(a.m[i]) : 1;
    }
    for (int st = 0; st < kStencil; ++st) {
      int ox, oy, oz, sx = 0, sy = 0, sz = 0, nx, ny, nz;
      if (MODE == kSurveyCross) {
        ox = st / 9 - 1;
        oy = (st / 3) % 3 - 1;
        oz = st % 3 - 1;
      } else {
        half_stencil(st, ox, oy, oz);
      }
      if (MODE == kPeriodic) {
        nx = wrap_axis(cx + ox, nc, sx);
        ny = wrap_axis(cy + oy, nc, sy);
        nz = wrap_axis(cz + oz, nc, sz);
      } else {
        nx = cx + ox;
        ny = cy + oy;
        nz = cz + oz;
        if (nx < 0 || nx >= nc || ny < 0 || ny >= nc || nz < 0 || nz >= nc) continue;
      }
      // the neighbour image's offset s L (s = -1, 0, 1), uniform over the
      // stencil cell; (x_i - x_j) - s L is exact whenever the result lies
      // inside R0 <= L/2 (Sterbenz)
      const double offx = double(sx) * L, offy = double(sy) * L, offz = double(sz) * L;
      const int64_t nb = (int64_t(nx) * nc + ny) * nc + nz;
      const int64_t js = b.cell_start[nb];
      const int nj = int(b.cell_start[nb + 1] - js);
      const bool self = MODE != kSurveyCross && st == 0;
      // in the home cell only pairs j > i: tiles wholly below the home tile
      // hold none
      for (int j0 = self ? i0 : 0; j0 < nj; j0 += kPairTile) {
        const int tj = nj - j0 < kPairTile ? nj - j0 : kPairTile;
        __syncthreads();
        if (lane < tj) {
          const int64_t j = js + j0 + lane;
          jx[lane] = b.x[j];
          jy[lane] = b.y[j];
          jz[lane] = b.z[j];
          jw[lane] = b.w[j];
          // the neighbour image, rounded to float for the prefilter
          jxf[lane] = float(b.x[j] + offx);
          jyf[lane] = float(b.y[j] + offy);
          jzf[lane] = float(b.z[j] + offz);
          if (MASKED) jm[lane] = b.m ? int(b.m[j]) : 1;
        }
        __syncthreads();
        const uint32_t total = uint32_t(ti) * uint32_t(tj);
        // candidate q = ii * tj + jj of the tile pair; lanes advance by 64
        // candidates per step, i.e. by (64 / tj, 64 % tj) with a carry
        const uint32_t utj = uint32_t(tj), d64 = 64u / utj, r64 = 64u - d64 * utj;
        uint32_t ii = uint32_t(lane) / utj, jj = uint32_t(lane) - ii * utj;
        const unsigned long long below = (1ull << lane) - 1ull;
        int qn = 0;
        // the exact test of queued candidates [0, cnt) (lane e takes entry e),
        // then the buckets, the counts and (write pass) the stream
        auto process = [&](int cnt) {
          bool hit = false, near = false;
          double r = 0.0, mu = 0.0, ww = 0.0;
          if (lane < cnt) {
            const int ci = q_ii[lane], cj = q_jj[lane];
            double dx = hx[ci] - jx[cj], dy = hy[ci] - jy[cj], dz = hz[ci] - jz[cj];
            if constexpr (MODE == kPeriodic) {
              dx -= offx;
              dy -= offy;
              dz -= offz;
            }
            const double r2 = sq_norm_exact(dx, dy, dz);
            if (r2 < r02) {
              // without masks every pair counts twice (i, j) and (j, i)
              const int mult = MASKED ? hm[ci] + jm[cj] : 2;
              if (MASKED) ord += unsigned(mult);
              if (mult > 0) {
                hit = true;
                near = r2 < rs2;
                if (WRITE) {
                  r = sqrt(r2);
                  if (MODE == kPeriodic) {
                    const double dl = los == 0 ? dx : (los == 1 ? dy : dz);
                    mu = r > 0.0 ? dl / r : 0.0;
                  } else {
                    // line of sight along the pair midpoint (x_i + x_j) / 2
                    const double mx = hx[ci] + jx[cj], my = hy[ci] + jy[cj], mz = hz[ci] + jz[cj];
                    const double mn = sqrt((mx * mx + my * my) + mz * mz);
                    mu = (r > 0.0 && mn > 0.0) ? ((dx * mx + dy * my) + dz * mz) / (r * mn) : 0.0;
                  }
                  ww = scale * (hw[ci] * jw[cj]) * double(mult);
                }
              }
            }
          }
          const unsigned long long bal_a = __ballot(hit && near), bal_b = __ballot(hit && !near);
          if (!MASKED) ord_w += 2u * unsigned(__popcll(bal_a | bal_b));
          if (WRITE && hit) {
            const int64_t k = near ? wbase_a + written_a + __popcll(bal_a & below)
                                   : wbase_b + written_b + __popcll(bal_b & below);
            out_r[k] = r;
            out_mu[k] = mu;
            out_ww[k] = ww;
          }
          written_a += __popcll(bal_a);
          written_b += __popcll(bal_b);
        };
        for (uint32_t q0 = 0; q0 < total; q0 += 64, ii += d64, jj += r64) {
          if (jj >= utj) {
            jj -= utj;
            ++ii;
          }
          const uint32_t q = q0 + lane;
          bool cand = false;
          if (q < total && (!self || j0 + int(jj) > i0 + int(ii))) {
            const float fx = hxf[ii] - jxf[jj], fy = hyf[ii] - jyf[jj], fz = hzf[ii] - jzf[jj];
            cand = fmaf(fx, fx, fmaf(fy, fy, fz * fz)) < lim2f;
          }
          const unsigned long long bal = __ballot(cand);
          if (bal) {
            if (cand) {
              const int at = qn + __popcll(bal & below);
              q_ii[at] = int(ii);
              q_jj[at] = int(jj);
            }
            qn += __popcll(bal);
            if (qn >= 64) {
              __syncthreads();
              process(64);
              const int rest = qn - 64;
              int vi = 0, vj = 0;
              if (lane < rest) {
                vi = q_ii[64 + lane];
                vj = q_jj[64 + lane];
              }
              __syncthreads();
              if (lane < rest) {
                q_ii[lane] = vi;
                q_jj[lane] = vj;
              }
              qn = rest;
              __syncthreads();
            }
          }
        }
        __syncthreads();
        if (qn > 0) process(qn);
      }
    }
  }
  if (!WRITE) {
    if (MASKED)
      for (int o = 32; o > 0; o >>= 1) ord += __shfl_xor(ord, o);
    else
      ord = ord_w;
    if (lane == 0) {
      cnt_a[unit] = written_a;
      cnt_b[unit] = written_b;
      if (ord) atomicAdd(ordered, ord);
    }
  }
}

// Tiles per cell of catalogue `a` (at least one for a non-empty cell).
__global__ void k_unit_tiles(const int64_t *__restrict__ cell_start, int64_t ncells, int64_t *__restrict__ tiles) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  tiles[c] = (cell_start[c + 1] - cell_start[c] + kPairTile - 1) / kPairTile;
}

// unit_cell[u], unit_tile[u] for the units [base[c], base[c + 1]) of cell c.
__global__ void k_unit_fill(const int64_t *__restrict__ base, int64_t ncells, int *__restrict__ unit_cell,
                            int *__restrict__ unit_tile) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  for (int64_t u = base[c], t = 0; u < base[c + 1]; ++u, ++t) {
    unit_cell[u] = int(c);
    unit_tile[u] = int(t);
  }
}

PairUnits make_pair_units(Ctx &c, const Sorted &a, const Grid &g) {
  const int64_t ncells = g.ncells();
  int64_t *tiles = static_cast<int64_t *>(ensure(c, c.unit_tiles, size_t(ncells) * 8));
  int64_t *base = static_cast<int64_t *>(ensure(c, c.unit_base, size_t(ncells + 1) * 8));
  const unsigned nb = unsigned((ncells + 255) / 256);
  k_unit_tiles<<<nb, 256, 0, c.stream>>>(a.cell_start, ncells, tiles);
  scan_i64(c, tiles, base, ncells, c.pair_total);
  int64_t total = 0;
  HIPSTER_HIP(hipMemcpyAsync(&total, base + ncells, 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  PairUnits u;
  u.n = total;
  u.cell = static_cast<int *>(ensure(c, c.unit_cell, size_t(std::max<int64_t>(total, 1)) * 4));
  u.tile = static_cast<int *>(ensure(c, c.unit_tile, size_t(std::max<int64_t>(total, 1)) * 4));
  if (total > 0) k_unit_fill<<<nb, 256, 0, c.stream>>>(base, ncells, u.cell, u.tile);
  HIPSTER_HIP(hipGetLastError());
  return u;
}

// Bound of the single-precision prefilter: (R0 + delta)^2 with
// delta = 2^-17 M, M the largest coordinate magnitude a test sees (2 L for a
// periodic neighbour image, else the grid's extent from the origin).  A
// coordinate rounds to float within 2^-24 M and the float distance errs by
// less than 2^-20 M, so no pair inside R0 is rejected.
static float prefilter_bound(const Grid &g, double r0) {
  double m = 2.0 * g.L;
  if (!g.periodic) {
    const double o[3] = {g.ox, g.oy, g.oz};
    m = 0.0;
    for (int d = 0; d < 3; ++d) m = std::max(m, std::max(fabs(o[d]), fabs(o[d] + g.L)));
  }
  const double b = r0 + 0x1p-17 * m;
  return float(b * b);
}

// One launch of the enumeration kernel, with the mask handling compiled in
// only when a catalogue carries a mask.
template <bool WRITE, int MODE, typename... Args>
static void launch_pairs(Ctx &c, dim3 grid, const Sorted &a, const Sorted &b, Args... args) {
  if (a.m || b.m)
    k_pk_pairs<WRITE, MODE, true><<<grid, dim3(64), 0, c.stream>>>(a, b, args...);
  else
    k_pk_pairs<WRITE, MODE, false><<<grid, dim3(64), 0, c.stream>>>(a, b, args...);
  HIPSTER_HIP(hipGetLastError());
}

void pk_pairs_count(Ctx &c, const Sorted &s, const Grid &g, const PairUnits &u, double r0, double r_split,
                    int64_t *cnt_a, int64_t *cnt_b, unsigned long long *ordered) {
  if (u.n <= 0) return;
  launch_pairs<false, kPeriodic>(c, dim3(unsigned(u.n)), s, s, g.nc, g.L, r0 * r0, prefilter_bound(g, r0), r_split * r_split, 2, 1.0,
                                 u.cell, u.tile, int64_t(0), cnt_a, cnt_b, ordered, (const int64_t *)nullptr,
                                 (const int64_t *)nullptr, int64_t(0), int64_t(0), int64_t(0), (double *)nullptr,
                                 (double *)nullptr, (double *)nullptr);
}

void pk_pairs_write(Ctx &c, const Sorted &s, const Grid &g, const PairUnits &u, double r0, double r_split, int los,
                    const int64_t *off_a, const int64_t *off_b, int64_t base_a, int64_t base_b, int64_t n_a,
                    int64_t u0, int64_t u1, PkPairs out) {
  if (u1 <= u0) return;
  launch_pairs<true, kPeriodic>(c, dim3(unsigned(u1 - u0)), s, s, g.nc, g.L, r0 * r0, prefilter_bound(g, r0), r_split * r_split, los, 1.0,
                                u.cell, u.tile, u0, (int64_t *)nullptr, (int64_t *)nullptr,
                                (unsigned long long *)nullptr, off_a, off_b, base_a, base_b, n_a, out.r,
                                static_cast<double *>(out.mu), static_cast<double *>(out.ww));
}

void survey_pairs_count(Ctx &c, const Sorted &a, const Sorted &b, bool cross, const Grid &g, const PairUnits &u,
                        double r0, double r_split, int64_t *cnt_a, int64_t *cnt_b, unsigned long long *ordered) {
  if (u.n <= 0) return;
  const dim3 grid(unsigned(u.n));
  if (cross)
    launch_pairs<false, kSurveyCross>(c, grid, a, b, g.nc, g.L, r0 * r0, prefilter_bound(g, r0), r_split * r_split, 0, 1.0, u.cell, u.tile,
                                      int64_t(0), cnt_a, cnt_b, ordered, (const int64_t *)nullptr,
                                      (const int64_t *)nullptr, int64_t(0), int64_t(0), int64_t(0),
                                      (double *)nullptr, (double *)nullptr, (double *)nullptr);
  else
    launch_pairs<false, kSurveySelf>(c, grid, a, a, g.nc, g.L, r0 * r0, prefilter_bound(g, r0), r_split * r_split, 0, 1.0, u.cell, u.tile,
                                     int64_t(0), cnt_a, cnt_b, ordered, (const int64_t *)nullptr,
                                     (const int64_t *)nullptr, int64_t(0), int64_t(0), int64_t(0),
                                     (double *)nullptr, (double *)nullptr, (double *)nullptr);
}

void survey_pairs_write(Ctx &c, const Sorted &a, const Sorted &b, bool cross, const Grid &g, const PairUnits &u,
                        double r0, double r_split, double scale, const int64_t *off_a, const int64_t *off_b,
                        int64_t base_a, int64_t base_b, int64_t n_a, int64_t u0, int64_t u1, PkPairs out) {
  if (u1 <= u0) return;
  const dim3 grid(unsigned(u1 - u0));
  double *mu = static_cast<double *>(out.mu), *ww = static_cast<double *>(out.ww);
  if (cross)
    launch_pairs<true, kSurveyCross>(c, grid, a, b, g.nc, g.L, r0 * r0, prefilter_bound(g, r0), r_split * r_split, 0, scale, u.cell, u.tile,
                                     u0, (int64_t *)nullptr, (int64_t *)nullptr, (unsigned long long *)nullptr,
                                     off_a, off_b, base_a, base_b, n_a, out.r, mu, ww);
  else
    launch_pairs<true, kSurveySelf>(c, grid, a, a, g.nc, g.L, r0 * r0, prefilter_bound(g, r0), r_split * r_split, 0, scale, u.cell, u.tile,
                                    u0, (int64_t *)nullptr, (int64_t *)nullptr, (unsigned long long *)nullptr, off_a,
                                    off_b, base_a, base_b, n_a, out.r, mu, ww);
}

}  // namespace hipster
