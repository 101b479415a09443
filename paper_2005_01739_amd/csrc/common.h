// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <initializer_list>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hipster.h"

namespace hipster {

// Largest sizes the kernels are compiled for.
constexpr int kMaxNk = 128;        // power-spectrum bins
constexpr int kMaxNkB = 64;        // bispectrum bins (more than 16: in groups of 16)
constexpr int kMaxCellsPerAxis = 160;
constexpr int kLMaxApi = 6;          // largest multipole
constexpr double kMaxPhaseMixed = 1e6;  // largest k * R0 of the mixed form
constexpr int kEiiMaxNodes = 8192;      // largest E^II table (intervals over [0, 2 R0])
constexpr int kEiiMaxNkApi = 16;        // bins of the E^II table (analytic DDR^II)

struct Error {
  hipster_status status;
  std::string msg;
};

#define HIPSTER_HIP(expr)                                                         \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::hipster::Error{HIPSTER_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// A grow-only device buffer owned by a context.
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
};

struct Ctx;
void *ensure(Ctx &c, DevBuf &b, size_t bytes);
// Bytes of the workspace still free after alignment (workspace mode only).
size_t arena_left(const Ctx &c);

// Cell grid: n_c cells per axis of side L / n_c > R0 covering the cube
// [o, o + L)^3.  A periodic box has o = 0; a survey grid is the bounding cube
// of its catalogues, with no periodicity.
struct Grid {
  int nc;
  double L;
  double scale;  // n_c / L
  double ox = 0.0, oy = 0.0, oz = 0.0;
  bool periodic = true;
  int64_t ncells() const { return int64_t(nc) * nc * nc; }
};

Grid make_grid(double L, double r0);
Grid make_survey_grid(const double lo[3], const double hi[3], double r0);

// Bounding box of a catalogue (device or host-copied positions), merged into
// lo/hi (host); throws HIPSTER_EOUTOFBOX on a non-finite coordinate.
void bounding_box(Ctx &c, const void *pos, int64_t n, int dtype, double lo[3], double hi[3]);

// A catalogue sorted by cell, structure-of-arrays, coordinates in double
// (exact for single-precision inputs).
struct Sorted {
  int64_t n = 0;
  const double *x = nullptr, *y = nullptr, *z = nullptr, *w = nullptr;
  const uint8_t *m = nullptr;      // primary mask per sorted particle (may be null)
  const int64_t *cell_start = nullptr; // [ncells + 1]
  const int *scell = nullptr;          // cell of each sorted point
};


// Pair stream for the power spectrum: one entry per unordered pair inside R0.
// mu and ww are kept in double in both forms: L_l(mu) has slopes up to
// l(l+1)/2, so a single-precision mu would cost ~1e-6 at l = 6.
struct PkPairs {
  double *r = nullptr;
  void *mu = nullptr;
  void *ww = nullptr;
};

// A batched sweep task: a contiguous range of one box's pairs.
struct PkTask {
  int64_t begin, end;
  int box;
  int pad;
};

// Per-box constants of the batched sweep.
struct BoxSweep {
  double inv_r0;
  int edge_off;
  int n_edges;
};

// A cached E^II table (analytic DDR^II).
struct EiiEntry {
  std::vector<double> key;
  DevBuf buf;
  uint64_t used = 0;
};

// Scratch of one catalogue's cell list.
struct CellScratch {
  DevBuf cell, count, start, cursor, idx, x, y, z, w, m, bad, scan_tmp, scell, sort_tmp;
};

// Device inputs of one box of a batched bispectrum (kept until the batch's
// queued sweep has run).
struct BkBoxScratch {
  CellScratch cd, cr;
  DevBuf pos, w, mask, rpos, rw, rmask, rgen, edges, coef, cnt;
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t mem_cap = 0;
  uint64_t mem_used = 0;
  // Workspace mode (the no-allocation entry point): when arena is set,
  // ensure() hands out 256-byte-aligned pieces of [arena, arena + arena_cap)
  // in order and never calls the allocator, and no HIP events are created.
  unsigned char *arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  std::string last_error;
  CellScratch cells_d, cells_r;
  DevBuf pos_in, w_in, mask_in, rpos_in, rw_in, rmask_in;
  DevBuf pair_cnt, pair_cnt_b, pair_ord, pair_off, pair_off_b, pair_total;
  DevBuf pr, pmu, pww, pux, puy, puz;
  DevBuf edges, partial, merged, ordered_count, bbox;
  DevBuf unit_tiles, unit_base, unit_cell, unit_tile;
  DevBuf bk_partial, bk_partial_r, bk_coef;
  DevBuf bq_count, bq_off, bq_scan, bq_quads, bk_abuf, bk_wbuf, bk_tiles, bk_gpart, bk_gmerged;
  DevBuf bq_jobs, bq_tasks, bq_slots, bq_counter;  // queued bispectrum sweep
  DevBuf bo_cnt, bo_key, bo_key2, bo_iota, bo_perm, bo_tmp;  // primaries ordered by neighbour count
  DevBuf ca_q, ca_l, ca_count, ca_out, ca_tab;      // anisotropic C term
  std::vector<BkBoxScratch> bt_bk;                  // batched bispectrum, per box
  DevBuf rgen, pk_l1;
  DevBuf bt_tasks, bt_boxes, bt_counter, bt_rows, bt_first, bt_out;
  DevBuf eii_consts, ddr2_partial, ddr2_hist, ddr2_counter, ddr2_T, ct_tab, ct_consts, ct_C, ct_wmax, ct_jbar, ct_sel;
  DevBuf pt_tab, pt_consts, pt_T;  // power spectrum, table form
  std::vector<double> pt_key;      // (R0, n_k, n_l, n_c, edges) of the table in pt_tab
  DevBuf th_r, th_w, th_p, th_wp, th_pk, th_ek, th_g, th_J, th_om, th_K, th_out, th_wt, th_pb, th_bk, th_T, th_X;
  // E^II tables on the device, keyed by (R0, n_x, ell_max, edges).
  std::vector<EiiEntry> eii_cache;
  uint64_t eii_clock = 0;
  // Measured kernel parameters (autotuner), keyed by kernel, shape and device.
  std::map<std::string, int> tune;
  bool tune_file_read = false;
  DevBuf tune_scratch;
  // W~^a depends only on (R0, k_a, k_{a+1}); repeated calls reuse it.
  std::map<std::tuple<double, double, double>, double> wtilde_cache;
};

// W~^a for each bin, through the context's cache.
void wtilde_bins(Ctx &c, double r0, int n_k, const double *k_edges, double *out);

// ---------------------------------------------------------------- kernels
// Cell list: sorts `n` points into the grid and fills `out` (device).
Sorted build_cells(Ctx &c, CellScratch &s, const Grid &g, const void *pos, const void *w,
                   const uint8_t *mask_dev, int64_t n, int dtype);

// Sorted-primary indices in cell order and, inside a cell, selected
// primaries by their number of secondaries within R0 (the others after
// them): the bispectrum sweep takes a cell's primaries four at a time in this
// order, so the four have about the same number of pairs.  Device array,
// valid until the next call on c; null when prim.n is 0.
const int *order_by_neighbours(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0,
                               bool self_set);

// Exclusive scan of n int64 values (in-place allowed); out has n + 1 entries.
void scan_i64(Ctx &c, const int64_t *in, int64_t *out, int64_t n, DevBuf &tmp);

// Work units of the pair enumeration: unit u is home cell unit_cell[u]'s
// tile unit_tile[u] of up to 64 points (one workgroup each); units are ordered
// by cell, then tile.  Built from the home catalogue's cell list (device
// arrays; n is read back to the host).
struct PairUnits {
  int64_t n = 0;
  int *cell = nullptr;
  int *tile = nullptr;
};
PairUnits make_pair_units(Ctx &c, const Sorted &a, const Grid &g);

// Power-spectrum pair enumeration.  The count pass fills cnt_a[u] / cnt_b[u]
// (pairs with r < r_split / the rest) for every unit and adds the
// ordered-pair multiplicity to *ordered.  The write pass over units [u0, u1)
// stores a unit's near pairs at off_a[u] - base_a and its far pairs at
// n_a + off_b[u] - base_b.
void pk_pairs_count(Ctx &c, const Sorted &s, const Grid &g, const PairUnits &u, double r0, double r_split,
                    int64_t *cnt_a, int64_t *cnt_b, unsigned long long *ordered);
void pk_pairs_write(Ctx &c, const Sorted &s, const Grid &g, const PairUnits &u, double r0, double r_split, int los,
                    const int64_t *off_a, const int64_t *off_b, int64_t base_a, int64_t base_b, int64_t n_a,
                    int64_t u0, int64_t u1, PkPairs out);

// Survey-geometry enumeration (no periodicity, line of sight along each
// pair's midpoint).  Home cells (and units) come from catalogue `a`.
// cross = false: `b` is `a` and every unordered pair is found once (half
// stencil); cross = true: every pair (i in a, j in b) is found once (27
// cells).  A pair's weight is scale * w_i w_j (m_i + m_j), m the mask bits (1
// without a mask); the count pass adds sum (m_i + m_j) to *ordered.
void survey_pairs_count(Ctx &c, const Sorted &a, const Sorted &b, bool cross, const Grid &g, const PairUnits &u,
                        double r0, double r_split, int64_t *cnt_a, int64_t *cnt_b, unsigned long long *ordered);
void survey_pairs_write(Ctx &c, const Sorted &a, const Sorted &b, bool cross, const Grid &g, const PairUnits &u,
                        double r0, double r_split, double scale, const int64_t *off_a, const int64_t *off_b,
                        int64_t base_a, int64_t base_b, int64_t n_a, int64_t u0, int64_t u1, PkPairs out);

// Pair-weight sweep: adds E'_l(e) = sum c_l k_e^3 G_l(k_e r) into
// partial[nwaves][n_ell][n_edges] (zeroed by the caller before the first
// chunk).  `ek` is the device edge table (k_e, 1/k_e, k_e^3, doubles).  The
// general kernel takes any pairs; the far kernel (either form) only pairs
// with r >= U_BIG / k_0 and k_0 > 0.
void pk_sweep_general(Ctx &c, const PkPairs &p, int64_t npairs, int n_ell, bool fp64, double r0, const double *ek,
                      int n_edges, double *partial, int nwaves);
void pk_sweep_far(Ctx &c, const PkPairs &p, int64_t npairs, int n_ell, bool fp64, double r0, const double *ek,
                  int n_edges, double *partial, int nwaves);
int pk_sweep_waves(Ctx &c);
void pk_sweep_tasks(Ctx &c, const PkPairs &p, const PkTask *tasks, int ntasks, int *counter, const double *edges,
                    const BoxSweep *boxes, int cols, double *rows, int n_ell, bool fp64, int nwaves);
void merge_boxes(Ctx &c, const double *rows, int cols, const int *first, int nboxes, double *out);
void merge_partials(Ctx &c, const double *partial, int rows, int cols, double *out);

// Bispectrum sums of one primary catalogue against the data (Sec. 4), host
// arrays: G [NL][NK][NK] = sum_p w_p (4 pi/(2l+1)) sum_m A^a_lm A^b_lm,
// C [NL][NK][NK] = sum_p w_p C^ab_l (with_c, FP64 form only; zeros
// otherwise), S0 [NK] = sum_p w_p sum_q w_q W jbar^b_0 (primaries p selected by
// prim.m, pairs q != p when self_set).  edges / coef: device n_k + 1 edges and
// n_k values 3 / (k_{a+1}^3 - k_a^3).  npairs (device) gains the ordered pairs.
struct BkSums {
  int NL = 0, NK = 0;
  std::vector<double> G, C, S0;
  uint64_t launches = 0;
  double ms_kernel = 0.0;  // the sweep launches alone (HIP events)
};
void bk_sweep(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
              const double *edges, const double *coef, int NK, int ell_max, bool fp64, bool with_c,
              unsigned long long *npairs, BkSums &out);
void widen_i32(Ctx &c, const int *in, int64_t *out, int64_t n);

// Many boxes' bispectrum sums in one queued sweep: each job is one primary
// set against its box's data (as for bk_sweep), all with ell_max and the
// form `fp64`, at most 16 bins each.  Quads of every job are cut into tasks
// that the waves of one launch take in turn, the jobs with the most pairs
// per quad first; each task's sums go to a row of their own and each job's
// rows are merged in task order, so the result does not depend on which wave
// ran which task.  out[j] receives job j's sums.
struct BkQueueJob {
  Sorted prim, sec;
  Grid g;
  double r0 = 0.0;
  bool self_set = false;
  const double *edges = nullptr, *coef = nullptr;  // device
  int NK = 0;
  unsigned long long *npairs = nullptr;  // device
  double cost = 0.0;                     // expected pairs per primary (task order)
};
void bk_sweep_queue(Ctx &c, const std::vector<BkQueueJob> &jobs, int ell_max, bool fp64, std::vector<BkSums> &out);

// Anisotropic bispectrum sums of one primary set against the data (mixed
// form, n_k <= 16, ell_max <= 4): G [n_c][n_k][n_k] = sum_p w_p
// sum_{mu = +-m} A^a_{l1 mu} A^b_{l2 mu} for the combinations (l1 <= l2, m <= l1)
// in (l1, l2, m) order, and T [ell_max+1][n_k] = sum_p w_p A^a_{l0}
// (real orthonormal harmonics about z).
void bk_aniso_sweep(Ctx &c, const Sorted &prim, const Sorted &sec, const Grid &g, double r0, bool self_set,
                    const double *edges, const double *coef, int NK, int ell_max, unsigned long long *npairs,
                    std::vector<double> &G, std::vector<double> &T, double &ms_kernel);

// n uniform points in [0, L)^3 (device, [n][3] doubles), point i from block
// i + 1 of the Philox4x64-10 generator keyed by (seed, 0): x_d = L (word_d >> 11)
// 2^-53, a coordinate that rounds to L set to 0.
void random_points(Ctx &c, uint64_t seed, int64_t n, double L, double *out);

// L1 mass of the power-spectrum pair sums in double precision: rows
// [nwaves][n_ell][n_k] += sum over the stream's pairs of
// |ww| W(r/R0) (2l+1) |L_l(mu)| |jbar^a_l(r)|, l = 0, 2, .. (zeroed by the caller).
void pk_l1_sweep(Ctx &c, const PkPairs &p, int64_t npairs, int n_ell, double r0, const double *edges, int n_edges,
                 double *rows, int nwaves);

// Analytic DDR^II term: the E^{II,ab}_l table on the nodes m 2 R0 / n_x
// (device, [ell_max+1][n_k][n_k][n_x+1]); the 2 R0 pair sweep of the
// cubic-interpolation weights and its contraction with the table into
// T[rows] (rows = (ell_max+1) n_k^2), adding the ordered (pair, image) count
// to *ordered.  `s` is the data sorted on a grid of cells >= 2 R0.
int eii_default_nodes(double r0, double k_max);
void eii_table(Ctx &c, double r0, int n_k, const double *k_edges, int ell_max, int n_x, double *table);
void ddr2_sweep(Ctx &c, const Sorted &s, const Grid &g, double r0, int n_x, const double *table, int rows,
                double *T, unsigned long long *ordered);
size_t ddr2_max_nodes(Ctx &c);
// Power spectrum, table form: T[li][a] = sum over ordered pairs inside R0 of
// w_i w_j W(r/R0) L_{2 li}(mu) jbar^a_{2 li}(r), with jbar through a quintic
// table on n_c intervals of [0, R0] (device output, n_l n_k doubles).
int pktab_default_nodes(double r0, double k_max);
void pktab_sweep(Ctx &c, const Sorted &s, const Grid &g, double r0, int n_k, const double *k_edges, int n_l, int los,
                 int n_c, double *T, unsigned long long *ordered);
// The same for the survey geometry: `a` against `b` (cross: every (a, b) pair
// once, both orientations counted; else the unordered pairs of a), no
// periodicity, the pair-midpoint line of sight from the origin, every pair
// weight times pair_scale; coord_bound bounds every |coordinate|.
void pktab_survey_sweep(Ctx &c, const Sorted &a, const Sorted &b, bool cross, const Grid &g, double coord_bound,
                        double pair_scale, double r0, int n_k, const double *k_edges, int n_l, int n_c, double *T,
                        unsigned long long *ordered);
// C term of the bispectrum in the mixed form:
// C^ab_l = sum over ordered pairs (p, q != p) inside R0, p selected by the
// mask, of w_p w_q^2 W(r/R0)^2 jbar^a_l(r) jbar^b_l(r), from a pair histogram
// of interpolation weights on the nodes m R0 / n_c and a table of
// jbar^a jbar^b; C [ell_max+1][n_k][n_k] (device).  `s` is the data sorted on
// the R0 grid `g`.
int cterm_default_nodes(double r0, double k_max);
// Anisotropic C term (fixed line of sight z): host C[n_comb][n_k][n_k] =
// sum over ordered pairs (p, q) of w_p w_q^2 W(r/R0)^2 jbar^a_{l1} jbar^b_{l2}
// Q_c(mu_pq), Q_c = sum_L q[c][L] P_L (L = 0 .. 2 ell_max), through
// fixed-point r-histograms of w_p w_q^2 W^2 P_L(mu) (one section per L, in
// passes the LDS holds) contracted with tables of q_L jbar^a_{l1} jbar^b_{l2}.
// cross: primaries s against neighbours b (all 27 cells), else s with
// itself.  The first pass adds the ordered pairs to *ordered.
void cterm_aniso_sweep(Ctx &c, const Sorted &s, const Sorted &b, bool cross, const Grid &g, double r0, int n_k,
                       const double *k_edges, int ell_max, int n_c, uint64_t n_ordered, int n_comb, const int *cl1,
                       const int *cl2, const double *q, double *C, unsigned long long *ordered);
// cross = false: `s` with itself (b ignored); cross = true: primaries `s`
// (random primaries) against secondaries `b` (the data), every pair once.
// n_ordered: the ordered pairs inside R0 (bounds the fixed-point sums).
void cterm_sweep(Ctx &c, const Sorted &s, const Sorted &b, bool cross, const Grid &g, double r0, int n_k,
                 const double *k_edges, int ell_max, int n_c, uint64_t n_ordered, double *C,
                 unsigned long long *ordered);

// Theory side (Secs. 5, 6), double precision throughout.  theory_omega:
// om_dev[l][i][a] = omega^a_{l l_step}(p_i) for n_l multipoles; theory_pk:
// windowed P^a_l of model multipoles xi[l/2][m] on the caller's r quadrature;
// theory_cov: Gaussian covariance [n_l][n_k][n_l][n_k] of even multipoles on
// the caller's p quadrature with model multipoles pk[l/2][i].  Host inputs.
void theory_omega(Ctx &c, double r0, int n_k, const double *k_edges, int n_l, int l_step, int n_p, const double *p,
                  double *om_dev);
void theory_pk(Ctx &c, double r0, int n_k, const double *k_edges, int n_l, int n_r, const double *r, const double *wr,
               const double *xi, double *out_dev);
void theory_cov(Ctx &c, double r0, double volume, int n_k, const double *k_edges, int n_l, int n_p, const double *p,
                const double *wp, const double *pk, double *out_dev);
// Poisson two-point covariance term of even multipoles on the caller's x
// quadrature with model multipoles xi[L/2][m] (even L < 2 n_l).
void theory_c2(Ctx &c, double r0, double nbar, double volume, int n_k, const double *k_edges, int n_l, int n_r,
               const double *r, const double *wr, const double *xi, double *out_dev);
// Non-Gaussian intrinsic covariance term on the caller's p quadrature with
// the collapsed-trispectrum multipoles tbar [n_l][n_l][n_p][n_p] (host).
void theory_ng(Ctx &c, double r0, double volume, int n_k, const double *k_edges, int n_l, int n_p, const double *p,
               const double *wp, const double *tbar, double *out_dev);
// Poisson three-point covariance term on the caller's p quadrature; wt the
// host W~ per bin, pbin [n_l][n_k] and bk [n_l][n_k][n_k] host arrays or null.
void theory_c3(Ctx &c, double r0, double nbar, double volume, int n_k, const double *k_edges, int n_l, int n_p,
               const double *p, const double *wp, const double *pk, const double *wt, const double *pbin,
               const double *bk, double *out_dev);

// Autotuner cache: tune_key names a kernel, its shape and the device (name
// and compute-unit count); tune_lookup returns a stored value (0 if none),
// reading the file named by HIPSTER_TUNE_CACHE once; tune_store records a
// value in the context and appends it to that file.
std::string tune_key(Ctx &c, const char *kernel, std::initializer_list<int> shape);
int tune_lookup(Ctx &c, const std::string &key);
void tune_store(Ctx &c, const std::string &key, int value);

// Host analytic terms.
double wtilde_bin(double r0, double k1, double k2);

}  // namespace hipster
