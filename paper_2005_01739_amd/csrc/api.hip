// C ABI entry points: argument checks, context and scratch memory, the
// host-side orchestration of the device passes, and the final normalisation
// (Sec. 3 binned power spectrum; Sec. 4 bispectrum summary estimator).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"
#include "specfun.h"

struct hipster_ctx {
  hipster::Ctx c;
};

namespace hipster {

void *ensure(Ctx &c, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return b.p;
  if (c.arena) {
    const size_t off = (c.arena_used + 255) & ~size_t(255);
    if (off > c.arena_cap || bytes > c.arena_cap - off)
      throw Error{HIPSTER_ENOMEM, "the call needs more device scratch than the " +
                                      std::to_string(c.arena_cap >> 20) +
                                      " MiB static workspace of the no-allocation entry point holds"};
    b.p = c.arena + off;
    b.cap = bytes;
    c.arena_used = off + bytes;
    return b.p;
  }
  if (b.p) {
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
    HIPSTER_HIP(hipFree(b.p));
    c.mem_used -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 8;  // headroom for the next, slightly larger call
  if (c.mem_cap && c.mem_used + want > c.mem_cap) {
    want = bytes;
    if (c.mem_used + want > c.mem_cap) throw Error{HIPSTER_ENOMEM, "device memory cap exceeded"};
  }
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    throw Error{HIPSTER_ENOMEM, std::string("hipMalloc of ") + std::to_string(want) + " bytes failed"};
  }
  b.cap = want;
  c.mem_used += want;
  return b.p;
}

size_t arena_left(const Ctx &c) {
  const size_t off = (c.arena_used + 255) & ~size_t(255);
  return off < c.arena_cap ? c.arena_cap - off : 0;
}

void wtilde_bins(Ctx &c, double r0, int n_k, const double *k_edges, double *out) {
  for (int a = 0; a < n_k; ++a) {
    const auto key = std::make_tuple(r0, k_edges[a], k_edges[a + 1]);
    auto it = c.wtilde_cache.find(key);
    if (it == c.wtilde_cache.end()) {
      if (c.wtilde_cache.size() > 100000) c.wtilde_cache.clear();
      it = c.wtilde_cache.emplace(key, wtilde_bin(r0, k_edges[a], k_edges[a + 1])).first;
    }
    out[a] = it->second;
  }
}

static void free_buf(DevBuf &b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

static void free_cells(CellScratch &s) {
  DevBuf *all[] = {&s.cell,  &s.count, &s.start, &s.cursor,   &s.idx,   &s.x,       &s.y,
                   &s.z,     &s.w,     &s.m,     &s.bad,      &s.scan_tmp, &s.scell, &s.sort_tmp};
  for (DevBuf *b : all) free_buf(*b);
}

// ------------------------------------------------------------ validation
static void check_points(const hipster_points *p, const char *what, double box) {
  if (!p || !p->pos) throw Error{HIPSTER_EINVAL, std::string(what) + ": NULL catalogue or positions"};
  if (p->dtype != HIPSTER_F32 && p->dtype != HIPSTER_F64) throw Error{HIPSTER_EINVAL, std::string(what) + ": bad dtype"};
  if (p->n < 0 || p->n > int64_t(0x7fffffff)) throw Error{HIPSTER_EUNSUPPORTED, std::string(what) + ": n outside [0, 2^31)"};
  if (p->on_device != 0 && p->on_device != 1) throw Error{HIPSTER_EINVAL, std::string(what) + ": on_device must be 0 or 1"};
  (void)box;
}

static void check_params(const hipster_params *q, bool bispectrum, bool allow_table = false) {
  if (!q) throw Error{HIPSTER_EINVAL, "NULL parameters"};
  if (!(q->box > 0.0) || !isfinite(q->box)) throw Error{HIPSTER_EDOMAIN, "box size must be finite and positive"};
  if (!(q->r0 > 0.0) || !(q->r0 <= 0.5 * q->box)) throw Error{HIPSTER_EDOMAIN, "R0 must lie in (0, L/2]"};
  const int maxk = bispectrum ? kMaxNkB : kMaxNk;
  if (q->n_k < 1 || q->n_k > maxk)
    throw Error{HIPSTER_EUNSUPPORTED, "n_k must lie in [1, " + std::to_string(maxk) + "]"};
  if (!q->k_edges) throw Error{HIPSTER_EINVAL, "NULL k_edges"};
  for (int a = 0; a <= q->n_k; ++a) {
    if (!isfinite(q->k_edges[a]) || q->k_edges[a] < 0.0) throw Error{HIPSTER_EDOMAIN, "k edges must be finite and >= 0"};
    if (a > 0 && !(q->k_edges[a] > q->k_edges[a - 1])) throw Error{HIPSTER_EDOMAIN, "k edges must increase strictly"};
  }
  if (q->ell_max < 0 || q->ell_max > kLMaxApi) throw Error{HIPSTER_EDOMAIN, "ell_max must lie in [0, 6]"};
  if (!bispectrum && (q->ell_max & 1)) throw Error{HIPSTER_EDOMAIN, "power spectrum: ell_max must be even"};
  if (!bispectrum && (q->los_axis < 0 || q->los_axis > 2)) throw Error{HIPSTER_EINVAL, "los_axis must be 0, 1 or 2"};
  if (q->precision == HIPSTER_TABLE && !allow_table)
    throw Error{HIPSTER_EUNSUPPORTED, "HIPSTER_TABLE is available for hipster_pk_ell and hipster_pk_survey only"};
  if (q->precision != HIPSTER_MIXED && q->precision != HIPSTER_FP64 && q->precision != HIPSTER_TABLE)
    throw Error{HIPSTER_EINVAL, "bad precision"};
  // the mixed form's table-driven sine and cosine reduce u = k r exactly only
  // below ~1.6e6 (a 27-bit pi/128 times the table index)
  if (q->precision == HIPSTER_MIXED && q->k_edges[q->n_k] * q->r0 > kMaxPhaseMixed)
    throw Error{HIPSTER_EUNSUPPORTED, "mixed precision needs k_max * R0 <= 1e6; use HIPSTER_FP64"};
}

// Device copy of a catalogue when it lives on the host.
static const void *device_view(Ctx &c, DevBuf &b, const void *p, int64_t bytes, int on_device) {
  if (!p) return nullptr;
  if (on_device) return p;
  void *d = ensure(c, b, size_t(bytes));
  HIPSTER_HIP(hipMemcpyAsync(d, p, size_t(bytes), hipMemcpyHostToDevice, c.stream));
  return d;
}

static const uint8_t *device_mask(Ctx &c, DevBuf &b, const uint8_t *mask, int64_t n) {
  if (!mask) return nullptr;
  void *d = ensure(c, b, size_t(n));
  HIPSTER_HIP(hipMemcpyAsync(d, mask, size_t(n), hipMemcpyHostToDevice, c.stream));
  return static_cast<const uint8_t *>(d);
}

static int64_t pair_chunk_capacity() {
  const char *e = getenv("HIPSTER_PAIR_CHUNK");
  int64_t cap = int64_t(1) << 28;
  if (e) {
    long long v = atoll(e);
    if (v >= 1024) cap = v;
  }
  return cap;
}

struct Timer {
  Ctx &c;
  std::vector<hipEvent_t> evs;
  explicit Timer(Ctx &cc) : c(cc) {}
  hipEvent_t mark() {
    if (c.arena) return nullptr;  // workspace mode: no events, times read 0
    hipEvent_t e;
    HIPSTER_HIP(hipEventCreate(&e));
    HIPSTER_HIP(hipEventRecord(e, c.stream));
    evs.push_back(e);
    return e;
  }
  static double ms(hipEvent_t a, hipEvent_t b) {
    if (!a || !b) return 0.0;
    float t = 0.f;
    if (hipEventElapsedTime(&t, a, b) != hipSuccess) return 0.0;
    return double(t);
  }
  ~Timer() {
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  }
};

// Sum of a catalogue's weights in input order (FP64; n for unit weights).
static double weight_sum(const hipster_points *pts) {
  const int64_t n = pts->n;
  if (!pts->w) return double(n);
  const size_t esz = pts->dtype == HIPSTER_F32 ? 4 : 8;
  std::vector<unsigned char> raw(size_t(n) * esz);
  if (pts->on_device) HIPSTER_HIP(hipMemcpy(raw.data(), pts->w, size_t(n) * esz, hipMemcpyDeviceToHost));
  else memcpy(raw.data(), pts->w, size_t(n) * esz);
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i)
    s += esz == 4 ? double(reinterpret_cast<const float *>(raw.data())[i]) : reinterpret_cast<const double *>(raw.data())[i];
  return s;
}

static int device_cus(Ctx &c) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c.device) == hipSuccess && prop.multiProcessorCount > 0)
    return prop.multiProcessorCount;
  return 256;
}

// ---------------------------------------------------------- power spectrum
// One set of pairs through the power-spectrum sweep: the count pass (two
// r-buckets per work unit, a home cell's tile), offsets, then chunks of units
// whose pairs fit the pair buffer, each written and swept into `partial`.
// count(cnt_a, cnt_b, ord) and write(off_a, off_b, base_a, base_b, n_a, u0,
// u1, pairs) run the set's enumeration kernels.  far_ok (k_0 > 0) says the second bucket,
// r >= U_BIG / k_0, may take the sweep's far path.
struct SweepStats {
  uint64_t ordered = 0;
  double ms_pairs = 0.0, ms_sweep = 0.0, ms_far = 0.0;
  uint64_t launches = 0, far_pairs = 0;
};

template <typename CountF, typename WriteF>
static SweepStats sweep_pair_set(Ctx &c, Timer &tm, int64_t nunits, CountF &&count, WriteF &&write, int n_ell,
                                 bool fp64, double r0, const double *edges, int n_edges, bool far_ok,
                                 double *partial, int nwaves, double *l1_rows = nullptr, bool main_sweep = true) {
  SweepStats st;
  int64_t *cnt_a = static_cast<int64_t *>(ensure(c, c.pair_cnt, size_t(nunits) * 8));
  int64_t *cnt_b = static_cast<int64_t *>(ensure(c, c.pair_cnt_b, size_t(nunits) * 8));
  int64_t *off_a = static_cast<int64_t *>(ensure(c, c.pair_off, size_t(nunits + 1) * 8));
  int64_t *off_b = static_cast<int64_t *>(ensure(c, c.pair_off_b, size_t(nunits + 1) * 8));
  unsigned long long *ord = static_cast<unsigned long long *>(ensure(c, c.ordered_count, 16));
  hipEvent_t e0 = tm.mark();
  HIPSTER_HIP(hipMemsetAsync(ord, 0, 8, c.stream));
  count(cnt_a, cnt_b, ord);
  scan_i64(c, cnt_a, off_a, nunits, c.pair_total);
  scan_i64(c, cnt_b, off_b, nunits, c.pair_total);
  std::vector<int64_t> ha(size_t(nunits) + 1), hb(size_t(nunits) + 1);
  unsigned long long hord = 0;
  HIPSTER_HIP(hipMemcpyAsync(ha.data(), off_a, size_t(nunits + 1) * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(hb.data(), off_b, size_t(nunits + 1) * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(&hord, ord, 8, hipMemcpyDeviceToHost, c.stream));
  hipEvent_t e1 = tm.mark();
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  st.ordered = hord;
  st.ms_pairs += Timer::ms(e0, e1);
  auto pairs_in = [&](int64_t a, int64_t b) { return (ha[size_t(b)] - ha[size_t(a)]) + (hb[size_t(b)] - hb[size_t(a)]); };
  const int64_t total = pairs_in(0, nunits);
  if (total == 0) return st;
  int64_t cap = std::min<int64_t>(pair_chunk_capacity(), total);
  int64_t unit_max = 0;
  for (int64_t a = 0; a < nunits; ++a) unit_max = std::max(unit_max, pairs_in(a, a + 1));
  cap = std::max(cap, unit_max);
  if (c.arena && c.pr.cap == 0) {
    // workspace mode: the three 8-byte pair arrays take what is left after
    // a reserve for the merged sums, so a larger catalogue runs in more chunks
    constexpr size_t kReserve = size_t(1) << 16;
    const size_t left = arena_left(c);
    const int64_t fit = left > kReserve + 1024 ? int64_t((left - kReserve - 1024) / 24) : 0;
    if (fit < unit_max)
      throw Error{HIPSTER_ENOMEM, "the pair stream of one cell tile does not fit the static workspace of the "
                                  "no-allocation entry point"};
    cap = std::min(cap, fit);
  }
  PkPairs pp;
  pp.r = static_cast<double *>(ensure(c, c.pr, size_t(cap) * 8));
  pp.mu = ensure(c, c.pmu, size_t(cap) * 8);
  pp.ww = ensure(c, c.pww, size_t(cap) * 8);
  int64_t c0 = 0;
  while (c0 < nunits) {
    int64_t c1 = c0 + 1;
    while (c1 < nunits && pairs_in(c0, c1 + 1) <= cap) ++c1;
    const int64_t np = pairs_in(c0, c1), n_a = ha[size_t(c1)] - ha[size_t(c0)];
    if (np > 0) {
      hipEvent_t a = tm.mark();
      write(off_a, off_b, ha[size_t(c0)], hb[size_t(c0)], n_a, c0, c1, pp);
      hipEvent_t b = tm.mark();
      // near bucket (or every pair) through the general kernel, the far
      // bucket through the far kernel
      const int64_t n_gen = main_sweep ? (far_ok ? n_a : np) : np;
      if (main_sweep) pk_sweep_general(c, pp, n_gen, n_ell, fp64, r0, edges, n_edges, partial, nwaves);
      hipEvent_t m = tm.mark();
      if (main_sweep && n_gen < np) {
        PkPairs far;
        far.r = pp.r + n_gen;
        far.mu = static_cast<double *>(pp.mu) + n_gen;
        far.ww = static_cast<double *>(pp.ww) + n_gen;
        pk_sweep_far(c, far, np - n_gen, n_ell, fp64, r0, edges, n_edges, partial, nwaves);
      }
      hipEvent_t d = tm.mark();
      // the L1 mass, an extra double-precision pass over the same pairs
      if (l1_rows) pk_l1_sweep(c, pp, np, n_ell, r0, edges, n_edges, l1_rows, nwaves);
      if (d) HIPSTER_HIP(hipEventSynchronize(d));
      else HIPSTER_HIP(hipStreamSynchronize(c.stream));
      st.ms_pairs += Timer::ms(a, b);
      st.ms_sweep += Timer::ms(b, d);
      st.ms_far += Timer::ms(m, d);
      st.far_pairs += uint64_t(np - n_gen);
      ++st.launches;
    }
    c0 = c1;
  }
  return st;
}

// The sweep's edge table on the device: k_e, 1/k_e, k_e^3 (doubles).  A zero
// edge stores 0 for its reciprocal; its u = 0 always takes the general
// (Taylor) path.
static double *upload_edges(Ctx &c, int n_k, const double *k_edges) {
  const int n_edges = n_k + 1;
  std::vector<double> he(size_t(3 * n_edges));
  for (int e = 0; e < n_edges; ++e) {
    const double k = k_edges[e];
    he[size_t(e)] = k;
    he[size_t(n_edges + e)] = k > 0.0 ? 1.0 / k : 0.0;
    he[size_t(2 * n_edges + e)] = k * k * k;
  }
  double *edges = static_cast<double *>(ensure(c, c.edges, he.size() * 8));
  HIPSTER_HIP(hipMemcpyAsync(edges, he.data(), he.size() * 8, hipMemcpyHostToDevice, c.stream));
  return edges;
}

// Merged edge sums -> S^a_l = 3 (2l+1)(-i)^l [E'_{a+1} - E'_a] / (k_{a+1}^3 - k_a^3),
// E'_e = k_e^3 E_e as accumulated by the sweep.
static std::vector<double> bin_sums(Ctx &c, double *partial, int nwaves, int n_ell, int n_k, const double *k_edges) {
  const int n_edges = n_k + 1, cols = n_ell * n_edges;
  double *merged = static_cast<double *>(ensure(c, c.merged, size_t(cols) * 8));
  merge_partials(c, partial, nwaves, cols, merged);
  std::vector<double> E(static_cast<size_t>(cols));
  HIPSTER_HIP(hipMemcpyAsync(E.data(), merged, size_t(cols) * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  std::vector<double> S(static_cast<size_t>(n_ell * n_k));
  for (int li = 0; li < n_ell; ++li) {
    const int ell = 2 * li;
    const double phase = (li & 1) ? -1.0 : 1.0;  // (-i)^ell for even ell
    for (int a = 0; a < n_k; ++a) {
      const double ka = k_edges[a], kb = k_edges[a + 1];
      const double a3 = ka * ka * ka, b3 = kb * kb * kb;
      const double Ea = E[size_t(li * n_edges + a)], Eb = E[size_t(li * n_edges + a + 1)];
      S[size_t(li * n_k + a)] = 3.0 * (2.0 * ell + 1.0) * phase * (Eb - Ea) / (b3 - a3);
    }
  }
  return S;
}

// diag->l1_mass of the power spectrum: the pair stream enumerated once more and
// swept by the double-precision L1 kernel only.
static void pk_l1_mass(Ctx &c, Timer &tm, const Sorted &s, const Grid &g, const hipster_params *q, double *out) {
  const int n_ell = q->ell_max / 2 + 1, n_edges = q->n_k + 1;
  const double r_split = q->k_edges[0] > 0.0 ? HIPSTER_U_BIG / q->k_edges[0] : 0.0;
  double *edges = upload_edges(c, q->n_k, q->k_edges);
  const int nwaves = pk_sweep_waves(c);
  const int cols = n_ell * q->n_k;
  double *rows = static_cast<double *>(ensure(c, c.pk_l1, size_t(nwaves) * cols * 8));
  HIPSTER_HIP(hipMemsetAsync(rows, 0, size_t(nwaves) * cols * 8, c.stream));
  const PairUnits units = make_pair_units(c, s, g);
  sweep_pair_set(
      c, tm, units.n,
      [&](int64_t *ca, int64_t *cb, unsigned long long *ord) {
        pk_pairs_count(c, s, g, units, q->r0, r_split, ca, cb, ord);
      },
      [&](const int64_t *oa, const int64_t *ob, int64_t ba, int64_t bb, int64_t na, int64_t u0, int64_t u1,
          PkPairs pp) { pk_pairs_write(c, s, g, units, q->r0, r_split, q->los_axis, oa, ob, ba, bb, na, u0, u1, pp); },
      n_ell, true, q->r0, edges, n_edges, false, nullptr, nwaves, rows, false);
  double *merged = static_cast<double *>(ensure(c, c.merged, size_t(cols) * 8));
  merge_partials(c, rows, nwaves, cols, merged);
  HIPSTER_HIP(hipMemcpyAsync(out, merged, size_t(cols) * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
}

static void run_pk(Ctx &c, const hipster_points *pts, const hipster_params *q, double *pk, hipster_diag *diag) {
  check_points(pts, "data", q ? q->box : 0.0);
  check_params(q, false, true);
  if (!pk) throw Error{HIPSTER_EINVAL, "NULL output"};
  if (pts->n < 2) throw Error{HIPSTER_EINVAL, "need at least two points"};
  const int n_c_tab = q->precision == HIPSTER_TABLE ? pktab_default_nodes(q->r0, q->k_edges[q->n_k]) : 0;
  if (q->precision == HIPSTER_TABLE && size_t(q->ell_max / 2 + 1) * size_t(n_c_tab + 3) > ddr2_max_nodes(c))
    throw Error{HIPSTER_EUNSUPPORTED, "table form: k_max R0 too large for the LDS histogram; use HIPSTER_MIXED"};
  HIPSTER_HIP(hipSetDevice(c.device));
  Timer tm(c);
  hipEvent_t t0 = tm.mark();

  const int64_t n = pts->n;
  const size_t esz = pts->dtype == HIPSTER_F32 ? 4 : 8;
  const void *pos = device_view(c, c.pos_in, pts->pos, n * 3 * int64_t(esz), pts->on_device);
  const void *w = device_view(c, c.w_in, pts->w, n * int64_t(esz), pts->on_device);
  const uint8_t *mask = device_mask(c, c.mask_in, q->primary_mask, n);
  const Grid g = make_grid(q->box, q->r0);
  const Sorted s = build_cells(c, c.cells_d, g, pos, w, mask, n, pts->dtype);
  hipEvent_t t1 = tm.mark();

  const int n_ell = q->ell_max / 2 + 1, n_edges = q->n_k + 1;
  if (q->precision == HIPSTER_TABLE) {
    // one histogram sweep of the ordered pairs and its contraction with
    // the jbar table: S^a_l = (2l+1) (-i)^l T^a_l
    unsigned long long *ord = static_cast<unsigned long long *>(ensure(c, c.ordered_count, 8));
    HIPSTER_HIP(hipMemsetAsync(ord, 0, 8, c.stream));
    double *Td = static_cast<double *>(ensure(c, c.pt_T, size_t(n_ell) * q->n_k * 8));
    hipEvent_t ts = tm.mark();
    pktab_sweep(c, s, g, q->r0, q->n_k, q->k_edges, n_ell, q->los_axis, n_c_tab, Td, ord);
    hipEvent_t te = tm.mark();
    std::vector<double> T(size_t(n_ell) * q->n_k);
    unsigned long long ordered = 0;
    HIPSTER_HIP(hipMemcpyAsync(T.data(), Td, T.size() * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipMemcpyAsync(&ordered, ord, 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
    if (diag && diag->l1_mass) pk_l1_mass(c, tm, s, g, q, diag->l1_mass);
    const double p1 = weight_sum(pts);
    const double V = q->box * q->box * q->box, nw = p1 / V, norm = 1.0 / (nw * nw * V);
    std::vector<double> wt(static_cast<size_t>(q->n_k));
    wtilde_bins(c, q->r0, q->n_k, q->k_edges, wt.data());
    for (int li = 0; li < n_ell; ++li)
      for (int a = 0; a < q->n_k; ++a) {
        const double Sa = (4.0 * li + 1.0) * ((li & 1) ? -1.0 : 1.0) * T[size_t(li * q->n_k + a)];
        if (diag && diag->raw) diag->raw[li * q->n_k + a] = Sa;
        pk[li * q->n_k + a] = Sa * norm - (li == 0 ? wt[size_t(a)] : 0.0);
      }
    if (diag) {
      diag->n_pairs = ordered;
      diag->n_pairs_rand = 0;
      diag->n_pairs_rr = 0;
      if (diag->wtilde) memcpy(diag->wtilde, wt.data(), size_t(q->n_k) * 8);
      diag->ms_build = Timer::ms(t0, t1);
      diag->ms_pairs = 0.0;
      diag->ms_sweep = Timer::ms(ts, te);
      diag->ms_total = Timer::ms(t0, te);
      diag->sweep_launches = 1;
      diag->ms_sweep_far = 0.0;
      diag->n_pairs_far = 0;
      diag->eii_nodes = n_c_tab;
    }
    return;
  }
  const bool fp64 = q->precision == HIPSTER_FP64;
  // pairs with r >= U_BIG / k_0 evaluate every edge on the large-argument
  // path (closed form with the Si auxiliaries); the near bucket holds the rest
  const double r_split = q->k_edges[0] > 0.0 ? HIPSTER_U_BIG / q->k_edges[0] : 0.0;
  double *edges = upload_edges(c, q->n_k, q->k_edges);
  const int nwaves = pk_sweep_waves(c);
  const int cols = n_ell * n_edges;
  double *partial = static_cast<double *>(ensure(c, c.partial, size_t(nwaves) * cols * 8));
  HIPSTER_HIP(hipMemsetAsync(partial, 0, size_t(nwaves) * cols * 8, c.stream));
  const PairUnits units = make_pair_units(c, s, g);
  const SweepStats st = sweep_pair_set(
      c, tm, units.n,
      [&](int64_t *ca, int64_t *cb, unsigned long long *ord) {
        pk_pairs_count(c, s, g, units, q->r0, r_split, ca, cb, ord);
      },
      [&](const int64_t *oa, const int64_t *ob, int64_t ba, int64_t bb, int64_t na, int64_t u0, int64_t u1,
          PkPairs pp) { pk_pairs_write(c, s, g, units, q->r0, r_split, q->los_axis, oa, ob, ba, bb, na, u0, u1, pp); },
      n_ell, fp64, q->r0, edges, n_edges, q->k_edges[0] > 0.0, partial, nwaves);
  const std::vector<double> S = bin_sums(c, partial, nwaves, n_ell, q->n_k, q->k_edges);
  hipEvent_t t3 = tm.mark();
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  if (diag && diag->l1_mass) pk_l1_mass(c, tm, s, g, q, diag->l1_mass);

  // finalize (host, FP64): P^a_l = S^a_l / (n_w^2 V) - delta_l0 W~^a
  const double p1 = weight_sum(pts);
  const double V = q->box * q->box * q->box, nw = p1 / V, norm = 1.0 / (nw * nw * V);
  std::vector<double> wt(static_cast<size_t>(q->n_k));
  wtilde_bins(c, q->r0, q->n_k, q->k_edges, wt.data());
  for (int li = 0; li < n_ell; ++li)
    for (int a = 0; a < q->n_k; ++a) {
      const double Sa = S[size_t(li * q->n_k + a)];
      if (diag && diag->raw) diag->raw[li * q->n_k + a] = Sa;
      pk[li * q->n_k + a] = Sa * norm - (li == 0 ? wt[size_t(a)] : 0.0);
    }
  if (diag) {
    diag->n_pairs = st.ordered;
    diag->n_pairs_rand = 0;
    diag->n_pairs_rr = 0;
    if (diag->wtilde) memcpy(diag->wtilde, wt.data(), size_t(q->n_k) * 8);
    diag->ms_build = Timer::ms(t0, t1);
    diag->ms_pairs = st.ms_pairs;
    diag->ms_sweep = st.ms_sweep;
    diag->ms_total = Timer::ms(t0, t3);
    diag->sweep_launches = st.launches;
    diag->ms_sweep_far = st.ms_far;
    diag->n_pairs_far = st.far_pairs;
  }
}

// ------------------------------------------------- survey power spectrum
// Sec. 2 general estimator with the binned kernels of Sec. 3: the DD, DR
// and RR pair sets, each with its signed weight scale, go through the same
// sweep into one set of edge sums, so the result is DD - 2DR + RR.
static void run_pk_survey(Ctx &c, const hipster_points *dp, const hipster_points *rp,
                          const hipster_survey_params *q, double *pk, hipster_diag *diag) {
  check_points(dp, "data", 0.0);
  check_points(rp, "randoms", 0.0);
  if (!q) throw Error{HIPSTER_EINVAL, "NULL parameters"};
  if (!pk) throw Error{HIPSTER_EINVAL, "NULL output"};
  if (dp->n < 1 || rp->n < 1) throw Error{HIPSTER_EINVAL, "survey: need at least one data and one random point"};
  if (!(q->volume > 0.0) || !isfinite(q->volume)) throw Error{HIPSTER_EDOMAIN, "survey: volume must be finite and positive"};
  if (!(q->r0 > 0.0) || !isfinite(q->r0)) throw Error{HIPSTER_EDOMAIN, "R0 must be finite and positive"};
  {
    // the binning and precision checks of the periodic estimator
    hipster_params pp{};
    pp.box = 2.0 * q->r0;
    pp.r0 = q->r0;
    pp.n_k = q->n_k;
    pp.ell_max = q->ell_max;
    pp.k_edges = q->k_edges;
    pp.los_axis = 2;
    pp.precision = q->precision;
    check_params(&pp, false, true);
  }
  HIPSTER_HIP(hipSetDevice(c.device));
  Timer tm(c);
  hipEvent_t t0 = tm.mark();

  const int64_t nd = dp->n, nr = rp->n;
  const size_t ed = dp->dtype == HIPSTER_F32 ? 4 : 8, er = rp->dtype == HIPSTER_F32 ? 4 : 8;
  const void *dpos = device_view(c, c.pos_in, dp->pos, nd * 3 * int64_t(ed), dp->on_device);
  const void *dw = device_view(c, c.w_in, dp->w, nd * int64_t(ed), dp->on_device);
  const void *rpos = device_view(c, c.rpos_in, rp->pos, nr * 3 * int64_t(er), rp->on_device);
  const void *rw = device_view(c, c.rw_in, rp->w, nr * int64_t(er), rp->on_device);
  const uint8_t *dmask = device_mask(c, c.mask_in, q->primary_mask, nd);
  const uint8_t *rmask = device_mask(c, c.rmask_in, q->random_mask, nr);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bounding_box(c, dpos, nd, dp->dtype, lo, hi);
  bounding_box(c, rpos, nr, rp->dtype, lo, hi);
  const Grid g = make_survey_grid(lo, hi, q->r0);
  const Sorted sd = build_cells(c, c.cells_d, g, dpos, dw, dmask, nd, dp->dtype);
  const Sorted sr = build_cells(c, c.cells_r, g, rpos, rw, rmask, nr, rp->dtype);
  hipEvent_t t1 = tm.mark();

  const double p1 = weight_sum(dp), pr1 = weight_sum(rp), sR = p1 / pr1;
  if (q->precision == HIPSTER_TABLE) {
    // DD (+1), DR + RD (-s_R), RR (+s_R^2), each a histogram sweep with its
    // own fixed-point scale, contracted with the jbar table and summed here
    const int n_ell_t = q->ell_max / 2 + 1, n_c = pktab_default_nodes(q->r0, q->k_edges[q->n_k]);
    if (size_t(n_ell_t) * size_t(n_c + 3) > ddr2_max_nodes(c))
      throw Error{HIPSTER_EUNSUPPORTED, "table form: k_max R0 too large for the LDS histogram; use HIPSTER_MIXED"};
    double cb = 0.0;
    for (int d = 0; d < 3; ++d) cb = std::max(cb, std::max(fabs(lo[d]), fabs(hi[d])));
    const size_t nt = size_t(n_ell_t) * q->n_k;
    double *Td = static_cast<double *>(ensure(c, c.pt_T, 3 * nt * 8));
    unsigned long long *ord = static_cast<unsigned long long *>(ensure(c, c.ordered_count, 3 * 8));
    HIPSTER_HIP(hipMemsetAsync(ord, 0, 3 * 8, c.stream));
    hipEvent_t ts = tm.mark();
    pktab_survey_sweep(c, sd, sd, false, g, cb, 1.0, q->r0, q->n_k, q->k_edges, n_ell_t, n_c, Td, ord);
    pktab_survey_sweep(c, sd, sr, true, g, cb, -sR, q->r0, q->n_k, q->k_edges, n_ell_t, n_c, Td + nt, ord + 1);
    pktab_survey_sweep(c, sr, sr, false, g, cb, sR * sR, q->r0, q->n_k, q->k_edges, n_ell_t, n_c, Td + 2 * nt,
                       ord + 2);
    hipEvent_t te = tm.mark();
    std::vector<double> T(3 * nt);
    unsigned long long oc[3] = {0, 0, 0};
    HIPSTER_HIP(hipMemcpyAsync(T.data(), Td, T.size() * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipMemcpyAsync(oc, ord, 3 * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
    const double nw = p1 / q->volume, norm = 1.0 / (nw * nw * q->volume);
    for (int li = 0; li < n_ell_t; ++li)
      for (int a = 0; a < q->n_k; ++a) {
        const size_t i = size_t(li) * q->n_k + a;
        const double Sa = (4.0 * li + 1.0) * ((li & 1) ? -1.0 : 1.0) * ((T[i] + T[nt + i]) + T[2 * nt + i]);
        if (diag && diag->raw) diag->raw[i] = Sa;
        pk[i] = Sa * norm;
      }
    if (diag) {
      diag->n_pairs = oc[0];
      diag->n_pairs_rand = oc[1];
      diag->n_pairs_rr = oc[2];
      diag->ms_build = Timer::ms(t0, t1);
      diag->ms_pairs = 0.0;
      diag->ms_sweep = Timer::ms(ts, te);
      diag->ms_total = Timer::ms(t0, te);
      diag->sweep_launches = 3;
      diag->ms_sweep_far = 0.0;
      diag->n_pairs_far = 0;
      diag->eii_nodes = n_c;
    }
    return;
  }
  const bool fp64 = q->precision == HIPSTER_FP64;
  const double r_split = q->k_edges[0] > 0.0 ? HIPSTER_U_BIG / q->k_edges[0] : 0.0;
  const int n_ell = q->ell_max / 2 + 1, n_edges = q->n_k + 1;
  double *edges = upload_edges(c, q->n_k, q->k_edges);
  const int nwaves = pk_sweep_waves(c);
  const int cols = n_ell * n_edges;
  double *partial = static_cast<double *>(ensure(c, c.partial, size_t(nwaves) * cols * 8));
  HIPSTER_HIP(hipMemsetAsync(partial, 0, size_t(nwaves) * cols * 8, c.stream));
  // DD (+1), DR + RD (-s_R: each (d, r) pair once, weighted by m_d + m_r),
  // RR (+s_R^2)
  struct Set {
    const Sorted *a, *b;
    bool cross;
    double scale;
  } sets[3] = {{&sd, &sd, false, 1.0}, {&sd, &sr, true, -sR}, {&sr, &sr, false, sR * sR}};
  SweepStats st[3];
  for (int k = 0; k < 3; ++k) {
    const Set &z = sets[k];
    const PairUnits units = make_pair_units(c, *z.a, g);
    st[k] = sweep_pair_set(
        c, tm, units.n,
        [&](int64_t *ca, int64_t *cb, unsigned long long *ord) {
          survey_pairs_count(c, *z.a, *z.b, z.cross, g, units, q->r0, r_split, ca, cb, ord);
        },
        [&](const int64_t *oa, const int64_t *ob, int64_t ba, int64_t bb, int64_t na, int64_t u0, int64_t u1,
            PkPairs pp) {
          survey_pairs_write(c, *z.a, *z.b, z.cross, g, units, q->r0, r_split, z.scale, oa, ob, ba, bb, na, u0, u1,
                             pp);
        },
        n_ell, fp64, q->r0, edges, n_edges, q->k_edges[0] > 0.0, partial, nwaves);
  }
  const std::vector<double> S = bin_sums(c, partial, nwaves, n_ell, q->n_k, q->k_edges);
  hipEvent_t t3 = tm.mark();
  HIPSTER_HIP(hipStreamSynchronize(c.stream));

  // P^a_l = S^a_l / (n_w^2 V), n_w = sum(w_data) / V
  const double nw = p1 / q->volume, norm = 1.0 / (nw * nw * q->volume);
  for (int i = 0; i < n_ell * q->n_k; ++i) {
    if (diag && diag->raw) diag->raw[i] = S[size_t(i)];
    pk[i] = S[size_t(i)] * norm;
  }
  if (diag) {
    diag->n_pairs = st[0].ordered;
    diag->n_pairs_rand = st[1].ordered;
    diag->n_pairs_rr = st[2].ordered;
    diag->ms_build = Timer::ms(t0, t1);
    diag->ms_pairs = st[0].ms_pairs + st[1].ms_pairs + st[2].ms_pairs;
    diag->ms_sweep = st[0].ms_sweep + st[1].ms_sweep + st[2].ms_sweep;
    diag->ms_total = Timer::ms(t0, t3);
    diag->sweep_launches = st[0].launches + st[1].launches + st[2].launches;
    diag->ms_sweep_far = st[0].ms_far + st[1].ms_far + st[2].ms_far;
    diag->n_pairs_far = st[0].far_pairs + st[1].far_pairs + st[2].far_pairs;
  }
}

// -------------------------------------------------------------- bispectrum
// E^{II,ab}_l table of the analytic DDR^II term on the device, rebuilt only
// when (R0, n_x, ell_max, edges) change; *ms is its build time (0 if reused).
// The context keeps up to kEiiCacheBytes of tables (so the boxes of a batch,
// each with its own R0, keep theirs across calls); the least recently used
// table goes first.
constexpr size_t kEiiCacheBytes = size_t(2) << 30;

static const double *eii_device_table(Ctx &c, Timer &tm, double r0, int n_k, const double *k, int ell_max, int n_x,
                                      double *ms) {
  std::vector<double> key = {r0, double(n_k), double(ell_max), double(n_x)};
  key.insert(key.end(), k, k + n_k + 1);
  const size_t bytes = size_t(ell_max + 1) * n_k * n_k * (size_t(n_x) + 1) * 8;
  *ms = 0.0;
  ++c.eii_clock;
  for (EiiEntry &e : c.eii_cache)
    if (e.key == key) {
      e.used = c.eii_clock;
      return static_cast<const double *>(e.buf.p);
    }
  // make room: drop least recently used tables until the new one fits
  size_t held = 0;
  for (const EiiEntry &e : c.eii_cache) held += e.buf.cap;
  while (!c.eii_cache.empty() && held + bytes > kEiiCacheBytes) {
    size_t oldest = 0;
    for (size_t i = 1; i < c.eii_cache.size(); ++i)
      if (c.eii_cache[i].used < c.eii_cache[oldest].used) oldest = i;
    held -= c.eii_cache[oldest].buf.cap;
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
    c.mem_used -= c.eii_cache[oldest].buf.cap;
    free_buf(c.eii_cache[oldest].buf);
    c.eii_cache.erase(c.eii_cache.begin() + long(oldest));
  }
  c.eii_cache.push_back(EiiEntry{});
  EiiEntry &ent = c.eii_cache.back();
  double *tab = static_cast<double *>(ensure(c, ent.buf, bytes));
  hipEvent_t e0 = tm.mark();
  eii_table(c, r0, n_k, k, ell_max, n_x, tab);
  hipEvent_t e1 = tm.mark();
  HIPSTER_HIP(hipEventSynchronize(e1));
  *ms = Timer::ms(e0, e1);
  ent.key = key;
  ent.used = c.eii_clock;
  return tab;
}

// Table size of the analytic DDR^II term: n_x = 0 picks the default.
static int check_eii_nodes(Ctx &c, const hipster_params *q, int n_x) {
  if (q->k_edges[q->n_k] * q->r0 > kMaxPhaseMixed)
    throw Error{HIPSTER_EUNSUPPORTED, "analytic DDR^II: the kernel table needs k_max * R0 <= 1e6"};
  if (n_x == 0) n_x = eii_default_nodes(q->r0, q->k_edges[q->n_k]);
  if (n_x < 2 || n_x > kEiiMaxNodes)
    throw Error{HIPSTER_EUNSUPPORTED, "analytic DDR^II: n_x must lie in [2, " + std::to_string(kEiiMaxNodes) + "]"};
  if (size_t(n_x) + 1 > ddr2_max_nodes(c))
    throw Error{HIPSTER_EUNSUPPORTED, "analytic DDR^II: the pair histogram exceeds the device's LDS"};
  return n_x;
}

// analytic_nx < 0: the DDR^II term from the random primaries `rp`;
// otherwise from the E^II kernel with that many table intervals (0: default)
// and no randoms.
// One box's bispectrum call in stages: checks, device inputs, the sweeps, the
// C-term and analytic stages, and the host assembly.  A single call runs them
// in turn on the context's scratch; a batch prepares every box on scratch of
// its own, sweeps all of them in one queued launch, then finishes each.
struct BkBufs {
  CellScratch *cd, *cr;
  DevBuf *pos, *w, *mask, *rpos, *rw, *rmask, *rgen, *edges, *coef, *cnt;
};

struct BkBox {
  const hipster_points *dp = nullptr, *rp = nullptr;
  hipster_points genp{};
  const hipster_params *q = nullptr;
  double *bk = nullptr;
  hipster_diag *diag = nullptr;
  double f_rand = 0.0;
  uint64_t seed = 0;
  int analytic_nx = -1;
  bool analytic = false, have_r = false, gen_r = false, c_hist = false, fp64 = false;
  int64_t n_gen = 0;
  Grid g{};
  Sorted sd, sr;
  const void *pos = nullptr, *w = nullptr;
  const uint8_t *mask = nullptr;
  double *edges = nullptr, *coef = nullptr;
  unsigned long long *cnt = nullptr;  // [data pairs, random (or 2 R0) pairs, C-term pairs]
  BkSums sums[2];
  std::vector<double> Ch[2], T;
  unsigned long long hcnt[2] = {0, 0};
  double ms_build = 0.0, ms_sweep = 0.0, ms_cterm = 0.0, ms_table = 0.0, ms_ddr2 = 0.0;
  hipEvent_t ev_b0 = nullptr, ev_b1 = nullptr;  // around the preparation (read after the last sync)
  uint64_t launches = 0;
};

static void bk_check(Ctx &c, BkBox &x) {
  const hipster_params *q = x.q;
  check_points(x.dp, "data", q ? q->box : 0.0);
  check_params(q, true);
  if (!x.bk) throw Error{HIPSTER_EINVAL, "NULL output"};
  if (x.dp->n < 2) throw Error{HIPSTER_EINVAL, "need at least two points"};
  x.analytic = x.analytic_nx >= 0;
  if (x.analytic) {
    if (q->n_k > kEiiMaxNkApi)
      throw Error{HIPSTER_EUNSUPPORTED, "analytic DDR^II: n_k must lie in [1, " + std::to_string(kEiiMaxNkApi) + "]"};
    x.analytic_nx = check_eii_nodes(c, q, x.analytic_nx);
  }
  const bool given_r = !x.analytic && x.rp && x.rp->n > 0;
  if (given_r) check_points(x.rp, "randoms", q->box);
  if (!given_r) x.rp = nullptr;
  x.gen_r = !x.analytic && !given_r;
  if (x.gen_r) {
    if (!(x.f_rand > 0.0) || !isfinite(x.f_rand))
      throw Error{HIPSTER_EINVAL,
                  "bispectrum: no random catalogue and f_rand <= 0; the DDR^II term needs random primaries "
                  "(or use hipster_bk_ell_analytic)"};
    const double want = std::llround(x.f_rand * double(x.dp->n));
    if (want < 1.0 || want > 2147483647.0) throw Error{HIPSTER_EINVAL, "bispectrum: f_rand * N must round into [1, 2^31)"};
    x.n_gen = int64_t(want);
  }
  x.have_r = given_r || x.gen_r;
  x.fp64 = q->precision == HIPSTER_FP64;
  // the mixed form takes C from the C-term pair histogram (exact window,
  // tabulated jbar^a jbar^b); the FP64 form sums C in the pair sweep
  x.c_hist = !x.fp64;
}

// Randoms (drawn on the device when not given), cell lists, edges and 1/bin
// volumes, zeroed pair counters.
static void bk_prepare(Ctx &c, Timer &tm, BkBox &x, const BkBufs &b) {
  const hipster_params *q = x.q;
  x.ev_b0 = tm.mark();
  if (x.gen_r) {
    double *gp = static_cast<double *>(ensure(c, *b.rgen, size_t(x.n_gen) * 24));
    random_points(c, x.seed, x.n_gen, q->box, gp);
    x.genp = hipster_points{};
    x.genp.n = x.n_gen;
    x.genp.dtype = HIPSTER_F64;
    x.genp.on_device = 1;
    x.genp.pos = gp;
    x.genp.w = nullptr;
    x.rp = &x.genp;
  }
  const int64_t n = x.dp->n;
  const size_t esz = x.dp->dtype == HIPSTER_F32 ? 4 : 8;
  x.pos = device_view(c, *b.pos, x.dp->pos, n * 3 * int64_t(esz), x.dp->on_device);
  x.w = device_view(c, *b.w, x.dp->w, n * int64_t(esz), x.dp->on_device);
  x.mask = device_mask(c, *b.mask, q->primary_mask, n);
  x.g = make_grid(q->box, q->r0);
  x.sd = build_cells(c, *b.cd, x.g, x.pos, x.w, x.mask, n, x.dp->dtype);
  if (x.have_r) {
    const int64_t nr = x.rp->n;
    const size_t rsz = x.rp->dtype == HIPSTER_F32 ? 4 : 8;
    const void *rpos = device_view(c, *b.rpos, x.rp->pos, nr * 3 * int64_t(rsz), x.rp->on_device);
    const void *rw = device_view(c, *b.rw, x.rp->w, nr * int64_t(rsz), x.rp->on_device);
    const uint8_t *rmask = device_mask(c, *b.rmask, q->random_mask, nr);
    x.sr = build_cells(c, *b.cr, x.g, rpos, rw, rmask, nr, x.rp->dtype);
  }
  const int NK = q->n_k;
  std::vector<double> coef(static_cast<size_t>(NK));
  for (int a = 0; a < NK; ++a) {
    const double ka = q->k_edges[a], kb = q->k_edges[a + 1];
    coef[size_t(a)] = 3.0 / (kb * kb * kb - ka * ka * ka);
  }
  x.edges = static_cast<double *>(ensure(c, *b.edges, size_t(NK + 1) * 8));
  x.coef = static_cast<double *>(ensure(c, *b.coef, size_t(NK) * 8));
  HIPSTER_HIP(hipMemcpyAsync(x.edges, q->k_edges, size_t(NK + 1) * 8, hipMemcpyHostToDevice, c.stream));
  HIPSTER_HIP(hipMemcpyAsync(x.coef, coef.data(), size_t(NK) * 8, hipMemcpyHostToDevice, c.stream));
  x.cnt = static_cast<unsigned long long *>(ensure(c, *b.cnt, 24));
  HIPSTER_HIP(hipMemsetAsync(x.cnt, 0, 24, c.stream));
  x.ev_b1 = tm.mark();
}

// The sweep jobs of a box: data primaries, then random primaries if any.
static int bk_jobs(const BkBox &x, std::vector<BkQueueJob> &out) {
  const int sets = x.have_r ? 2 : 1;
  for (int set = 0; set < sets; ++set) {
    BkQueueJob j;
    j.prim = set == 0 ? x.sd : x.sr;
    j.sec = x.sd;
    j.g = x.g;
    j.r0 = x.q->r0;
    j.self_set = set == 0;
    j.edges = x.edges;
    j.coef = x.coef;
    j.NK = x.q->n_k;
    j.npairs = x.cnt + set;
    // expected pairs per primary, n (4 pi / 3) R0^3: the same for both sets of a box
    const double V = x.q->box * x.q->box * x.q->box;
    j.cost = double(x.dp->n) / V * (4.0 * kPi / 3.0) * x.q->r0 * x.q->r0 * x.q->r0;
    out.push_back(j);
  }
  return sets;
}

// The sweeps of a single box.
static void bk_sweeps(Ctx &c, Timer &tm, BkBox &x) {
  for (int set = 0; set < (x.have_r ? 2 : 1); ++set) {
    const Sorted &prim = set == 0 ? x.sd : x.sr;
    bk_sweep(c, prim, x.sd, x.g, x.q->r0, set == 0, x.edges, x.coef, x.q->n_k, x.q->ell_max, x.fp64, !x.c_hist,
             x.cnt + set, x.sums[set]);
    // the sweep kernels alone (the quads and their order are built before)
    x.ms_sweep += x.sums[set].ms_kernel;
    x.launches += x.sums[set].launches;
  }
}

// After the sweeps: C of the data primaries (Ch[0]) and of the random
// primaries (Ch[1]) from the pair histogram (mixed form), the analytic DDR^II
// stage (the kernel table, then every data pair inside 2 R0 on a grid of cells
// >= 2 R0, the data re-sorted into the randoms' scratch), the pair counts.
static void bk_finish_device(Ctx &c, Timer &tm, BkBox &x, const BkBufs &b) {
  const hipster_params *q = x.q;
  const int NK = q->n_k, NL = q->ell_max + 1;
  if (x.c_hist) {
    hipEvent_t c0 = tm.mark();
    const int rows = NL * NK * NK;
    double *Cd = static_cast<double *>(ensure(c, c.ct_C, size_t(2 * rows) * 8));
    unsigned long long n_ord[2] = {0, 0};
    HIPSTER_HIP(hipMemcpyAsync(n_ord, x.cnt, 16, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
    const int n_c = cterm_default_nodes(q->r0, q->k_edges[NK]);
    for (int set = 0; set < (x.have_r ? 2 : 1); ++set) {
      cterm_sweep(c, set == 0 ? x.sd : x.sr, x.sd, set == 1, x.g, q->r0, NK, q->k_edges, q->ell_max, n_c,
                  n_ord[set], Cd + size_t(set) * rows, x.cnt + 2);
      x.Ch[set].resize(size_t(rows));
      HIPSTER_HIP(hipMemcpyAsync(x.Ch[set].data(), Cd + size_t(set) * rows, size_t(rows) * 8,
                                 hipMemcpyDeviceToHost, c.stream));
    }
    hipEvent_t c1 = tm.mark();
    if (c1) HIPSTER_HIP(hipEventSynchronize(c1));
    else HIPSTER_HIP(hipStreamSynchronize(c.stream));
    x.ms_cterm += Timer::ms(c0, c1);
  }
  if (x.analytic) {
    const double *tab = eii_device_table(c, tm, q->r0, NK, q->k_edges, q->ell_max, x.analytic_nx, &x.ms_table);
    hipEvent_t d0 = tm.mark();
    const Grid g2 = make_grid(q->box, 2.0 * q->r0);
    const Sorted s2 = build_cells(c, *b.cr, g2, x.pos, x.w, x.mask, x.dp->n, x.dp->dtype);
    const int rows = NL * NK * NK;
    double *Td = static_cast<double *>(ensure(c, c.ddr2_T, size_t(rows) * 8));
    ddr2_sweep(c, s2, g2, q->r0, x.analytic_nx, tab, rows, Td, x.cnt + 1);
    x.T.resize(size_t(rows));
    HIPSTER_HIP(hipMemcpyAsync(x.T.data(), Td, size_t(rows) * 8, hipMemcpyDeviceToHost, c.stream));
    hipEvent_t d1 = tm.mark();
    if (d1) HIPSTER_HIP(hipEventSynchronize(d1));
    x.ms_ddr2 += Timer::ms(d0, d1);
  }
  HIPSTER_HIP(hipMemcpyAsync(x.hcnt, x.cnt, 16, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
}

// Assembly (Sec. 4 summary estimator), host FP64.
static void bk_assemble(Ctx &c, BkBox &x) {
  x.ms_build = Timer::ms(x.ev_b0, x.ev_b1);
  const hipster_params *q = x.q;
  hipster_diag *diag = x.diag;
  double *bk = x.bk;
  const int NK = q->n_k, NL = q->ell_max + 1;
  const bool analytic = x.analytic, have_r = x.have_r, c_hist = x.c_hist;
  const BkSums *sums = x.sums;
  const std::vector<double> *Ch = x.Ch;
  const std::vector<double> &T = x.T;
  const double p1 = weight_sum(x.dp), pr = have_r ? (x.gen_r ? double(x.n_gen) : weight_sum(x.rp)) : 0.0;
  const double V = q->box * q->box * q->box, nw = p1 / V, sR = have_r ? p1 / pr : 0.0;
  std::vector<double> wt(static_cast<size_t>(NK));
  wtilde_bins(c, q->r0, NK, q->k_edges, wt.data());
  // S0 from the data primaries' A_00 sums: sum_q w_q W jbar_0 = A_00 / y_00
  constexpr double kInvY00 = 3.5449077018110320546;  // 2 sqrt(pi)
  std::vector<double> S0(static_cast<size_t>(NK));
  for (int b = 0; b < NK; ++b) S0[size_t(b)] = sums[0].S0[size_t(b)] * kInvY00;
  for (int l = 0; l < NL; ++l)
    for (int a = 0; a < NK; ++a)
      for (int b = 0; b < NK; ++b) {
        const size_t o = (size_t(l) * NK + a) * NK + b;
        const size_t tc = (size_t(l) * NK + std::min(a, b)) * NK + std::max(a, b);
        const double GD = sums[0].G[o];
        const double CD = c_hist ? Ch[0][tc] : sums[0].C[o];
        // the random-primary term s_R (G_R - C_R) estimates n_w T, T = sum_{i!=j} w_i w_j E^II
        const double GR = analytic ? T[tc] : (have_r ? sums[1].G[o] : 0.0);
        const double CR = analytic ? 0.0 : (have_r ? (c_hist ? Ch[1][tc] : sums[1].C[o]) : 0.0);
        const double sgn = (l & 1) ? -1.0 : 1.0;
        const double ddr2 = analytic ? nw * GR : sR * (GR - CR);
        double v = sgn * (2.0 * l + 1.0) / (V * nw * nw * nw) * ((GD - CD) - ddr2);
        if (l == 0) v += -(wt[size_t(a)] * S0[size_t(b)] + wt[size_t(b)] * S0[size_t(a)]) / (V * nw * nw) +
                         2.0 * wt[size_t(a)] * wt[size_t(b)];
        bk[o] = v;
        if (diag && diag->l1_mass) {
          auto sq = [&](auto get) { return sqrt(fabs(get(a, a)) * fabs(get(b, b))); };
          const double sGD = sq([&](int x, int y) { return sums[0].G[(size_t(l) * NK + x) * NK + y]; });
          const double sCD = sq([&](int x, int y) {
            return c_hist ? Ch[0][(size_t(l) * NK + std::min(x, y)) * NK + std::max(x, y)]
                          : sums[0].C[(size_t(l) * NK + x) * NK + y];
          });
          double sR2 = 0.0;
          if (analytic) {
            sR2 = nw * fabs(GR);
          } else if (have_r) {
            const double sGR = sq([&](int x, int y) { return sums[1].G[(size_t(l) * NK + x) * NK + y]; });
            const double sCR = sq([&](int x, int y) {
              return c_hist ? Ch[1][(size_t(l) * NK + std::min(x, y)) * NK + std::max(x, y)]
                            : sums[1].C[(size_t(l) * NK + x) * NK + y];
            });
            sR2 = sR * (sGR + sCR);
          }
          double m = (2.0 * l + 1.0) / (V * nw * nw * nw) * (sGD + sCD + sR2);
          if (l == 0)
            m += (wt[size_t(a)] * fabs(S0[size_t(b)]) + wt[size_t(b)] * fabs(S0[size_t(a)])) / (V * nw * nw) +
                 2.0 * fabs(wt[size_t(a)] * wt[size_t(b)]);
          diag->l1_mass[o] = m;
        }
        if (diag) {
          if (diag->gd) diag->gd[o] = GD;
          if (diag->cd) diag->cd[o] = CD;
          if (diag->gr) diag->gr[o] = GR;
          if (diag->cr) diag->cr[o] = CR;
        }
      }
  if (diag) {
    if (diag->s0)
      for (int b = 0; b < NK; ++b) diag->s0[b] = S0[size_t(b)];
    if (diag->wtilde) memcpy(diag->wtilde, wt.data(), size_t(NK) * 8);
    diag->n_pairs = x.hcnt[0];
    diag->n_pairs_rr = 0;
    diag->n_pairs_rand = analytic ? 0 : x.hcnt[1];
    diag->n_rand = have_r ? uint64_t(x.rp->n) : 0;
    diag->ms_build = x.ms_build;
    diag->ms_pairs = 0.0;  // enumeration is fused into the sweep
    diag->ms_sweep = x.ms_sweep;
    diag->sweep_launches = x.launches;
    diag->ms_sweep_far = 0.0;
    diag->n_pairs_far = 0;
    diag->ms_eii_table = x.ms_table;
    diag->ms_ddr2 = x.ms_ddr2;
    diag->n_pairs_2r0 = analytic ? x.hcnt[1] : 0;
    diag->eii_nodes = analytic ? x.analytic_nx : 0;
    diag->ms_cterm = x.ms_cterm;
  }
}


static void run_bk(Ctx &c, const hipster_points *dp, const hipster_points *rp, double f_rand, uint64_t seed,
                   const hipster_params *q, double *bk, hipster_diag *diag, int analytic_nx = -1) {
  BkBox x;
  x.dp = dp;
  x.rp = rp;
  x.q = q;
  x.bk = bk;
  x.diag = diag;
  x.f_rand = f_rand;
  x.seed = seed;
  x.analytic_nx = analytic_nx;
  bk_check(c, x);
  HIPSTER_HIP(hipSetDevice(c.device));
  Timer tm(c);
  hipEvent_t t0 = tm.mark();
  const BkBufs b{&c.cells_d, &c.cells_r, &c.pos_in, &c.w_in, &c.mask_in, &c.rpos_in, &c.rw_in,
                 &c.rmask_in, &c.rgen, &c.edges, &c.bk_coef, &c.ordered_count};
  bk_prepare(c, tm, x, b);
  bk_sweeps(c, tm, x);
  bk_finish_device(c, tm, x, b);
  hipEvent_t t3 = tm.mark();
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  bk_assemble(c, x);
  if (diag) diag->ms_total = Timer::ms(t0, t3);
}
// ------------------------------------------------- anisotropic bispectrum
// Legendre coefficients q[c][L], L = 0 .. 2 ell_max, of
//   Q_c(mu) = sum_{mu' = +-m} y_{l1 mu'} y_{l2 mu'} = (2 - delta_m0) N_{l1 m} N_{l2 m} P^m_{l1}(mu) P^m_{l2}(mu)
// (real orthonormal harmonics about z; the azimuth drops out), by 32-point
// Gauss-Legendre quadrature, exact for these polynomials of degree <= 2 ell_max.
static void aniso_qcoef(int ell_max, const std::vector<int> &cl1, const std::vector<int> &cl2,
                        const std::vector<int> &cm, std::vector<double> &q) {
  const int nc = int(cl1.size()), ns = 2 * ell_max + 1;
  constexpr int NG = 32;
  double xg[NG], wg[NG];
  for (int i = 0; i < NG; ++i) {  // Newton on P_NG from the Chebyshev guess
    double x = cos(kPi * (i + 0.75) / (NG + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int n = 2; n <= NG; ++n) {
        const double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
        p0 = p1;
        p1 = p2;
      }
      dp = NG * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    xg[i] = x;
    wg[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  // associated Legendre P^m_l without the Condon-Shortley phase (it cancels in Q)
  auto plm = [](int l, int m, double x) {
    double pmm = 1.0;
    const double sx = sqrt(std::max(0.0, 1.0 - x * x));
    for (int i = 1; i <= m; ++i) pmm *= (2.0 * i - 1.0) * sx;
    if (l == m) return pmm;
    double p1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return p1;
    double p0 = pmm;
    for (int n = m + 2; n <= l; ++n) {
      const double p2 = ((2.0 * n - 1.0) * x * p1 - (n + m - 1.0) * p0) / (n - m);
      p0 = p1;
      p1 = p2;
    }
    return p1;
  };
  auto norm = [](int l, int m) {
    double r = 1.0;
    for (int i = l - m + 1; i <= l + m; ++i) r /= double(i);
    return sqrt((2.0 * l + 1.0) / (4.0 * kPi) * r);
  };
  q.assign(size_t(nc) * ns, 0.0);
  for (int c = 0; c < nc; ++c) {
    const int l1 = cl1[size_t(c)], l2 = cl2[size_t(c)], m = cm[size_t(c)];
    const double f = (m == 0 ? 1.0 : 2.0) * norm(l1, m) * norm(l2, m);
    for (int L = 0; L < ns; ++L) {
      double acc = 0.0;
      for (int i = 0; i < NG; ++i) acc += wg[i] * f * plm(l1, m, xg[i]) * plm(l2, m, xg[i]) * plm(L, 0, xg[i]);
      q[size_t(c) * ns + L] = 0.5 * (2.0 * L + 1.0) * acc;
    }
  }
}

// B^{ab}_{l1 l2 m} about the line of sight z (the reading of Sec. 10 in the
// header): the sweep's G and T sums, the C term from the Legendre-section
// histograms, and the assembly of the Sec. 4 summary estimator with the
// harmonic products of different order.
static void run_bk_aniso(Ctx &c, const hipster_points *dp, const hipster_points *rp, double f_rand, uint64_t seed,
                         const hipster_params *q, double *bk, hipster_diag *diag) {
  BkBox x;
  x.dp = dp;
  x.rp = rp;
  x.q = q;
  x.bk = bk;
  x.diag = nullptr;
  x.f_rand = f_rand;
  x.seed = seed;
  bk_check(c, x);
  if (x.fp64)
    throw Error{HIPSTER_EUNSUPPORTED, "anisotropic bispectrum: the mixed form only (its C term is tabulated)"};
  if (q->n_k > 16) throw Error{HIPSTER_EUNSUPPORTED, "anisotropic bispectrum: n_k must lie in [1, 16]"};
  if (q->ell_max > 4) throw Error{HIPSTER_EUNSUPPORTED, "anisotropic bispectrum: ell_max must lie in [0, 4]"};
  HIPSTER_HIP(hipSetDevice(c.device));
  Timer tm(c);
  hipEvent_t t0 = tm.mark();
  const BkBufs b{&c.cells_d, &c.cells_r, &c.pos_in, &c.w_in, &c.mask_in, &c.rpos_in, &c.rw_in,
                 &c.rmask_in, &c.rgen, &c.edges, &c.bk_coef, &c.ordered_count};
  bk_prepare(c, tm, x, b);
  const int NK = q->n_k, NL = q->ell_max + 1;
  std::vector<int> cl1, cl2, cm;
  for (int l1 = 0; l1 < NL; ++l1)
    for (int l2 = l1; l2 < NL; ++l2)
      for (int m = 0; m <= l1; ++m) {
        cl1.push_back(l1);
        cl2.push_back(l2);
        cm.push_back(m);
      }
  const int NC = int(cl1.size());
  std::vector<double> G[2], T[2], C[2];
  double ms_sw = 0.0;
  for (int set = 0; set < 2; ++set)
    bk_aniso_sweep(c, set == 0 ? x.sd : x.sr, x.sd, x.g, q->r0, set == 0, x.edges, x.coef, NK, q->ell_max,
                   x.cnt + set, G[set], T[set], ms_sw);
  unsigned long long n_ord[2] = {0, 0};
  HIPSTER_HIP(hipMemcpyAsync(n_ord, x.cnt, 16, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  std::vector<double> qc;
  aniso_qcoef(q->ell_max, cl1, cl2, cm, qc);
  const int n_c = cterm_default_nodes(q->r0, q->k_edges[NK]);
  hipEvent_t c0 = tm.mark();
  for (int set = 0; set < 2; ++set) {
    C[set].resize(size_t(NC) * NK * NK);
    cterm_aniso_sweep(c, set == 0 ? x.sd : x.sr, x.sd, set == 1, x.g, q->r0, NK, q->k_edges, q->ell_max, n_c,
                      n_ord[set], NC, cl1.data(), cl2.data(), qc.data(), C[set].data(), x.cnt + 2);
  }
  hipEvent_t c1 = tm.mark();
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  // assembly, host FP64
  const double p1 = weight_sum(dp), pr = x.gen_r ? double(x.n_gen) : weight_sum(x.rp);
  const double V = q->box * q->box * q->box, nw = p1 / V, sR = p1 / pr;
  std::vector<double> wt(static_cast<size_t>(NK));
  wtilde_bins(c, q->r0, NK, q->k_edges, wt.data());
  const double sq4pi = sqrt(4.0 * kPi);
  for (int ci = 0; ci < NC; ++ci) {
    const int l1 = cl1[size_t(ci)], l2 = cl2[size_t(ci)], m = cm[size_t(ci)], L = l1 + l2;
    // the real factor of (-i)^{l1 + l2}
    const double sgn = ((((L & 1) ? (L - 1) / 2 : L / 2) & 1) != 0) ? -1.0 : 1.0;
    for (int a = 0; a < NK; ++a)
      for (int bb = 0; bb < NK; ++bb) {
        const size_t o = (size_t(ci) * NK + a) * NK + bb;
        double v = sgn * 4.0 * kPi / (V * nw * nw * nw) * ((G[0][o] - C[0][o]) - sR * (G[1][o] - C[1][o]));
        if (m == 0) {
          double d1 = 0.0;
          if (l2 == 0) d1 += wt[size_t(bb)] * T[0][size_t(l1) * NK + a];
          if (l1 == 0) d1 += wt[size_t(a)] * T[0][size_t(l2) * NK + bb];
          v -= sgn * sq4pi / (V * nw * nw) * d1;
          if (l1 == 0 && l2 == 0) v += 2.0 * wt[size_t(a)] * wt[size_t(bb)];
        }
        bk[o] = v;
      }
  }
  if (diag) {
    unsigned long long hcnt[2] = {0, 0};
    HIPSTER_HIP(hipMemcpy(hcnt, x.cnt, 16, hipMemcpyDeviceToHost));
    diag->n_pairs = hcnt[0];
    diag->n_pairs_rand = hcnt[1];
    diag->n_pairs_rr = 0;
    diag->n_rand = uint64_t(x.rp->n);
    diag->ms_build = Timer::ms(x.ev_b0, x.ev_b1);
    diag->ms_pairs = 0.0;
    diag->ms_sweep = ms_sw;
    diag->ms_cterm = Timer::ms(c0, c1);
    diag->ms_total = Timer::ms(t0, c1);
    diag->sweep_launches = 2;
    diag->ms_sweep_far = 0.0;
    diag->n_pairs_far = 0;
    if (diag->wtilde) memcpy(diag->wtilde, wt.data(), size_t(NK) * 8);
  }
}

// ------------------------------------------------------------ autotuner
std::string tune_key(Ctx &c, const char *kernel, std::initializer_list<int> shape) {
  hipDeviceProp_t prop{};
  std::string dev = "device";
  if (hipGetDeviceProperties(&prop, c.device) == hipSuccess)
    dev = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
  std::string k = kernel;
  for (int v : shape) k += ":" + std::to_string(v);
  // no spaces: one whitespace-separated (key, value) pair per line
  for (char &ch : dev)
    if (ch == ' ') ch = '_';
  return k + "@" + dev;
}

int tune_lookup(Ctx &c, const std::string &key) {
  if (!c.tune_file_read) {
    c.tune_file_read = true;
    if (const char *path = getenv("HIPSTER_TUNE_CACHE")) {
      if (FILE *f = fopen(path, "r")) {
        char kbuf[512];
        int v = 0;
        while (fscanf(f, "%511s %d", kbuf, &v) == 2)
          if (v > 0) c.tune[kbuf] = v;
        fclose(f);
      }
    }
  }
  auto it = c.tune.find(key);
  return it == c.tune.end() ? 0 : it->second;
}

void tune_store(Ctx &c, const std::string &key, int value) {
  c.tune[key] = value;
  if (const char *path = getenv("HIPSTER_TUNE_CACHE")) {
    if (FILE *f = fopen(path, "a")) {
      fprintf(f, "%s %d\n", key.c_str(), value);
      fclose(f);
    }
  }
}

// Arguments of the theory-side calls: R0 > 0, n_k in [1, 128], strictly
// increasing non-negative edges, ell_max in [0, 6] (even when `even`).
static void check_theory(double r0, int n_k, const double *k_edges, int ell_max, bool even) {
  if (!k_edges) throw Error{HIPSTER_EINVAL, "NULL k_edges"};
  if (!(r0 > 0.0) || !isfinite(r0)) throw Error{HIPSTER_EDOMAIN, "R0 must be finite and positive"};
  if (n_k < 1 || n_k > kMaxNk) throw Error{HIPSTER_EUNSUPPORTED, "n_k must lie in [1, 128]"};
  for (int a = 0; a <= n_k; ++a) {
    if (!isfinite(k_edges[a]) || k_edges[a] < 0.0) throw Error{HIPSTER_EDOMAIN, "k edges must be finite and >= 0"};
    if (a > 0 && !(k_edges[a] > k_edges[a - 1])) throw Error{HIPSTER_EDOMAIN, "k edges must increase strictly"};
  }
  if (ell_max < 0 || ell_max > kLMaxApi || (even && (ell_max & 1)))
    throw Error{HIPSTER_EDOMAIN, even ? "ell_max must be even, <= 6" : "ell_max must lie in [0, 6]"};
}

// The table sine and cosine reduce exactly only below ~1.6e6: max(p, k) R0.
static void theory_phase_check(double r0, int n_k, const double *k_edges, int n_p, const double *p) {
  double m = k_edges[n_k];
  for (int i = 0; i < n_p; ++i) m = std::max(m, p[i]);
  if (m * r0 > kMaxPhaseMixed) throw Error{HIPSTER_EUNSUPPORTED, "theory: max(p, k_max) * R0 must be <= 1e6"};
}

// E^{II,ab}_l on the nodes m 2 R0 / n_x, copied to the host.
static void run_eii_table(Ctx &c, double r0, int32_t n_k, const double *k_edges, int32_t ell_max, int32_t n_x,
                          double *out) {
  if (!out || !k_edges) throw Error{HIPSTER_EINVAL, "NULL argument"};
  hipster_params q{};
  q.box = 2.0 * r0;
  q.r0 = r0;
  q.n_k = n_k;
  q.ell_max = ell_max;
  q.k_edges = k_edges;
  q.precision = HIPSTER_FP64;
  check_params(&q, true);
  if (n_x < 2) throw Error{HIPSTER_EUNSUPPORTED, "E^II table: n_x must be >= 2"};
  HIPSTER_HIP(hipSetDevice(c.device));
  n_x = check_eii_nodes(c, &q, n_x);
  Timer tm(c);
  double ms = 0.0;
  const double *tab = eii_device_table(c, tm, r0, n_k, k_edges, ell_max, n_x, &ms);
  const size_t bytes = size_t(ell_max + 1) * n_k * n_k * (size_t(n_x) + 1) * 8;
  HIPSTER_HIP(hipMemcpyAsync(out, tab, bytes, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
}

// ------------------------------------------------------------------ batch
// Power spectra of many boxes through one work-queue sweep per filled pair
// stream; bispectra box by box on the same stream.
static void run_batch(Ctx &c, int nb, hipster_box_job *jobs, hipster_diag *diag) {
  if (nb < 1 || !jobs) throw Error{HIPSTER_EINVAL, "batch: need n_boxes >= 1 and a job array"};
  int pk_prec = -1, ne_max = 1, cols_edges = 0;
  for (int b = 0; b < nb; ++b) {
    const hipster_box_job &j = jobs[b];
    check_points(&j.data, "batch data", j.pk_params.box);
    if (j.data.n < 2) throw Error{HIPSTER_EINVAL, "batch: every box needs at least two points"};
    if (j.pk_params.n_k > 0) {
      check_params(&j.pk_params, false);
      if (!j.pk) throw Error{HIPSTER_EINVAL, "batch: NULL pk output"};
      if (pk_prec >= 0 && j.pk_params.precision != pk_prec)
        throw Error{HIPSTER_EINVAL, "batch: all power spectra must share one precision"};
      pk_prec = j.pk_params.precision;
      ne_max = std::max(ne_max, j.pk_params.ell_max / 2 + 1);
      cols_edges = std::max(cols_edges, j.pk_params.n_k + 1);
    }
    if (j.bk_params.n_k > 0) {
      check_params(&j.bk_params, true);
      if (!j.bk) throw Error{HIPSTER_EINVAL, "batch: NULL bk output"};
      if (j.bk_eii_nodes < 0 && j.randoms.n > 0) check_points(&j.randoms, "batch randoms", j.bk_params.box);
      if (j.bk_eii_nodes < 0 && j.randoms.n <= 0 && (!(j.f_rand > 0.0) || !isfinite(j.f_rand)))
        throw Error{HIPSTER_EINVAL, "batch: a bispectrum box needs randoms, f_rand > 0 or bk_eii_nodes >= 0"};
    }
  }
  HIPSTER_HIP(hipSetDevice(c.device));
  Timer tm(c);
  hipEvent_t t0 = tm.mark();
  double ms_pairs = 0.0, ms_sweep = 0.0, ms_build = 0.0;
  uint64_t launches = 0;

  // boxes with a power spectrum, largest expected pair count first; a box
  // with more than kBatchOwnPairs expected pairs takes the single-box path
  // (near and far kernels over its own stream) after the shared queue
  constexpr double kBatchOwnPairs = double(int64_t(1) << 25);
  std::vector<int> order, own;
  auto pairs_expected = [&](int b) {
    const hipster_params &q = jobs[b].pk_params;
    const double n = double(jobs[b].data.n), V = q.box * q.box * q.box;
    return 0.5 * n * n / V * (4.0 * kPi / 3.0) * q.r0 * q.r0 * q.r0;
  };
  for (int b = 0; b < nb; ++b) {
    if (jobs[b].pk_params.n_k <= 0) continue;
    if (pairs_expected(b) > kBatchOwnPairs) own.push_back(b);
    else order.push_back(b);
  }
  auto cost = [&](int b) { return pairs_expected(b) * double(jobs[b].pk_params.n_k + 1); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });

  const int cols = ne_max * std::max(cols_edges, 1);
  const bool fp64 = pk_prec == HIPSTER_FP64;
  const int64_t cap = pair_chunk_capacity();
  const int64_t task_pairs = int64_t(1) << 16;
  const int nwaves = pk_sweep_waves(c);
  // per-box constants and packed edges
  std::vector<BoxSweep> hbox(static_cast<size_t>(nb));
  std::vector<double> hedges;
  for (int b = 0; b < nb; ++b) {
    const hipster_params &q = jobs[b].pk_params;
    hbox[size_t(b)] = BoxSweep{q.n_k > 0 ? 1.0 / q.r0 : 0.0, int(hedges.size()), q.n_k > 0 ? q.n_k + 1 : 0};
    for (int e = 0; q.n_k > 0 && e <= q.n_k; ++e) hedges.push_back(q.k_edges[e]);
  }
  BoxSweep *dbox = static_cast<BoxSweep *>(ensure(c, c.bt_boxes, hbox.size() * sizeof(BoxSweep)));
  double *dedges = static_cast<double *>(ensure(c, c.edges, std::max<size_t>(hedges.size(), 1) * 8));
  double *dout = static_cast<double *>(ensure(c, c.bt_out, size_t(nb) * cols * 8));
  int *counter = static_cast<int *>(ensure(c, c.bt_counter, 16));
  HIPSTER_HIP(hipMemcpyAsync(dbox, hbox.data(), hbox.size() * sizeof(BoxSweep), hipMemcpyHostToDevice, c.stream));
  if (!hedges.empty())
    HIPSTER_HIP(hipMemcpyAsync(dedges, hedges.data(), hedges.size() * 8, hipMemcpyHostToDevice, c.stream));
  HIPSTER_HIP(hipMemsetAsync(dout, 0, size_t(nb) * cols * 8, c.stream));

  PkPairs pp;
  pp.r = static_cast<double *>(ensure(c, c.pr, size_t(cap) * 8));
  pp.mu = ensure(c, c.pmu, size_t(cap) * 8);
  pp.ww = ensure(c, c.pww, size_t(cap) * 8);
  std::vector<PkTask> tasks;
  std::vector<int> task_box_first;
  int64_t fill = 0;
  std::vector<uint64_t> ordered(static_cast<size_t>(nb), 0);
  // write-pass event pairs, read once the stream has drained (no host wait
  // per chunk)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> write_marks;

  auto flush = [&]() {
    if (tasks.empty()) return;
    // tasks are grouped by box in the order the boxes were written
    std::vector<int> first(static_cast<size_t>(nb) + 1, 0);
    std::vector<PkTask> sorted;
    sorted.reserve(tasks.size());
    for (int b = 0; b < nb; ++b) {
      first[size_t(b)] = int(sorted.size());
      for (const PkTask &t : tasks)
        if (t.box == b) sorted.push_back(t);
    }
    first[size_t(nb)] = int(sorted.size());
    // queue order: largest boxes' tasks first (LPT), rows indexed by queue slot
    std::vector<PkTask> queue;
    std::vector<int> qfirst(static_cast<size_t>(nb) + 1, 0);
    std::vector<int> box_pos(static_cast<size_t>(nb), 0);
    int pos = 0;
    for (int b : order) {
      box_pos[size_t(b)] = pos;
      pos += first[size_t(b) + 1] - first[size_t(b)];
    }
    queue.resize(sorted.size());
    for (int b = 0; b < nb; ++b)
      for (int t = first[size_t(b)]; t < first[size_t(b) + 1]; ++t) queue[size_t(box_pos[size_t(b)] + t - first[size_t(b)])] = sorted[size_t(t)];
    PkTask *dtasks = static_cast<PkTask *>(ensure(c, c.bt_tasks, queue.size() * sizeof(PkTask)));
    double *rows = static_cast<double *>(ensure(c, c.bt_rows, queue.size() * size_t(cols) * 8));
    HIPSTER_HIP(hipMemcpyAsync(dtasks, queue.data(), queue.size() * sizeof(PkTask), hipMemcpyHostToDevice, c.stream));
    HIPSTER_HIP(hipMemsetAsync(counter, 0, 4, c.stream));
    hipEvent_t a = tm.mark();
    pk_sweep_tasks(c, pp, dtasks, int(queue.size()), counter, dedges, dbox, cols, rows, ne_max, fp64, nwaves);
    hipEvent_t d = tm.mark();
    // rows of box b are queue slots [box_pos[b], box_pos[b] + n_b): merge each box's range
    std::vector<int> mfirst(static_cast<size_t>(nb) * 2);
    for (int b = 0; b < nb; ++b) {
      mfirst[size_t(2 * b)] = box_pos[size_t(b)];
      mfirst[size_t(2 * b + 1)] = box_pos[size_t(b)] + first[size_t(b) + 1] - first[size_t(b)];
    }
    int *dfirst = static_cast<int *>(ensure(c, c.bt_first, mfirst.size() * 4));
    HIPSTER_HIP(hipMemcpyAsync(dfirst, mfirst.data(), mfirst.size() * 4, hipMemcpyHostToDevice, c.stream));
    merge_boxes(c, rows, cols, dfirst, nb, dout);
    HIPSTER_HIP(hipEventSynchronize(d));
    ms_sweep += Timer::ms(a, d);
    ++launches;
    tasks.clear();
    fill = 0;
  };

  for (int b : order) {
    const hipster_box_job &j = jobs[b];
    const hipster_params &q = j.pk_params;
    const int64_t n = j.data.n;
    const size_t esz = j.data.dtype == HIPSTER_F32 ? 4 : 8;
    hipEvent_t a0 = tm.mark();
    const void *pos = device_view(c, c.pos_in, j.data.pos, n * 3 * int64_t(esz), j.data.on_device);
    const void *w = device_view(c, c.w_in, j.data.w, n * int64_t(esz), j.data.on_device);
    const uint8_t *mask = device_mask(c, c.mask_in, q.primary_mask, n);
    const Grid g = make_grid(q.box, q.r0);
    const Sorted s = build_cells(c, c.cells_d, g, pos, w, mask, n, j.data.dtype);
    const PairUnits units = make_pair_units(c, s, g);
    hipEvent_t a1 = tm.mark();
    const int64_t ncells = units.n;  // work units (home-cell tiles) of this box
    const double r_split = q.k_edges[0] > 0.0 ? HIPSTER_U_BIG / q.k_edges[0] : 0.0;
    int64_t *cnt_a = static_cast<int64_t *>(ensure(c, c.pair_cnt, size_t(ncells) * 8));
    int64_t *cnt_b = static_cast<int64_t *>(ensure(c, c.pair_cnt_b, size_t(ncells) * 8));
    int64_t *off_a = static_cast<int64_t *>(ensure(c, c.pair_off, size_t(ncells + 1) * 8));
    int64_t *off_b = static_cast<int64_t *>(ensure(c, c.pair_off_b, size_t(ncells + 1) * 8));
    unsigned long long *ord = static_cast<unsigned long long *>(ensure(c, c.ordered_count, 16));
    HIPSTER_HIP(hipMemsetAsync(ord, 0, 8, c.stream));
    pk_pairs_count(c, s, g, units, q.r0, r_split, cnt_a, cnt_b, ord);
    scan_i64(c, cnt_a, off_a, ncells, c.pair_total);
    scan_i64(c, cnt_b, off_b, ncells, c.pair_total);
    std::vector<int64_t> ha(static_cast<size_t>(ncells) + 1), hb(static_cast<size_t>(ncells) + 1);
    unsigned long long hord = 0;
    HIPSTER_HIP(hipMemcpyAsync(ha.data(), off_a, size_t(ncells + 1) * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipMemcpyAsync(hb.data(), off_b, size_t(ncells + 1) * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipMemcpyAsync(&hord, ord, 8, hipMemcpyDeviceToHost, c.stream));
    hipEvent_t a2 = tm.mark();
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
    ms_build += Timer::ms(a0, a1);
    ms_pairs += Timer::ms(a1, a2);
    ordered[size_t(b)] = hord;
    int64_t c0 = 0;
    while (c0 < ncells) {
      // largest cell range that fits the remaining stream
      int64_t c1 = c0;
      auto in = [&](int64_t x, int64_t y) { return (ha[size_t(y)] - ha[size_t(x)]) + (hb[size_t(y)] - hb[size_t(x)]); };
      while (c1 < ncells && in(c0, c1 + 1) <= cap - fill) ++c1;
      if (c1 == c0) {
        if (fill > 0) {
          flush();
          continue;
        }
        throw Error{HIPSTER_EUNSUPPORTED, "batch: one cell tile holds more pairs than the pair stream"};
      }
      const int64_t np = in(c0, c1), n_a = ha[size_t(c1)] - ha[size_t(c0)];
      if (np > 0) {
        hipEvent_t w0 = tm.mark();
        // shift the bases so the cells' pairs land at [fill, fill + np)
        pk_pairs_write(c, s, g, units, q.r0, r_split, q.los_axis, off_a, off_b, ha[size_t(c0)] - fill,
                       hb[size_t(c0)] - fill,
                       n_a, c0, c1, pp);
        hipEvent_t w1 = tm.mark();
        write_marks.push_back({w0, w1});
        for (int64_t t0p = fill; t0p < fill + np; t0p += task_pairs)
          tasks.push_back(PkTask{t0p, std::min(fill + np, t0p + task_pairs), b, 0});
        fill += np;
      }
      c0 = c1;
    }
  }
  flush();
  std::vector<double> E(static_cast<size_t>(nb) * cols);
  HIPSTER_HIP(hipMemcpyAsync(E.data(), dout, E.size() * 8, hipMemcpyDeviceToHost, c.stream));
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  for (const auto &wm : write_marks) ms_pairs += Timer::ms(wm.first, wm.second);
  for (int b : order) {
    hipster_box_job &j = jobs[b];
    const hipster_params &q = j.pk_params;
    const int n_ell = q.ell_max / 2 + 1, n_edges = q.n_k + 1;
    const double p1 = weight_sum(&j.data);
    const double V = q.box * q.box * q.box, nw = p1 / V, norm = 1.0 / (nw * nw * V);
    std::vector<double> wt(static_cast<size_t>(q.n_k));
    wtilde_bins(c, q.r0, q.n_k, q.k_edges, wt.data());
    const double *Eb = E.data() + size_t(b) * cols;
    for (int li = 0; li < n_ell; ++li) {
      const int ell = 2 * li;
      const double phase = (li & 1) ? -1.0 : 1.0;
      for (int a = 0; a < q.n_k; ++a) {
        const double ka = q.k_edges[a], kb = q.k_edges[a + 1];
        const double a3 = ka * ka * ka, b3 = kb * kb * kb;
        const double S = 3.0 * (2.0 * ell + 1.0) * phase * (b3 * Eb[li * n_edges + a + 1] - a3 * Eb[li * n_edges + a]) / (b3 - a3);
        j.pk[li * q.n_k + a] = S * norm - (ell == 0 ? wt[size_t(a)] : 0.0);
      }
    }
    j.n_pairs = ordered[size_t(b)];
  }
  for (int b : own) {
    hipster_box_job &j = jobs[b];
    hipster_diag d{};
    run_pk(c, &j.data, &j.pk_params, j.pk, &d);
    ms_build += d.ms_build;
    ms_pairs += d.ms_pairs;
    ms_sweep += d.ms_sweep;
    launches += d.sweep_launches;
    j.n_pairs = d.n_pairs;
  }
  // bispectra: every box prepared on scratch of its own, the sweeps of all
  // boxes that share (ell_max, form) in one queued launch (boxes with more
  // than 16 bins sweep alone), then each box's C-term or analytic stage and
  // its assembly
  std::vector<int> bb;
  for (int b = 0; b < nb; ++b)
    if (jobs[b].bk_params.n_k > 0) bb.push_back(b);
  if (!bb.empty()) {
    const size_t nbk = bb.size();
    if (c.bt_bk.size() < nbk) c.bt_bk.resize(nbk);
    std::vector<BkBox> xs(nbk);
    std::vector<hipster_diag> ds(nbk);
    std::vector<BkBufs> bufs(nbk);
    for (size_t i = 0; i < nbk; ++i) {
      hipster_box_job &j = jobs[bb[i]];
      BkBox &x = xs[i];
      ds[i] = hipster_diag{};
      x.dp = &j.data;
      x.rp = j.bk_eii_nodes >= 0 ? nullptr : (j.randoms.n > 0 ? &j.randoms : nullptr);
      x.q = &j.bk_params;
      x.bk = j.bk;
      x.diag = &ds[i];
      x.f_rand = j.f_rand;
      x.seed = j.seed;
      x.analytic_nx = j.bk_eii_nodes >= 0 ? j.bk_eii_nodes : -1;
      bk_check(c, x);
      BkBoxScratch &sc = c.bt_bk[i];
      bufs[i] = BkBufs{&sc.cd, &sc.cr, &sc.pos, &sc.w, &sc.mask, &sc.rpos, &sc.rw, &sc.rmask, &sc.rgen, &sc.edges,
                       &sc.coef, &sc.cnt};
    }
    for (size_t i = 0; i < nbk; ++i) bk_prepare(c, tm, xs[i], bufs[i]);
    std::map<std::pair<int, int>, std::vector<size_t>> classes;
    for (size_t i = 0; i < nbk; ++i) {
      if (xs[i].q->n_k <= 16) classes[{xs[i].q->ell_max, xs[i].fp64 ? 1 : 0}].push_back(i);
      else bk_sweeps(c, tm, xs[i]);
    }
    for (const auto &cl : classes) {
      std::vector<BkQueueJob> qj;
      std::vector<std::pair<size_t, int>> owner;
      for (size_t i : cl.second) {
        const int n = bk_jobs(xs[i], qj);
        for (int set = 0; set < n; ++set) owner.push_back({i, set});
      }
      std::vector<BkSums> res;
      hipEvent_t a = tm.mark();
      bk_sweep_queue(c, qj, cl.first.first, cl.first.second != 0, res);
      hipEvent_t d = tm.mark();
      if (d) HIPSTER_HIP(hipEventSynchronize(d));
      ms_sweep += Timer::ms(a, d);
      ++launches;
      for (size_t k = 0; k < owner.size(); ++k) xs[owner[k].first].sums[owner[k].second] = std::move(res[k]);
    }
    for (size_t i = 0; i < nbk; ++i) {
      bk_finish_device(c, tm, xs[i], bufs[i]);
      bk_assemble(c, xs[i]);
      ms_build += xs[i].ms_build;
      ms_sweep += xs[i].ms_sweep;
      launches += xs[i].launches;
      hipster_box_job &j = jobs[bb[i]];
      if (j.pk_params.n_k <= 0) j.n_pairs = ds[i].n_pairs;
    }
  }
  hipEvent_t t9 = tm.mark();
  HIPSTER_HIP(hipStreamSynchronize(c.stream));
  if (diag) {
    diag->n_pairs_rr = 0;
    diag->ms_build = ms_build;
    diag->ms_pairs = ms_pairs;
    diag->ms_sweep = ms_sweep;
    diag->ms_total = Timer::ms(t0, t9);
    diag->sweep_launches = launches;
    diag->ms_sweep_far = 0.0;
    diag->n_pairs_far = 0;
  }
}

template <class F>
static hipster_status guarded(hipster_ctx *ctx, F &&f) {
  if (!ctx) return HIPSTER_EINVAL;
  try {
    f();
    ctx->c.last_error.clear();
    return HIPSTER_OK;
  } catch (const Error &e) {
    ctx->c.last_error = e.msg;
    if (e.status == HIPSTER_EHIP) (void)hipGetLastError();
    return e.status;
  } catch (const std::exception &e) {
    ctx->c.last_error = e.what();
    return HIPSTER_ENOMEM;
  }
}

// ------------------------------------------------ no-allocation workspace
// Device scratch of hipster_pk_ell_noalloc: a static array that each device
// holds from the code object's load until the process ends.  In host code the
// array's name is not a device address: hipster_create looks up the calling
// device's copy once with hipGetSymbolAddress and the entry point passes that
// pointer on.  Every call on one device shares its copy, so calls that overlap
// on a device race; each call clears what its kernels need zeroed.
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kScratchDevices];

// With `device` current, record its copy of the workspace (once per device).
static hipster_status scratch_setup(int device) {
  if (device < 0 || device >= kScratchDevices) return HIPSTER_OK;  // the entry point reports it
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return HIPSTER_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return HIPSTER_EHIP;
  }
  g_scratch_ptr[device] = static_cast<unsigned char *>(p);
  return HIPSTER_OK;
}

static unsigned char *scratch_of(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// hipster_pk_ell with every device buffer carved from the workspace: a
// context of its own (device, stream and the measured kernel parameters of
// the caller's context) in workspace mode, discarded afterwards without
// freeing anything.
static void run_pk_noalloc(Ctx &parent, const hipster_points *pts, const hipster_params *q, double *pk,
                           hipster_diag *diag) {
  if (diag && diag->l1_mass)
    throw Error{HIPSTER_EUNSUPPORTED, "diag->l1_mass is not available from hipster_pk_ell_noalloc"};
  unsigned char *ws = scratch_of(parent.device);
  if (!ws) throw Error{HIPSTER_EUNSUPPORTED, "no static workspace on this device"};
  Ctx w;
  w.device = parent.device;
  w.stream = parent.stream;
  w.tune = parent.tune;
  w.tune_file_read = parent.tune_file_read;
  w.arena = ws;
  w.arena_cap = kScratchBytes;
  run_pk(w, pts, q, pk, diag);
}

}  // namespace hipster

using namespace hipster;

extern "C" {

hipster_status hipster_create(hipster_ctx **out, int device, void *hip_stream) {
  if (!out) return HIPSTER_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return HIPSTER_EHIP;
  }
  if (hipSetDevice(device) != hipSuccess) return HIPSTER_EHIP;
  if (scratch_setup(device) != HIPSTER_OK) return HIPSTER_EHIP;
  hipster_ctx *h = new (std::nothrow) hipster_ctx();
  if (!h) return HIPSTER_ENOMEM;
  h->c.device = device;
  h->c.stream = static_cast<hipStream_t>(hip_stream);
  *out = h;
  return HIPSTER_OK;
}

void hipster_destroy(hipster_ctx *ctx) {
  if (!ctx) return;
  Ctx &c = ctx->c;
  (void)hipSetDevice(c.device);
  (void)hipStreamSynchronize(c.stream);
  free_cells(c.cells_d);
  free_cells(c.cells_r);
  DevBuf *all[] = {&c.pos_in, &c.w_in, &c.mask_in, &c.rpos_in, &c.rw_in, &c.rmask_in, &c.pair_cnt, &c.pair_cnt_b,
                   &c.pair_ord, &c.pair_off, &c.pair_off_b, &c.pair_total, &c.pr, &c.pmu, &c.pww, &c.pux, &c.puy, &c.puz, &c.edges,
                   &c.partial, &c.merged, &c.ordered_count, &c.bbox, &c.bk_partial, &c.bk_partial_r, &c.bk_coef, &c.bq_count, &c.bq_off, &c.bq_scan, &c.bq_quads, &c.bk_abuf, &c.bk_wbuf, &c.bk_tiles, &c.bk_gpart, &c.bk_gmerged, &c.bt_tasks, &c.bt_boxes, &c.bt_counter, &c.bt_rows, &c.bt_first, &c.bt_out,
                   &c.unit_tiles, &c.unit_base, &c.unit_cell, &c.unit_tile, &c.eii_consts,
                   &c.ddr2_partial, &c.ddr2_hist, &c.ddr2_counter, &c.ddr2_T, &c.ct_tab, &c.ct_consts, &c.ct_C,
                   &c.ct_wmax, &c.ct_jbar, &c.ct_sel, &c.rgen, &c.pk_l1, &c.th_r, &c.th_w, &c.th_p, &c.th_wp, &c.th_pk, &c.th_ek, &c.th_g, &c.th_J, &c.th_om,
                   &c.th_K, &c.th_out, &c.th_wt, &c.th_pb, &c.th_bk, &c.th_T, &c.th_X, &c.pt_tab, &c.pt_consts,
                   &c.pt_T, &c.bq_jobs, &c.bq_tasks, &c.bq_slots, &c.bq_counter,
                   &c.bo_cnt, &c.bo_key, &c.bo_key2, &c.bo_iota, &c.bo_perm, &c.bo_tmp,
                   &c.ca_q, &c.ca_l, &c.ca_count, &c.ca_out, &c.ca_tab,
                   &c.tune_scratch};
  for (DevBuf *b : all) free_buf(*b);
  for (BkBoxScratch &s : c.bt_bk) {
    free_cells(s.cd);
    free_cells(s.cr);
    DevBuf *own[] = {&s.pos, &s.w, &s.mask, &s.rpos, &s.rw, &s.rmask, &s.rgen, &s.edges, &s.coef, &s.cnt};
    for (DevBuf *b : own) free_buf(*b);
  }
  for (EiiEntry &e : c.eii_cache) free_buf(e.buf);
  delete ctx;
}

hipster_status hipster_pk_ell(hipster_ctx *ctx, const hipster_points *pts, const hipster_params *prm, double *pk,
                              hipster_diag *diag) {
  return guarded(ctx, [&] { run_pk(ctx->c, pts, prm, pk, diag); });
}

hipster_status hipster_pk_ell_noalloc(hipster_ctx *ctx, const hipster_points *pts, const hipster_params *prm,
                                      double *pk, hipster_diag *diag) {
  return guarded(ctx, [&] { run_pk_noalloc(ctx->c, pts, prm, pk, diag); });
}

hipster_status hipster_pk_survey(hipster_ctx *ctx, const hipster_points *data, const hipster_points *randoms,
                                 const hipster_survey_params *prm, double *pk, hipster_diag *diag) {
  return guarded(ctx, [&] { run_pk_survey(ctx->c, data, randoms, prm, pk, diag); });
}

hipster_status hipster_bk_ell(hipster_ctx *ctx, const hipster_points *data, const hipster_points *randoms,
                              double f_rand, uint64_t seed, const hipster_params *prm, double *bk,
                              hipster_diag *diag) {
  return guarded(ctx, [&] { run_bk(ctx->c, data, randoms, f_rand, seed, prm, bk, diag); });
}

hipster_status hipster_bk_aniso(hipster_ctx *ctx, const hipster_points *data, const hipster_points *randoms,
                                double f_rand, uint64_t seed, const hipster_params *prm, double *bk,
                                hipster_diag *diag) {
  return guarded(ctx, [&] { run_bk_aniso(ctx->c, data, randoms, f_rand, seed, prm, bk, diag); });
}

hipster_status hipster_bk_ell_analytic(hipster_ctx *ctx, const hipster_points *data, const hipster_params *prm,
                                       int32_t n_x, double *bk, hipster_diag *diag) {
  if (n_x < 0) return HIPSTER_EINVAL;
  return guarded(ctx, [&] { run_bk(ctx->c, data, nullptr, 0.0, 0, prm, bk, diag, n_x); });
}

hipster_status hipster_eii_table(hipster_ctx *ctx, double r0, int32_t n_k, const double *k_edges, int32_t ell_max,
                                 int32_t n_x, double *table) {
  return guarded(ctx, [&] { run_eii_table(ctx->c, r0, n_k, k_edges, ell_max, n_x, table); });
}

hipster_status hipster_omega(hipster_ctx *ctx, double r0, int32_t n_k, const double *k_edges, int32_t ell_max,
                             int32_t n_p, const double *p, double *out) {
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    check_theory(r0, n_k, k_edges, ell_max, false);
    if (!p || !out) throw Error{HIPSTER_EINVAL, "NULL argument"};
    if (n_p < 1) throw Error{HIPSTER_EINVAL, "n_p must be >= 1"};
    for (int i = 0; i < n_p; ++i)
      if (!(p[i] >= 0.0) || !isfinite(p[i])) throw Error{HIPSTER_EDOMAIN, "p must be finite and >= 0"};
    theory_phase_check(r0, n_k, k_edges, n_p, p);
    HIPSTER_HIP(hipSetDevice(c.device));
    const int n_l = ell_max + 1;
    double *om = static_cast<double *>(ensure(c, c.th_om, size_t(n_l) * n_p * n_k * 8));
    theory_omega(c, r0, n_k, k_edges, n_l, 1, n_p, p, om);
    HIPSTER_HIP(hipMemcpyAsync(out, om, size_t(n_l) * n_p * n_k * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
  });
}

hipster_status hipster_pk_window_theory(hipster_ctx *ctx, double r0, int32_t n_k, const double *k_edges,
                                        int32_t ell_max, int32_t n_r, const double *r, const double *wr,
                                        const double *xi, double *out) {
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    check_theory(r0, n_k, k_edges, ell_max, true);
    if (!r || !wr || !xi || !out) throw Error{HIPSTER_EINVAL, "NULL argument"};
    if (n_r < 1) throw Error{HIPSTER_EINVAL, "n_r must be >= 1"};
    for (int m = 0; m < n_r; ++m)
      if (!(r[m] >= 0.0) || !(r[m] <= r0)) throw Error{HIPSTER_EDOMAIN, "r nodes must lie in [0, R0]"};
    HIPSTER_HIP(hipSetDevice(c.device));
    const int n_l = ell_max / 2 + 1;
    double *od = static_cast<double *>(ensure(c, c.th_out, size_t(n_l) * n_k * 8));
    theory_pk(c, r0, n_k, k_edges, n_l, n_r, r, wr, xi, od);
    HIPSTER_HIP(hipMemcpyAsync(out, od, size_t(n_l) * n_k * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
  });
}

hipster_status hipster_cov_gauss(hipster_ctx *ctx, double r0, double volume, int32_t n_k, const double *k_edges,
                                 int32_t ell_max, int32_t n_p, const double *p, const double *wp, const double *pk,
                                 double *out) {
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    check_theory(r0, n_k, k_edges, ell_max, true);
    if (!p || !wp || !pk || !out) throw Error{HIPSTER_EINVAL, "NULL argument"};
    if (n_p < 1) throw Error{HIPSTER_EINVAL, "n_p must be >= 1"};
    if (!(volume > 0.0) || !isfinite(volume)) throw Error{HIPSTER_EDOMAIN, "volume must be finite and positive"};
    for (int i = 0; i < n_p; ++i)
      if (!(p[i] >= 0.0) || !isfinite(p[i])) throw Error{HIPSTER_EDOMAIN, "p must be finite and >= 0"};
    theory_phase_check(r0, n_k, k_edges, n_p, p);
    HIPSTER_HIP(hipSetDevice(c.device));
    const int n_l = ell_max / 2 + 1;
    const size_t nout = size_t(n_l) * n_k * n_l * n_k;
    double *od = static_cast<double *>(ensure(c, c.th_out, nout * 8));
    theory_cov(c, r0, volume, n_k, k_edges, n_l, n_p, p, wp, pk, od);
    HIPSTER_HIP(hipMemcpyAsync(out, od, nout * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
  });
}

hipster_status hipster_cov_poisson2(hipster_ctx *ctx, double r0, double nbar, double volume, int32_t n_k,
                                    const double *k_edges, int32_t ell_max, int32_t n_r, const double *r,
                                    const double *wr, const double *xi, double *out) {
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    check_theory(r0, n_k, k_edges, ell_max, true);
    if (!r || !wr || !xi || !out) throw Error{HIPSTER_EINVAL, "NULL argument"};
    if (n_r < 1) throw Error{HIPSTER_EINVAL, "n_r must be >= 1"};
    if (!(nbar > 0.0) || !isfinite(nbar)) throw Error{HIPSTER_EDOMAIN, "density must be finite and positive"};
    if (!(volume > 0.0) || !isfinite(volume)) throw Error{HIPSTER_EDOMAIN, "volume must be finite and positive"};
    for (int m = 0; m < n_r; ++m)
      if (!(r[m] >= 0.0) || !(r[m] <= r0)) throw Error{HIPSTER_EDOMAIN, "r nodes must lie in [0, R0]"};
    HIPSTER_HIP(hipSetDevice(c.device));
    const int n_l = ell_max / 2 + 1;
    const size_t nout = size_t(n_l) * n_k * n_l * n_k;
    double *od = static_cast<double *>(ensure(c, c.th_out, nout * 8));
    theory_c2(c, r0, nbar, volume, n_k, k_edges, n_l, n_r, r, wr, xi, od);
    HIPSTER_HIP(hipMemcpyAsync(out, od, nout * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
  });
}

hipster_status hipster_cov_poisson3(hipster_ctx *ctx, double r0, double nbar, double volume, int32_t n_k,
                                    const double *k_edges, int32_t ell_max, int32_t n_p, const double *p,
                                    const double *wp, const double *pk, const double *pbin, const double *bk,
                                    double *out) {
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    check_theory(r0, n_k, k_edges, ell_max, true);
    if (!p || !wp || !pk || !out) throw Error{HIPSTER_EINVAL, "NULL argument"};
    if (n_p < 1) throw Error{HIPSTER_EINVAL, "n_p must be >= 1"};
    if (!(nbar > 0.0) || !isfinite(nbar)) throw Error{HIPSTER_EDOMAIN, "density must be finite and positive"};
    if (!(volume > 0.0) || !isfinite(volume)) throw Error{HIPSTER_EDOMAIN, "volume must be finite and positive"};
    for (int i = 0; i < n_p; ++i)
      if (!(p[i] >= 0.0) || !isfinite(p[i])) throw Error{HIPSTER_EDOMAIN, "p must be finite and >= 0"};
    theory_phase_check(r0, n_k, k_edges, n_p, p);
    HIPSTER_HIP(hipSetDevice(c.device));
    const int n_l = ell_max / 2 + 1;
    std::vector<double> wt(static_cast<size_t>(n_k));
    wtilde_bins(c, r0, n_k, k_edges, wt.data());
    const size_t nout = size_t(n_l) * n_k * n_l * n_k;
    double *od = static_cast<double *>(ensure(c, c.th_out, nout * 8));
    theory_c3(c, r0, nbar, volume, n_k, k_edges, n_l, n_p, p, wp, pk, wt.data(), pbin, bk, od);
    HIPSTER_HIP(hipMemcpyAsync(out, od, nout * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
  });
}

hipster_status hipster_cov_nongauss(hipster_ctx *ctx, double r0, double volume, int32_t n_k, const double *k_edges,
                                    int32_t ell_max, int32_t n_p, const double *p, const double *wp,
                                    const double *tbar, double *out) {
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    check_theory(r0, n_k, k_edges, ell_max, true);
    if (!p || !wp || !tbar || !out) throw Error{HIPSTER_EINVAL, "NULL argument"};
    if (n_p < 1) throw Error{HIPSTER_EINVAL, "n_p must be >= 1"};
    if (!(volume > 0.0) || !isfinite(volume)) throw Error{HIPSTER_EDOMAIN, "volume must be finite and positive"};
    for (int i = 0; i < n_p; ++i)
      if (!(p[i] >= 0.0) || !isfinite(p[i])) throw Error{HIPSTER_EDOMAIN, "p must be finite and >= 0"};
    theory_phase_check(r0, n_k, k_edges, n_p, p);
    HIPSTER_HIP(hipSetDevice(c.device));
    const int n_l = ell_max / 2 + 1;
    const size_t nout = size_t(n_l) * n_k * n_l * n_k;
    double *od = static_cast<double *>(ensure(c, c.th_out, nout * 8));
    theory_ng(c, r0, volume, n_k, k_edges, n_l, n_p, p, wp, tbar, od);
    HIPSTER_HIP(hipMemcpyAsync(out, od, nout * 8, hipMemcpyDeviceToHost, c.stream));
    HIPSTER_HIP(hipStreamSynchronize(c.stream));
  });
}

hipster_status hipster_batch(hipster_ctx *ctx, int n_boxes, hipster_box_job *jobs, hipster_diag *diag) {
  return guarded(ctx, [&] { run_batch(ctx->c, n_boxes, jobs, diag); });
}

hipster_status hipster_wtilde(double r0, int32_t n_k, const double *k_edges, double *out) {
  if (!k_edges || !out || n_k < 1) return HIPSTER_EINVAL;
  if (!(r0 > 0.0) || !isfinite(r0)) return HIPSTER_EDOMAIN;
  for (int a = 0; a <= n_k; ++a) {
    if (!isfinite(k_edges[a]) || k_edges[a] < 0.0) return HIPSTER_EDOMAIN;
    if (a > 0 && !(k_edges[a] > k_edges[a - 1])) return HIPSTER_EDOMAIN;
  }
  for (int a = 0; a < n_k; ++a) out[a] = wtilde_bin(r0, k_edges[a], k_edges[a + 1]);
  return HIPSTER_OK;
}

hipster_status hipster_set_memory_cap(hipster_ctx *ctx, uint64_t bytes) {
  if (!ctx) return HIPSTER_EINVAL;
  ctx->c.mem_cap = bytes;
  return HIPSTER_OK;
}

const char *hipster_last_error(const hipster_ctx *ctx) {
  if (!ctx) return "NULL context";
  return ctx->c.last_error.c_str();
}

const char *hipster_status_string(hipster_status s) {
  switch (s) {
    case HIPSTER_OK: return "HIPSTER_OK";
    case HIPSTER_EINVAL: return "HIPSTER_EINVAL";
    case HIPSTER_EDOMAIN: return "HIPSTER_EDOMAIN";
    case HIPSTER_EOUTOFBOX: return "HIPSTER_EOUTOFBOX";
    case HIPSTER_ENOMEM: return "HIPSTER_ENOMEM";
    case HIPSTER_EHIP: return "HIPSTER_EHIP";
    case HIPSTER_EUNSUPPORTED: return "HIPSTER_EUNSUPPORTED";
  }
  return "HIPSTER_UNKNOWN";
}

}  // extern "C"
