// Host side of the slpic C ABI (include/slpic.h): validation, the derived
// per-instance constants, the device workspace layout, launches and graph
// capture, and the host readers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/slpic.h"
#include "slpic_internal.hpp"

namespace slpic {
template <typename R> hipError_t launch_particles(const Ctx<R>&, int, hipStream_t);
template <typename R> hipError_t launch_tail(const Ctx<R>&, int, hipStream_t);
template <typename R>
hipError_t launch_seed(const Ctx<R>&, int, int, int64_t, double, uint32_t, hipStream_t);
template <typename R> hipError_t occupancy_gen(int*, size_t, bool, int);
// dynamic LDS of the particle kernel: tile offsets of the (instance,
// species) pairs
inline size_t gen_lds_bytes(int n_inst) { return ((size_t)(2 * n_inst + 1) * 4 + 15) & ~size_t(15); }
// dynamic LDS of the cell sort's count (arrays = 1) and scatter (2) kernels:
// the tail kernel's dynamic LDS: a double per node (charge, then its sums),
// then for each species a float per node and one more (deposit, then its
// prefix sums)
inline int tail_lds_bytes(int max_cells) {
  return (max_cells + 1) * (int)sizeof(double) + 2 * (max_cells + 2) * (int)sizeof(float);
}
// the tile offsets, then arrays of max_cells words
inline size_t sort_lds_bytes(int n_inst, int max_cells, int arrays) {
  return ((size_t)(2 * n_inst + 1 + 3) & ~size_t(3)) * 4 + (size_t)arrays * max_cells * 4;
}
template <typename R> hipError_t launch_sort(const Ctx<R>&, hipStream_t);
hipError_t launch_philox_test(const uint32_t*, uint32_t, uint32_t, int64_t, uint32_t*,
                              hipStream_t);
hipError_t static_workspace(int dev, char** ptr);
}  // namespace slpic

using namespace slpic;

namespace {

constexpr double kQE = 1.602176634e-19;
constexpr double kKB = 1.380649e-23;
constexpr double kME = 9.1093837015e-31;
constexpr double kMAR = 39.948 * 1.66053906660e-27;
constexpr double kTorr = 101325.0 / 760.0;

thread_local std::string g_create_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// channels per row of the particle kernel's cross-section table
int row_channels(int n_chan) { return n_chan <= 4 ? 4 : MAX_CHAN; }

// Integer form of a per-step probability: with u = (2m + 1) 2^-24 for the
// 23-bit integer m = r >> 9, u < P holds exactly for m < ceil((P 2^24 - 1)/2).
uint32_t prob_threshold(double P) {
  if (!(P > 0.0)) return 0u;
  if (P >= 1.0) return 1u << 23;
  double t = std::ceil((P * 16777216.0 - 1.0) * 0.5);
  if (t < 0) t = 0;
  if (t > 8388608.0) t = 8388608.0;
  return (uint32_t)t;
}

// Weight splitting (Sec. III) is on for a split fraction strictly between 0
// and 1; 0 and 1 collide whole markers.
bool splitting(const slpic_config* cfg) { return cfg->split_frac > 0.0 && cfg->split_frac < 1.0; }

struct Layout {
  size_t ip, st, counts, tiles, cross, flux, ev, maxw, acc, E, E64, phi, rho, ring, inst_err, sort_hist, sort_cur,
      glob, xs_e, xs_sig, xs_thr, xs_kind;
  size_t blk[2][2];      // [buffer][species] chunk arrays of the markers
  size_t wt[2][2];       // [buffer][species] marker flux weights (splitting), or 0
  size_t total;
  int total_nodes, max_tiles;
  int64_t total_cap;
  std::vector<int> node, parts;
  std::vector<int64_t> seg, cap_p;
};

// Output partitions of an instance (a power of two): enough that the
// per-emit compaction counters are spread over several addresses for large
// instances, while every partition keeps room for at least 32 tiles, so that
// the random spread of emits over partitions stays small against a
// partition's capacity.  Each partition gets an equal share of the capacity
// plus one tile of slack.
static_assert(MAX_PART == SLPIC_MAX_PARTITIONS, "partition cap of the public header");
static_assert(STATIC_WS_BYTES == SLPIC_STATIC_WORKSPACE_BYTES,
              "static workspace size of the public header");

int partitions_for(int64_t cap) {
  int p = 1;
  while (p < MAX_PART && (int64_t)p * 2 * 32 * BLOCK <= cap) p *= 2;
  return p;
}

bool make_layout(const slpic_config* cfg, const slpic_instance* inst, int n_inst,
                 const slpic_xs* xs, Layout& L) {
  const size_t rs = cfg->precision == 64 ? 8 : 4;
  L.node.resize(n_inst);
  L.seg.resize(n_inst);
  L.parts.resize(n_inst);
  L.cap_p.resize(n_inst);
  int nodes = 0;
  int64_t cap = 0, tiles = 0;
  for (int i = 0; i < n_inst; ++i) {
    L.node[i] = nodes;
    nodes += inst[i].cells + 1;
    const int P = partitions_for(inst[i].capacity);
    // partitions start on marker-chunk boundaries
    int64_t cp = (inst[i].capacity + P - 1) / P + (P > 1 ? BLOCK : 0);
    cp = (cp + CH - 1) / CH * CH;
    // the kernels address a partition's slots by 32-bit byte offsets
    if (cp / CH * (int64_t)(CH * (4 + 4 * rs + 8)) > 0x7fffffffll) return false;
    L.parts[i] = P;
    L.cap_p[i] = cp;
    L.seg[i] = cap;
    cap += (int64_t)P * cp;
    tiles += 2 * (int64_t)P * ((cp + BLOCK - 1) / BLOCK);
  }
  if (tiles > 0x7fffffff) return false;
  L.total_nodes = nodes;
  L.total_cap = cap;
  L.max_tiles = (int)tiles;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.ip = take(sizeof(InstParams) * n_inst);
  L.st = take(sizeof(InstState) * 2 * n_inst);
  L.counts = take(sizeof(uint32_t) * CSTRIDE * 3 * 2 * MAX_PART * (size_t)n_inst);
  L.ev = take(sizeof(unsigned long long) * NEV * NSLOT * (size_t)n_inst);
  L.maxw = take(sizeof(uint32_t) * (size_t)n_inst);
  L.acc = take(sizeof(unsigned long long) * 2 * NSLOT * (size_t)nodes);
  L.E = take(rs * 2 * nodes);
  L.E64 = take(8 * 2 * (size_t)nodes);
  L.phi = take(8 * 2 * (size_t)nodes);
  L.rho = take(8 * 2 * (size_t)nodes);
  L.ring = take(sizeof(StatsRow) * RING * (size_t)n_inst);
  L.inst_err = take(sizeof(uint32_t) * n_inst);
  L.sort_hist = take(sizeof(uint32_t) * 2 * (size_t)nodes);
  L.sort_cur = take(sizeof(uint32_t) * 2 * (size_t)nodes);
  L.tiles = take(sizeof(uint32_t) * 3 * 2 * (size_t)n_inst);
  L.cross = take(sizeof(int32_t) * 2 * (size_t)nodes);
  L.flux = take(sizeof(double) * 2 * (size_t)nodes);
  L.glob = take(sizeof(Global));
  const int ng = xs->n_grid;
  L.xs_e = take(rs * ng);
  L.xs_sig = take(rs * (size_t)ng * 2 * row_channels(xs->n_chan));
  L.xs_thr = take(rs * MAX_CHAN);
  L.xs_kind = take(sizeof(int32_t) * MAX_CHAN);
  // cap is a whole number of chunks (every partition is)
  const size_t chunk_bytes = (size_t)CH * (4 + 4 * rs + 8);
  for (int b = 0; b < 2; ++b)
    for (int s = 0; s < 2; ++s) L.blk[b][s] = take(chunk_bytes * (size_t)(cap / CH));
  for (int b = 0; b < 2; ++b)
    for (int s = 0; s < 2; ++s) L.wt[b][s] = splitting(cfg) ? take(rs * (size_t)cap) : 0;
  L.total = o;
  return true;
}

std::string validate(const slpic_config* cfg, const slpic_instance* inst, int n_inst,
                     const slpic_xs* xs) {
  if (!cfg || !inst || !xs) return "null argument";
  if (cfg->precision != 32 && cfg->precision != 64) return "precision must be 32 or 64";
  if (n_inst < 1 || n_inst > MAX_INST) return "n_inst must be in 1..1024";
  if (!(cfg->T_gas > 0) || !(cfg->area > 0) || !(cfg->w_j0 > 0)) return "T_gas, area, w_j0 must be > 0";
  if (!(cfg->cfl > 0 && cfg->cfl <= 1)) return "cfl must be in (0, 1]";
  if (!(cfg->ion_B_eV > 0)) return "ion_B_eV must be > 0";
  if (cfg->resort_period < 0) return "resort_period must be >= 0";
  if (!(cfg->split_frac >= 0.0 && cfg->split_frac <= 1.0)) return "split_frac must be in [0, 1]";
  if (splitting(cfg) && (cfg->flags & SLPIC_FLAG_FLUX))
    return "the flux diagnostic is not available with weight splitting";
  if (cfg->flags & ~(uint32_t)(SLPIC_FLAG_PRODUCTS_AT_REST | SLPIC_FLAG_SEE_ENERGY | SLPIC_FLAG_FLUX))
    return "unknown flags";
  if (xs->n_chan < 0 || xs->n_chan > MAX_CHAN) return "n_chan must be in 0..8";
  if (xs->n_grid < 2 || !xs->energies) return "n_grid must be >= 2";
  if (xs->n_chan > 0 && (!xs->sigma || !xs->threshold_eV || !xs->kind)) return "missing tables";
  const double e0 = xs->energies[0], e1 = xs->energies[xs->n_grid - 1];
  if (!(e0 > 0) || !(e1 > e0)) return "energy grid must be positive and increasing";
  for (int j = 0; j < xs->n_grid; ++j) {
    const double want = e0 * std::exp(j * (std::log(e1 / e0) / (xs->n_grid - 1)));
    if (!(std::fabs(xs->energies[j] - want) <= 1e-9 * want)) return "energy grid is not log-uniform";
  }
  for (int k = 0; k < xs->n_chan; ++k) {
    if (xs->kind[k] < 0 || xs->kind[k] > 2) return "unknown channel kind";
    if (!(xs->threshold_eV[k] >= 0)) return "thresholds must be >= 0";
    for (int j = 0; j < xs->n_grid; ++j)
      if (!(xs->sigma[(size_t)k * xs->n_grid + j] >= 0)) return "cross sections must be >= 0";
  }
  if (xs->fixed_prob) {
    double s = 0;
    for (int k = 0; k < xs->n_chan; ++k) {
      if (!(xs->fixed_prob[k] >= 0)) return "fixed probabilities must be >= 0";
      s += xs->fixed_prob[k];
    }
    if (s > 1.0) return "fixed probabilities sum above 1";
    if (!(xs->fixed_prob_cx >= 0 && xs->fixed_prob_cx <= 1)) return "fixed_prob_cx outside [0,1]";
  }
  if (!(xs->sigma_cx >= 0)) return "sigma_cx must be >= 0";
  for (int i = 0; i < n_inst; ++i) {
    const slpic_instance& I = inst[i];
    if (!(I.d > 0) || I.cells < 2 || !(I.p_torr >= 0)) return "instance needs d > 0, cells >= 2, p >= 0";
    if (!(I.gamma_se >= 0 && I.gamma_se <= 1)) return "gamma_se must be in [0, 1]";
    if (I.seed_mode < 0 || I.seed_mode > 2) return "unknown seed mode";
    if (I.stream > 0xffffffffll) return "stream must be below 2^32 (or negative: the batch index)";
    if (I.n_seed < 0 || I.n_target < 0) return "n_seed and n_target must be >= 0";
    if (I.capacity < I.n_seed || I.capacity < 1 || I.capacity > 0x7fffffff)
      return "capacity must be in [max(1, n_seed), 2^31)";
    if (!(I.v_limit > 0) && !(std::fabs(I.V) > 0)) return "derived speed limit needs V != 0";
    if (I.v_limit == INFINITY && !(I.dt > 0) && !(std::fabs(I.V) > 0)) return "plain PIC needs dt or V";
  }
  return "";
}

// Null-collision bound for electrons: nu'(eps) = n_g sigma_T(eps) min(v, v0)
// (Eq. 16 with beta_n = 1).  On each table segment the interpolated total is
// below the larger node value and min(v, v0) grows with energy, so
// max(node totals) * min(v(right node), v0) bounds the segment; above the
// table the cross section is constant up to the cap energy 2|V| + 100 eV.
double electron_bound(const slpic_xs* xs, double n_g, double v0, double ecap) {
  const int n = xs->n_grid, nc = xs->n_chan;
  double best = 0.0;
  for (int j = 0; j + 1 < n; ++j) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nc; ++k) {
      a += xs->sigma[(size_t)k * n + j];
      b += xs->sigma[(size_t)k * n + j + 1];
    }
    const double v = std::sqrt(2.0 * kQE * xs->energies[j + 1] / kME);
    best = std::max(best, std::max(a, b) * std::min(v, v0));
  }
  double tail = 0.0;
  for (int k = 0; k < nc; ++k) tail += xs->sigma[(size_t)k * n + n - 1];
  best = std::max(best, tail * std::min(std::sqrt(2.0 * kQE * ecap / kME), v0));
  return n_g * best;
}

InstParams derive(const slpic_config* cfg, const slpic_instance& I, const slpic_xs* xs,
                  const Layout& L, int i) {
  InstParams P;
  std::memset(&P, 0, sizeof(P));
  P.d = I.d;
  P.cells = I.cells;
  P.dx = I.d / I.cells;
  P.inv_dx = 1.0 / P.dx;
  P.V = I.V;
  P.area = cfg->area;
  P.gamma_se = I.gamma_se;
  if (I.v_limit == INFINITY) P.v0 = INFINITY;
  else if (I.v_limit > 0) P.v0 = I.v_limit;
  else P.v0 = std::sqrt(2.0 * kQE * std::fabs(I.V) / kMAR);  // Sec. IV speed limit
  P.limited = std::isfinite(P.v0) ? 1 : 0;
  P.inv_v0 = P.limited ? 1.0 / P.v0 : 0.0;
  if (I.dt > 0) P.dt = I.dt;
  else if (P.limited) P.dt = cfg->cfl * P.dx / P.v0;
  else P.dt = cfg->cfl * P.dx / std::sqrt(2.0 * kQE * std::fabs(I.V) / kME);
  P.n_g = I.p_torr * kTorr / (kKB * cfg->T_gas);
  const double ecap = std::max(xs->energies[xs->n_grid - 1], 2.0 * std::fabs(I.V) + 100.0);
  P.nu_max_e = electron_bound(xs, P.n_g, P.v0, ecap);
  P.sigma_cx = xs->sigma_cx;
  P.nu_max_cx = P.n_g * xs->sigma_cx * std::min(P.v0, std::sqrt(2.0 * kQE * ecap / kMAR));
  P.qm_e = -kQE / kME;
  P.qm_i = kQE / kMAR;
  P.vth_i = std::sqrt(kKB * cfg->T_gas / kMAR);
  P.w_j0 = cfg->w_j0;
  P.seg = L.seg[i];
  P.cap = I.capacity;
  P.cap_p = L.cap_p[i];
  P.parts = L.parts[i];
  P.n_target = I.n_target;
  P.node = L.node[i];
  // collision strategy (Sec. III): candidates with q = min(1, P / s), the
  // fraction f = max(s, P) of a colliding candidate's flux weight collides;
  // whole markers: q = P, f = 1
  const bool split = splitting(cfg);
  const double sf = cfg->split_frac;
  auto cand = [&](double Pc) { return split ? std::min(1.0, Pc / sf) : Pc; };
  auto frac = [&](double Pc) { return split ? std::max(sf, Pc) : 1.0; };
  const double Pn_e = -std::expm1(-P.nu_max_e * P.dt), Pn_cx = -std::expm1(-P.nu_max_cx * P.dt);
  P.t_null_e = prob_threshold(cand(Pn_e));
  P.t_null_cx = prob_threshold(cand(Pn_cx));
  P.f_e = frac(Pn_e);
  P.f_cx = frac(Pn_cx);
  P.t_see = prob_threshold(I.gamma_se);
  P.key = I.stream >= 0 ? (uint32_t)I.stream : (uint32_t)i;
  if (xs->fixed_prob) {
    double tot = 0.0;
    for (int k = 0; k < xs->n_chan; ++k) tot += xs->fixed_prob[k];
    double cum = 0.0;
    for (int k = 0; k < xs->n_chan; ++k) {
      cum += xs->fixed_prob[k];
      P.t_fixed[k] = prob_threshold(cum);
      P.t_fsplit[k] = tot > 0.0 ? prob_threshold(cum / tot) : 0u;
    }
    P.t_cand_fixed_e = split ? prob_threshold(cand(tot))
                             : (xs->n_chan > 0 ? P.t_fixed[xs->n_chan - 1] : 0u);
    P.f_e = frac(tot);
    P.t_fixed_cx = prob_threshold(cand(xs->fixed_prob_cx));
    P.f_cx = frac(xs->fixed_prob_cx);
  }
  P.g_e = 1.0 - P.f_e;
  P.g_cx = 1.0 - P.f_cx;
  P.dt_f = (float)P.dt;
  P.v0_f = (float)P.v0;
  P.inv_v0_f = (float)P.inv_v0;
  P.dx_f = (float)P.dx;
  P.inv_dx_f = (float)P.inv_dx;
  P.qm_e_f = (float)P.qm_e;
  P.qm_i_f = (float)P.qm_i;
  P.n_g_f = (float)P.n_g;
  P.nu_max_e_f = (float)P.nu_max_e;
  P.nu_max_cx_f = (float)P.nu_max_cx;
  P.sigma_cx_f = (float)P.sigma_cx;
  P.vth_i_f = (float)P.vth_i;
  P.f_e_f = (float)P.f_e;
  P.g_e_f = (float)P.g_e;
  P.f_cx_f = (float)P.f_cx;
  P.g_cx_f = (float)P.g_cx;
  return P;
}

}  // namespace

struct slpic_handle {
  slpic_config cfg;
  std::vector<slpic_instance> inst;
  std::vector<InstParams> ip;
  int n_inst = 0;
  Layout L;
  char* ws = nullptr;
  int static_dev = -1;   // device whose static workspace this handle holds, or -1
  hipStream_t stream = nullptr;
  Ctx<float> c32;
  Ctx<double> c64;
  int grid = 0;
  int cus = 0, occ_per_cu = 0;  // compute units; resident particle workgroups per CU
  int occ = 5;                  // launch shape: waves per SIMD of the FP32 particle kernel
  int blocks_at[7] = {0, 0, 0, 0, 0, 0, 0};  // resident workgroups per CU for each shape
  int dist = 1;                 // work distribution: 1 claimed runs, 0 equal shares
  uint64_t gen = 0;      // generation launches issued
  int64_t steps = 0;
  bool use_graph = false;
  int graph_period = 16;
  hipGraphExec_t graph = nullptr;
  int graph_phase = 0;   // steps mod resort_period when the graph was captured
  int lds_max = 0;       // shared memory per block of the device
  // kernel timing: events before the particle kernel, between the two
  // kernels and after the tail kernel of each profiled step, in two pools
  // so that one can be read back while the other fills
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool[2];
  int ev_cur = 0, ev_used[2] = {0, 0};
  double t_gen_ms = 0, t_tail_ms = 0;
  int64_t t_steps = 0;
  std::string err;
};

namespace {

int fail(slpic_t* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return code;
}

int hip_fail(slpic_t* h, hipError_t e, const char* where) {
  return fail(h, SLPIC_HIP_ERROR, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
  } while (0)

template <typename R>
void fill_ctx(slpic_t* h, Ctx<R>& C) {
  const Layout& L = h->L;
  char* w = h->ws;
  C.ip = reinterpret_cast<const InstParams*>(w + L.ip);
  for (int b = 0; b < 2; ++b)
    for (int s = 0; s < 2; ++s) {
      C.buf[b][s].p = w + L.blk[b][s];
    }
  C.st = reinterpret_cast<InstState*>(w + L.st);
  C.counts = reinterpret_cast<uint32_t*>(w + L.counts);
  C.ev = reinterpret_cast<unsigned long long*>(w + L.ev);
  C.maxw = reinterpret_cast<uint32_t*>(w + L.maxw);
  C.acc = reinterpret_cast<unsigned long long*>(w + L.acc);
  C.E = reinterpret_cast<R*>(w + L.E);
  C.E64 = reinterpret_cast<double*>(w + L.E64);
  C.phi = reinterpret_cast<double*>(w + L.phi);
  C.rho = reinterpret_cast<double*>(w + L.rho);
  C.ring = reinterpret_cast<StatsRow*>(w + L.ring);
  C.inst_err = reinterpret_cast<uint32_t*>(w + L.inst_err);
  C.sort_hist = reinterpret_cast<uint32_t*>(w + L.sort_hist);
  C.sort_cur = reinterpret_cast<uint32_t*>(w + L.sort_cur);
  C.tiles = reinterpret_cast<uint32_t*>(w + L.tiles);
  C.cross = reinterpret_cast<int32_t*>(w + L.cross);
  C.flux = reinterpret_cast<double*>(w + L.flux);
  C.g = reinterpret_cast<Global*>(w + L.glob);
  C.split = splitting(&h->cfg) ? 1 : 0;
  C.dist = h->dist;
  C.sorted = h->cfg.resort_period > 0 ? 1 : 0;
  C.occ = h->occ;
  for (int b = 0; b < 2; ++b)
    for (int s = 0; s < 2; ++s) C.wt[b][s] = C.split ? reinterpret_cast<R*>(w + L.wt[b][s]) : nullptr;
  C.xs_e = reinterpret_cast<const R*>(w + L.xs_e);
  C.xs_sig = reinterpret_cast<const R*>(w + L.xs_sig);
  C.xs_thr = reinterpret_cast<const R*>(w + L.xs_thr);
  C.xs_kind = reinterpret_cast<const int32_t*>(w + L.xs_kind);
  C.n_inst = h->n_inst;
  C.total_nodes = L.total_nodes;
  C.max_tiles = L.max_tiles;
  C.grid = h->grid;
  C.flags = h->cfg.flags;
  C.seed = h->cfg.seed;
  C.ion_B = h->cfg.ion_B_eV;
  int64_t capmax = 1;
  for (auto& I : h->inst) capmax = std::max<int64_t>(capmax, I.capacity);
  int bits = 0;
  while ((1ll << bits) <= capmax) ++bits;
  // a node sums at most one unit per marker; markers produced beyond the
  // capacity (up to 4x with ionization and splitting) still deposit
  const int want = h->cfg.precision == 64 ? 44 : 31;
  C.dep_shift = std::min(want, 60 - bits);
  int maxc = 0;
  for (auto& I : h->inst) maxc = std::max(maxc, I.cells);
  C.tail_lds = tail_lds_bytes(maxc);
  C.gen_lds = (int)gen_lds_bytes(h->n_inst);
  C.max_cells = maxc;
  C.sort_lds1 = (int)sort_lds_bytes(h->n_inst, maxc, 1);
  C.sort_lds2 = (int)sort_lds_bytes(h->n_inst, maxc, 2);
}

// Cross-section table rows for the particle kernel: per node the channels'
// values and their changes to the next node, padded to 4 or MAX_CHAN
// channels, so that a collision reads its node's row in one aligned access.
// The change is b - a in the kernel's precision, the same number the
// interpolation a + t (b - a) would form.
template <typename R>
int upload_tables(slpic_t* h, Ctx<R>& C, const slpic_xs* xs) {
  const int ng = xs->n_grid, nc = xs->n_chan, ncp = row_channels(nc);
  std::vector<R> e(ng), sig((size_t)ng * 2 * ncp, R(0)), thr(MAX_CHAN, (R)INFINITY);
  std::vector<int32_t> kind(MAX_CHAN, 0);
  for (int j = 0; j < ng; ++j) e[j] = (R)xs->energies[j];
  for (int j = 0; j < ng; ++j)
    for (int k = 0; k < nc; ++k) {
      const R a = (R)xs->sigma[(size_t)k * ng + j];
      sig[(size_t)j * 2 * ncp + k] = a;
      if (j + 1 < ng) sig[(size_t)j * 2 * ncp + ncp + k] = (R)xs->sigma[(size_t)k * ng + j + 1] - a;
    }
  for (int k = 0; k < nc; ++k) {
    thr[k] = (R)xs->threshold_eV[k];
    kind[k] = xs->kind[k];
  }
  C.n_chan = nc;
  C.ncp = ncp;
  C.n_grid = ng;
  C.fixed = xs->fixed_prob ? 1 : 0;
  C.log_emin = (R)std::log(xs->energies[0]);
  C.e_lo = (R)xs->energies[0];
  C.e_hi = (R)xs->energies[ng - 1];
  C.inv_dlog = (R)((ng - 1) / std::log(xs->energies[ng - 1] / xs->energies[0]));
  const double dlog = std::log(xs->energies[ng - 1] / xs->energies[0]) / (ng - 1);
  C.log2_ratio = (R)(dlog / std::log(2.0));
  C.ratio_m1 = (R)std::expm1(dlog);
  HIPCHK(h, hipMemcpyAsync((void*)C.xs_e, e.data(), sizeof(R) * ng, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync((void*)C.xs_sig, sig.data(), sizeof(R) * sig.size(), hipMemcpyHostToDevice,
                           h->stream));
  HIPCHK(h, hipMemcpyAsync((void*)C.xs_thr, thr.data(), sizeof(R) * thr.size(), hipMemcpyHostToDevice,
                           h->stream));
  HIPCHK(h, hipMemcpyAsync((void*)C.xs_kind, kind.data(), sizeof(int32_t) * kind.size(),
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return SLPIC_OK;
}

template <typename R>
hipError_t launch_pair(const Ctx<R>& C, int mode, hipStream_t s) {
  hipError_t e = launch_particles<R>(C, mode, s);
  return e != hipSuccess ? e : launch_tail<R>(C, mode, s);
}

hipError_t launch_pair_any(slpic_t* h, int mode) {
  return h->cfg.precision == 64 ? launch_pair<double>(h->c64, mode, h->stream)
                                : launch_pair<float>(h->c32, mode, h->stream);
}

constexpr int kEvPool = 3 * 512;   // events per timing pool (512 steps)

// Adds the durations of the steps recorded in pool b to the totals.
int drain_pool(slpic_t* h, int b) {
  std::vector<hipEvent_t>& P = h->ev_pool[b];
  if (h->ev_used[b] == 0) return SLPIC_OK;
  HIPCHK(h, hipEventSynchronize(P[h->ev_used[b] - 1]));
  for (int k = 0; k < h->ev_used[b]; k += 3) {
    float a = 0, c = 0;
    HIPCHK(h, hipEventElapsedTime(&a, P[k], P[k + 1]));
    HIPCHK(h, hipEventElapsedTime(&c, P[k + 1], P[k + 2]));
    h->t_gen_ms += a;
    h->t_tail_ms += c;
    h->t_steps += 1;
  }
  h->ev_used[b] = 0;
  return SLPIC_OK;
}

int launch_timed(slpic_t* h, int mode) {
  int b = h->ev_cur;
  if (h->ev_used[b] + 3 > kEvPool) {
    b ^= 1;
    int rc = drain_pool(h, b);
    if (rc) return rc;
    h->ev_cur = b;
  }
  hipEvent_t* e = h->ev_pool[b].data() + h->ev_used[b];
  HIPCHK(h, hipEventRecord(e[0], h->stream));
  hipError_t r = h->cfg.precision == 64 ? launch_particles<double>(h->c64, mode, h->stream)
                                        : launch_particles<float>(h->c32, mode, h->stream);
  if (r != hipSuccess) return hip_fail(h, r, "particle kernel launch");
  HIPCHK(h, hipEventRecord(e[1], h->stream));
  r = h->cfg.precision == 64 ? launch_tail<double>(h->c64, mode, h->stream)
                             : launch_tail<float>(h->c32, mode, h->stream);
  if (r != hipSuccess) return hip_fail(h, r, "tail kernel launch");
  HIPCHK(h, hipEventRecord(e[2], h->stream));
  h->ev_used[b] += 3;
  return SLPIC_OK;
}

// a cell sort runs before every step whose number of completed steps is a
// multiple of resort_period (the seeded state included)
bool sort_due(const slpic_t* h, int64_t steps_done) {
  return h->cfg.resort_period > 0 && steps_done % h->cfg.resort_period == 0;
}

int sort_phase(const slpic_t* h) {
  return h->cfg.resort_period > 0 ? (int)(h->steps % h->cfg.resort_period) : 0;
}

hipError_t launch_sort_any(slpic_t* h) {
  return h->cfg.precision == 64 ? launch_sort<double>(h->c64, h->stream)
                                : launch_sort<float>(h->c32, h->stream);
}

int launch_gen_any(slpic_t* h, int mode) {
  if (mode == MODE_STEP && sort_due(h, h->steps)) {
    hipError_t e = launch_sort_any(h);
    if (e != hipSuccess) return hip_fail(h, e, "cell sort launch");
  }
  if (h->profiling && mode == MODE_STEP) {
    int rc = launch_timed(h, mode);
    if (rc) return rc;
  } else {
    hipError_t e = launch_pair_any(h, mode);
    if (e != hipSuccess) return hip_fail(h, e, "generation kernel launch");
  }
  h->gen += 1;
  return SLPIC_OK;
}

void release_events(slpic_t* h) {
  for (auto& P : h->ev_pool) {
    for (hipEvent_t e : P) (void)hipEventDestroy(e);
    P.clear();
  }
  h->ev_used[0] = h->ev_used[1] = 0;
}

Global read_global(slpic_t* h, hipError_t* e) {
  Global G;
  *e = hipMemcpy(&G, h->ws + h->L.glob, sizeof(Global), hipMemcpyDeviceToHost);
  return G;
}

}  // namespace

namespace {

int current(slpic_t* h, Global& G, uint32_t& slot3, uint32_t& bsel) {
  HIPCHK(h, hipStreamSynchronize(h->stream));
  hipError_t e;
  G = read_global(h, &e);
  if (e != hipSuccess) return hip_fail(h, e, "read state");
  if ((uint64_t)G.cur_gen != (h->gen & 0xffffffffull))
    return fail(h, SLPIC_HIP_ERROR, "device generation out of step with the host");
  slot3 = G.cur_gen % 3u;
  bsel = G.bufsel[G.cur_gen % 2u];
  return SLPIC_OK;
}

template <typename R>
Soa<R> buffer_of(slpic_t* h, uint32_t bsel, int sp);
template <>
Soa<float> buffer_of<float>(slpic_t* h, uint32_t bsel, int sp) { return h->c32.buf[bsel][sp]; }
template <>
Soa<double> buffer_of<double>(slpic_t* h, uint32_t bsel, int sp) { return h->c64.buf[bsel][sp]; }

size_t count_offset(slpic_t* h, uint32_t slot3, int inst, int sp, int p) {
  return h->L.counts + sizeof(uint32_t) * CSTRIDE * ((((size_t)slot3 * h->n_inst + inst) * 2 + sp) * MAX_PART + p);
}

// Markers are spread over the instance's P partitions: marker k of a loaded
// population goes to partition k mod P at slot k / P.
template <typename R>
int load_impl(slpic_t* h, int inst, int sp, int64_t n, const int32_t* cell, const double* off,
              const double* vx, const double* vy, const double* vz, const uint64_t* id) {
  Global G;
  uint32_t slot3, bsel;
  int rc = current(h, G, slot3, bsel);
  if (rc) return rc;
  const InstParams& P = h->ip[inst];
  for (int64_t k = 0; k < n; ++k)
    if (cell[k] < 0 || cell[k] >= P.cells || !(off[k] >= 0.0 && off[k] < 1.0) ||
        !std::isfinite(vx[k]) || !std::isfinite(vy[k]) || !std::isfinite(vz[k]))
      return fail(h, SLPIC_INVALID_ARG, "marker outside the gap or non-finite");
  if ((n + P.parts - 1) / P.parts > P.cap_p) return fail(h, SLPIC_CAPACITY_EXCEEDED, "load exceeds capacity");
  const Soa<R> B = buffer_of<R>(h, bsel, sp);
  for (int p = 0; p < P.parts; ++p) {
    const int64_t m = n / P.parts + (p < n % P.parts ? 1 : 0);
    // the partition's first chunks, packed on the host (slot q of the
    // partition is slot q of this image)
    const int64_t nch = (m + CH - 1) / CH;
    std::vector<char> img((size_t)(nch * Soa<R>::kChunk), 0);
    const Soa<R> H{img.data()};
    for (int64_t q = 0; q < m; ++q) {
      const int64_t k = q * P.parts + p;
      H.cell(q) = cell[k];
      R f = (R)off[k];
      H.off(q) = f < R(1) ? f : std::nextafter(R(1), R(0));
      H.vx(q) = (R)vx[k];
      H.vy(q) = (R)vy[k];
      H.vz(q) = (R)vz[k];
      H.id(q) = id[k];
    }
    const int64_t at = P.seg + (int64_t)p * P.cap_p;  // a multiple of CH
    if (m) HIPCHK(h, hipMemcpy(B.chunk(at), img.data(), img.size(), hipMemcpyHostToDevice));
    if (m && splitting(&h->cfg)) {
      // loaded markers carry the instance's flux weight (relative weight 1)
      const std::vector<R> ones((size_t)m, R(1));
      HIPCHK(h, hipMemcpy(h->ws + h->L.wt[bsel][sp] + (size_t)at * sizeof(R), ones.data(),
                          (size_t)m * sizeof(R), hipMemcpyHostToDevice));
    }
    const uint32_t cnt = (uint32_t)m;
    HIPCHK(h, hipMemcpy(h->ws + count_offset(h, slot3, inst, sp, p), &cnt, sizeof(uint32_t),
                        hipMemcpyHostToDevice));
  }
  const uint32_t tl = pair_tiles((uint32_t)((n + P.parts - 1) / P.parts), P.parts);
  HIPCHK(h, hipMemcpy(h->ws + h->L.tiles + sizeof(uint32_t) * (((size_t)slot3 * h->n_inst + inst) * 2 + sp),
                      &tl, sizeof(uint32_t), hipMemcpyHostToDevice));
  rc = launch_gen_any(h, MODE_REFRESH);
  if (rc) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return SLPIC_OK;
}

int part_counts(slpic_t* h, uint32_t slot3, int inst, int sp, std::vector<uint32_t>& c) {
  const int P = h->ip[inst].parts;
  c.assign(P, 0u);
  HIPCHK(h, hipMemcpy2D(c.data(), sizeof(uint32_t), h->ws + count_offset(h, slot3, inst, sp, 0),
                        sizeof(uint32_t) * CSTRIDE, sizeof(uint32_t), P, hipMemcpyDeviceToHost));
  return SLPIC_OK;
}

template <typename R>
int read_weights_impl(slpic_t* h, int inst, int sp, int64_t max_n, int64_t* n_out, double* w) {
  Global G;
  uint32_t slot3, bsel;
  int rc = current(h, G, slot3, bsel);
  if (rc) return rc;
  std::vector<uint32_t> cnt;
  rc = part_counts(h, slot3, inst, sp, cnt);
  if (rc) return rc;
  int64_t n = 0;
  for (uint32_t c : cnt) n += c;
  *n_out = n;
  if (n > max_n) return fail(h, SLPIC_INVALID_ARG, "output array too small");
  const InstParams& P = h->ip[inst];
  int64_t done = 0;
  std::vector<R> buf;
  for (int p = 0; p < P.parts; ++p) {
    const int64_t m = cnt[p], at = P.seg + (int64_t)p * P.cap_p;
    if (!m) continue;
    buf.resize((size_t)m);
    HIPCHK(h, hipMemcpy(buf.data(), h->ws + h->L.wt[bsel][sp] + (size_t)at * sizeof(R),
                        (size_t)m * sizeof(R), hipMemcpyDeviceToHost));
    for (int64_t q = 0; q < m; ++q) w[done + q] = (double)buf[(size_t)q];
    done += m;
  }
  return SLPIC_OK;
}

template <typename R>
int read_impl(slpic_t* h, int inst, int sp, int64_t max_n, int64_t* n_out, int32_t* cell,
              double* off, double* vx, double* vy, double* vz, uint64_t* id) {
  Global G;
  uint32_t slot3, bsel;
  int rc = current(h, G, slot3, bsel);
  if (rc) return rc;
  std::vector<uint32_t> cnt;
  rc = part_counts(h, slot3, inst, sp, cnt);
  if (rc) return rc;
  int64_t n = 0;
  for (uint32_t c : cnt) n += c;
  *n_out = n;
  if (n > max_n) return fail(h, SLPIC_INVALID_ARG, "output arrays too small");
  const InstParams& P = h->ip[inst];
  const Soa<R> B = buffer_of<R>(h, bsel, sp);
  int64_t done = 0;
  for (int p = 0; p < P.parts; ++p) {
    const int64_t m = cnt[p], at = P.seg + (int64_t)p * P.cap_p;  // at: a multiple of CH
    if (!m) continue;
    const int64_t nch = (m + CH - 1) / CH;
    std::vector<char> img((size_t)(nch * Soa<R>::kChunk));
    HIPCHK(h, hipMemcpy(img.data(), B.chunk(at), img.size(), hipMemcpyDeviceToHost));
    const Soa<R> H{img.data()};
    for (int64_t q = 0; q < m; ++q) {
      if (cell) cell[done + q] = H.cell(q);
      if (off) off[done + q] = (double)H.off(q);
      if (vx) vx[done + q] = (double)H.vx(q);
      if (vy) vy[done + q] = (double)H.vy(q);
      if (vz) vz[done + q] = (double)H.vz(q);
      if (id) id[done + q] = H.id(q);
    }
    done += m;
  }
  return SLPIC_OK;
}

}  // namespace

namespace {

// Handles holding each device's static workspace (slpic_create_static):
// at most one at a time per device.
std::mutex g_static_mu;
bool g_static_busy[MAX_DEVICES] = {};

// Create on a given device workspace (slpic_create, slpic_create_static).
int create_impl(const slpic_config* cfg, const slpic_instance* inst, int n_inst,
                const slpic_xs* xs, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                slpic_t** out) {
  if (!out) return fail(nullptr, SLPIC_INVALID_ARG, "out is NULL");
  *out = nullptr;
  const std::string v = validate(cfg, inst, n_inst, xs);
  if (!v.empty()) return fail(nullptr, SLPIC_INVALID_ARG, v);
  slpic_t* h = new slpic_handle();
  h->cfg = *cfg;
  h->inst.assign(inst, inst + n_inst);
  h->n_inst = n_inst;
  if (!make_layout(cfg, inst, n_inst, xs, h->L)) {
    delete h;
    return fail(nullptr, SLPIC_INVALID_ARG, "too many tiles, or a partition of 2 GiB or more");
  }
  if (!dev_workspace || ws_bytes < h->L.total || ((uintptr_t)dev_workspace & 255)) {
    delete h;
    return fail(nullptr, SLPIC_WORKSPACE_TOO_SMALL, "workspace missing, too small or misaligned");
  }
  h->ws = static_cast<char*>(dev_workspace);
  h->stream = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < n_inst; ++i) h->ip.push_back(derive(cfg, inst[i], xs, h->L, i));
  for (int i = 0; i < n_inst; ++i)
    if (inst[i].n_seed > (int64_t)h->L.parts[i] * h->L.cap_p[i]) {
      delete h;
      return fail(nullptr, SLPIC_INVALID_ARG, "seeds exceed the capacity");
    }
  // grid: enough workgroups to fill the device, never more than tiles exist
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = cfg->precision == 64 ? occupancy_gen<double>(&per_cu, gen_lds_bytes(n_inst), splitting(cfg), 5)
                             : occupancy_gen<float>(&per_cu, gen_lds_bytes(n_inst), splitting(cfg), 5);
  // the other launch shapes of the FP32 whole-marker kernel (autotuner)
  for (int oc = 4; oc <= 5 && e == hipSuccess; ++oc) {
    int b = 0;
    if (cfg->precision == 32 && !splitting(cfg)) e = occupancy_gen<float>(&b, gen_lds_bytes(n_inst), false, oc);
    h->blocks_at[oc] = oc == 5 ? per_cu : b;
  }
  if (e != hipSuccess) {
    int rc = hip_fail(nullptr, e, "device query");
    delete h;
    return rc;
  }
  h->grid = std::max(1, std::min(cus * std::max(per_cu, 1), h->L.max_tiles));
  // markers in cell order keep their deposits in the LDS window best with
  // equal contiguous shares; otherwise runs are claimed (balance)
  h->dist = cfg->resort_period > 0 ? 0 : 1;
  h->cus = cus;
  h->occ_per_cu = std::max(per_cu, 1);
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    lds_max = 65536;
  int maxc = 0;
  for (int i = 0; i < n_inst; ++i) maxc = std::max(maxc, inst[i].cells);
  if ((size_t)tail_lds_bytes(maxc) + 1024 > (size_t)lds_max) {
    delete h;
    return fail(nullptr, SLPIC_INVALID_ARG, "too many cells for the device's shared memory per block");
  }
  h->lds_max = lds_max;
  if (cfg->resort_period > 0 && sort_lds_bytes(n_inst, maxc, 2) + 64 > (size_t)lds_max) {
    delete h;
    return fail(nullptr, SLPIC_INVALID_ARG,
                "the cell sort needs more shared memory per block than the device has "
                "(fewer cells, or resort_period 0)");
  }
  fill_ctx(h, h->c32);
  fill_ctx(h, h->c64);
  int rc = cfg->precision == 64 ? upload_tables(h, h->c64, xs) : upload_tables(h, h->c32, xs);
  if (rc) {
    g_create_error = h->err;
    delete h;
    return rc;
  }
  const Layout& L = h->L;
  // constant and initial state: generation 0, buffer 0, seeds in counts[0]
  std::vector<InstState> st(2 * n_inst);
  std::vector<uint32_t> counts((size_t)CSTRIDE * 3 * 2 * MAX_PART * n_inst, 0u);
  std::vector<uint32_t> tiles((size_t)3 * 2 * n_inst, 0u);
  for (int i = 0; i < n_inst; ++i) {
    const int base_shift = cfg->precision == 64 ? h->c64.dep_shift : h->c32.dep_shift;
    st[i] = InstState{cfg->w_j0, 0u, POP_NONE, base_shift, {0, 0}};
    st[n_inst + i] = st[i];
    const int64_t ns = inst[i].seed_mode != SLPIC_SEED_NONE ? inst[i].n_seed : 0;
    const int P = L.parts[i];
    for (int p = 0; p < P; ++p)  // seed k sits in partition k mod P
      counts[((size_t)i * 2 * MAX_PART + p) * CSTRIDE] = (uint32_t)(ns / P + (p < ns % P ? 1 : 0));
    tiles[2 * (size_t)i] = pair_tiles((uint32_t)((ns + P - 1) / P), P);
  }
  Global G;
  std::memset(&G, 0, sizeof(G));
  auto up = [&](size_t off, const void* src, size_t n) {
    return hipMemcpyAsync(h->ws + off, src, n, hipMemcpyHostToDevice, h->stream);
  };
  e = up(L.ip, h->ip.data(), sizeof(InstParams) * n_inst);
  if (e == hipSuccess) e = up(L.st, st.data(), sizeof(InstState) * st.size());
  if (e == hipSuccess) e = up(L.counts, counts.data(), sizeof(uint32_t) * counts.size());
  if (e == hipSuccess) e = up(L.tiles, tiles.data(), sizeof(uint32_t) * tiles.size());
  if (e == hipSuccess) e = up(L.glob, &G, sizeof(G));
  if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.ev, 0, sizeof(unsigned long long) * NEV * NSLOT * n_inst, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.acc, 0, sizeof(unsigned long long) * 2 * NSLOT * L.total_nodes, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.sort_hist, 0, sizeof(uint32_t) * 2 * L.total_nodes, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.cross, 0, sizeof(int32_t) * 2 * L.total_nodes, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.flux, 0, sizeof(double) * 2 * L.total_nodes, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.inst_err, 0, sizeof(uint32_t) * n_inst, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.maxw, 0, sizeof(uint32_t) * n_inst, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.ring, 0, sizeof(StatsRow) * RING * n_inst, h->stream);
  for (int i = 0; i < n_inst && e == hipSuccess; ++i) {
    if (inst[i].seed_mode == SLPIC_SEED_NONE) continue;
    const double sv = std::sqrt(kQE * cfg->kTe_seed_eV / kME);
    e = cfg->precision == 64
            ? launch_seed<double>(h->c64, i, inst[i].seed_mode, inst[i].n_seed, sv, 0u, h->stream)
            : launch_seed<float>(h->c32, i, inst[i].seed_mode, inst[i].n_seed, sv, 0u, h->stream);
  }
  if (e != hipSuccess) {
    int r2 = hip_fail(nullptr, e, "create upload/seed");
    delete h;
    return r2;
  }
  rc = launch_gen_any(h, MODE_REFRESH);
  if (rc == SLPIC_OK) {
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = hip_fail(h, e, "create sync");
  }
  if (rc) {
    g_create_error = h->err;
    delete h;
    return rc;
  }
  *out = h;
  return SLPIC_OK;
}

}  // namespace

extern "C" {

size_t slpic_workspace_bytes(const slpic_config* cfg, const slpic_instance* inst, int n_inst,
                             const slpic_xs* xs) {
  if (!validate(cfg, inst, n_inst, xs).empty()) return 0;
  Layout L;
  if (!make_layout(cfg, inst, n_inst, xs, L)) return 0;
  return L.total;
}

int slpic_create(const slpic_config* cfg, const slpic_instance* inst, int n_inst,
                 const slpic_xs* xs, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                 slpic_t** out) {
  return create_impl(cfg, inst, n_inst, xs, dev_workspace, ws_bytes, hip_stream, out);
}

int slpic_create_static(const slpic_config* cfg, const slpic_instance* inst, int n_inst,
                        const slpic_xs* xs, void* hip_stream, slpic_t** out) {
  if (!out) return fail(nullptr, SLPIC_INVALID_ARG, "out is NULL");
  *out = nullptr;
  const std::string v = validate(cfg, inst, n_inst, xs);
  if (!v.empty()) return fail(nullptr, SLPIC_INVALID_ARG, v);
  Layout L;
  if (!make_layout(cfg, inst, n_inst, xs, L))
    return fail(nullptr, SLPIC_INVALID_ARG, "too many tiles, or a partition of 2 GiB or more");
  if (L.total > SLPIC_STATIC_WORKSPACE_BYTES)
    return fail(nullptr, SLPIC_WORKSPACE_TOO_SMALL,
                "the setup needs " + std::to_string(L.total) +
                    " workspace bytes, more than the static workspace's " +
                    std::to_string((size_t)SLPIC_STATIC_WORKSPACE_BYTES));
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(nullptr, SLPIC_INVALID_ARG, "device index too large");
  char* ws = nullptr;
  e = static_workspace(dev, &ws);
  if (e != hipSuccess) return hip_fail(nullptr, e, "static workspace address");
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_busy[dev])
      return fail(nullptr, SLPIC_INVALID_ARG,
                  "the static workspace of this device is held by another handle");
    g_static_busy[dev] = true;
  }
  const int rc = create_impl(cfg, inst, n_inst, xs, ws, SLPIC_STATIC_WORKSPACE_BYTES, hip_stream, out);
  if (rc == SLPIC_OK) {
    (*out)->static_dev = dev;
  } else {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_busy[dev] = false;
  }
  return rc;
}

// Captures graph_period steps (with the cell sorts due in them) as a HIP
// graph; nothing runs until the graph is launched.
static int capture_graph(slpic_t* h) {
  hipGraph_t gr;
  HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < h->graph_period; ++k) {
    hipError_t e = sort_due(h, h->steps + k) ? launch_sort_any(h) : hipSuccess;
    if (e == hipSuccess) e = launch_pair_any(h, MODE_STEP);
    if (e != hipSuccess) {
      (void)hipStreamEndCapture(h->stream, &gr);
      return hip_fail(h, e, "graph capture");
    }
  }
  HIPCHK(h, hipStreamEndCapture(h->stream, &gr));
  HIPCHK(h, hipGraphInstantiate(&h->graph, gr, nullptr, nullptr, 0));
  (void)hipGraphDestroy(gr);
  h->graph_phase = sort_phase(h);
  return SLPIC_OK;
}

int slpic_use_graph(slpic_t* h, int enable) {
  if (!h) return SLPIC_INVALID_ARG;
  h->use_graph = enable != 0;
  // capture now, so that the first replayed steps do not pay for it
  if (h->use_graph && !h->graph && !h->profiling) return capture_graph(h);
  return SLPIC_OK;
}

int slpic_step(slpic_t* h, int n_steps) {
  if (!h || n_steps < 0) return fail(h, SLPIC_INVALID_ARG, "bad step arguments");
  int done = 0;
  while (done < n_steps) {
    // graph replay needs a whole period and, with cell sorts, the same
    // position in the sort cycle as at capture (the sorts are in the graph)
    const bool graph = h->use_graph && !h->profiling && n_steps - done >= h->graph_period &&
                       (!h->graph || h->graph_phase == sort_phase(h));
    if (graph) {
      if (!h->graph) {
        const int rc = capture_graph(h);
        if (rc) return rc;
      }
      HIPCHK(h, hipGraphLaunch(h->graph, h->stream));
      h->gen += h->graph_period;
      h->steps += h->graph_period;
      done += h->graph_period;
    } else {
      int rc = launch_gen_any(h, MODE_STEP);
      if (rc) return rc;
      h->steps += 1;
      done += 1;
    }
  }
  return SLPIC_OK;
}

// Changes the particle kernel's launch shape (waves per SIMD of its
// register budget) and grid between steps.  Kernels read the generation
// from device words, so only the launch changes; a captured graph holds the
// old shape and is dropped.
static int set_shape(slpic_t* h, int occ, int grid, int dist) {
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->grid = grid;
  h->occ = occ;
  h->dist = dist;
  h->c32.grid = grid;
  h->c64.grid = grid;
  h->c32.occ = occ;
  h->c64.occ = occ;
  h->c32.dist = dist;
  h->c64.dist = dist;
  if (h->graph) {
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
  }
  return SLPIC_OK;
}

int slpic_grid(slpic_t* h, int* grid) {
  if (!h || !grid) return fail(h, SLPIC_INVALID_ARG, "null grid output");
  *grid = h->grid;
  return SLPIC_OK;
}

int slpic_autotune(slpic_t* h, int trial_steps, int* grid) {
  if (!h || trial_steps < 1 || h->profiling) return fail(h, SLPIC_INVALID_ARG, "bad autotune arguments");
  // candidates: launch shapes (the FP32 whole-marker kernel comes in two
  // register budgets) times grids (a quarter, half and all of the compute
  // units, then 1 .. the resident maximum workgroups per compute unit) times
  // work distributions (claimed runs, equal contiguous shares)
  struct Cand {
    int occ, grid, dist;
  };
  std::vector<Cand> cand;
  auto add = [&](int oc, int g, int d) {
    g = std::max(1, std::min(g, h->L.max_tiles));
    for (const Cand& c : cand)
      if (c.occ == oc && c.grid == g && c.dist == d) return;
    cand.push_back(Cand{oc, g, d});
  };
  const bool shapes = h->cfg.precision == 32 && !splitting(&h->cfg);
  for (int d : {1, 0})
    for (int oc : {5, 4}) {
      if (oc != 5 && !shapes) continue;
      const int per_cu = std::max(1, h->blocks_at[oc]);
      for (int q = 4; q >= 1; q /= 2) add(oc, h->cus / q, d);
      for (int pc = 1; pc <= per_cu; ++pc) add(oc, h->cus * pc, d);
    }
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  hipError_t er = hipEventCreate(&e1);
  if (er != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(h, er, "hipEventCreate");
  }
  // three rounds over all candidates, so that the population's drift
  // between trials spreads over every candidate; each keeps its median
  constexpr int kRounds = 3;
  std::vector<std::vector<float>> times(cand.size());
  int rc = SLPIC_OK;
  for (int round = 0; round < kRounds && rc == SLPIC_OK; ++round) {
    for (size_t c = 0; c < cand.size() && rc == SLPIC_OK; ++c) {
      rc = set_shape(h, cand[c].occ, cand[c].grid, cand[c].dist);
      // one untimed step in the new shape, then the timed ones
      for (int k = 0; k <= trial_steps && rc == SLPIC_OK; ++k) {
        if (k == 1 && hipEventRecord(e0, h->stream) != hipSuccess) rc = fail(h, SLPIC_HIP_ERROR, "event");
        if (rc == SLPIC_OK) rc = launch_gen_any(h, MODE_STEP);
        if (rc == SLPIC_OK) h->steps += 1;
      }
      float ms = 0.0f;
      if (rc == SLPIC_OK && (hipEventRecord(e1, h->stream) != hipSuccess ||
                             hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(h, SLPIC_HIP_ERROR, "autotune timing");
      if (rc == SLPIC_OK) times[c].push_back(ms);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  size_t best = 0;
  float best_ms = 0.0f;
  for (size_t c = 0; c < cand.size(); ++c) {
    std::vector<float> t = times[c];
    std::sort(t.begin(), t.end());
    const float med = t[t.size() / 2];
    if (c == 0 || med < best_ms) {
      best_ms = med;
      best = c;
    }
  }
  rc = set_shape(h, cand[best].occ, cand[best].grid, cand[best].dist);
  if (rc == SLPIC_OK && grid) *grid = cand[best].grid;
  return rc;
}

int slpic_set_launch_shape(slpic_t* h, int grid, int waves_per_simd) {
  if (!h || grid < 1 || h->profiling) return fail(h, SLPIC_INVALID_ARG, "bad launch shape");
  const bool shapes = h->cfg.precision == 32 && !splitting(&h->cfg);
  if (shapes ? (waves_per_simd != 4 && waves_per_simd != 5) : waves_per_simd != 0)
    return fail(h, SLPIC_INVALID_ARG, "waves per SIMD must be 4 or 5 (FP32 whole markers), else 0");
  return set_shape(h, shapes ? waves_per_simd : h->occ, std::min(grid, h->L.max_tiles), h->dist);
}

int slpic_set_work_distribution(slpic_t* h, int claimed) {
  if (!h || (claimed != 0 && claimed != 1) || h->profiling)
    return fail(h, SLPIC_INVALID_ARG, "work distribution must be 0 (equal shares) or 1 (claimed runs)");
  return set_shape(h, h->occ, h->grid, claimed);
}

int slpic_work_distribution(slpic_t* h, int* claimed) {
  if (!h || !claimed) return fail(h, SLPIC_INVALID_ARG, "null distribution output");
  *claimed = h->dist;
  return SLPIC_OK;
}

int slpic_launch_shape(slpic_t* h, int* grid, int* waves_per_simd) {
  if (!h || !grid || !waves_per_simd) return fail(h, SLPIC_INVALID_ARG, "null shape output");
  *grid = h->grid;
  *waves_per_simd = h->cfg.precision == 32 && !splitting(&h->cfg) ? h->occ : 0;
  return SLPIC_OK;
}

int slpic_profile(slpic_t* h, int enable) {
  if (!h) return SLPIC_INVALID_ARG;
  if (enable && !h->profiling) {
    for (auto& P : h->ev_pool) {
      P.resize(kEvPool);
      for (hipEvent_t& e : P) HIPCHK(h, hipEventCreate(&e));
    }
    h->ev_cur = 0;
    h->ev_used[0] = h->ev_used[1] = 0;
    h->t_gen_ms = h->t_tail_ms = 0;
    h->t_steps = 0;
    h->profiling = true;
  } else if (!enable && h->profiling) {
    int rc = drain_pool(h, h->ev_cur ^ 1);
    if (!rc) rc = drain_pool(h, h->ev_cur);
    release_events(h);
    h->profiling = false;
    if (rc) return rc;
  }
  return SLPIC_OK;
}

int slpic_kernel_times(slpic_t* h, double* gen_ms, double* tail_ms, int64_t* steps) {
  if (!h || !gen_ms || !tail_ms || !steps) return fail(h, SLPIC_INVALID_ARG, "null timing output");
  if (h->profiling) {
    int rc = drain_pool(h, h->ev_cur ^ 1);
    if (!rc) rc = drain_pool(h, h->ev_cur);
    if (rc) return rc;
  }
  *gen_ms = h->t_gen_ms;
  *tail_ms = h->t_tail_ms;
  *steps = h->t_steps;
  return SLPIC_OK;
}

int slpic_sort(slpic_t* h) {
  if (!h) return SLPIC_INVALID_ARG;
  if (h->cfg.resort_period <= 0 &&
      sort_lds_bytes(h->n_inst, h->c32.max_cells, 2) + 64 > (size_t)h->lds_max)
    return fail(h, SLPIC_INVALID_ARG, "the cell sort needs more shared memory per block than the device has");
  hipError_t e = launch_sort_any(h);
  if (e != hipSuccess) return hip_fail(h, e, "cell sort launch");
  return SLPIC_OK;
}

int slpic_sync(slpic_t* h) {
  if (!h) return SLPIC_INVALID_ARG;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  std::vector<uint32_t> err(h->n_inst);
  HIPCHK(h, hipMemcpy(err.data(), h->ws + h->L.inst_err, sizeof(uint32_t) * h->n_inst,
                      hipMemcpyDeviceToHost));
  uint32_t all = 0;
  for (uint32_t v : err) all |= v;
  if (all) HIPCHK(h, hipMemset(h->ws + h->L.inst_err, 0, sizeof(uint32_t) * h->n_inst));
  if (all & ERR_CAPACITY) return fail(h, SLPIC_CAPACITY_EXCEEDED, "marker capacity exceeded");
  if (all & ERR_NONFINITE) return fail(h, SLPIC_NONFINITE_STATE, "non-finite marker state");
  if (all & ERR_NU_BOUND) return fail(h, SLPIC_NU_BOUND_EXCEEDED, "collision rate above bound");
  return SLPIC_OK;
}

int slpic_load_markers(slpic_t* h, int inst, int species, int64_t n, const int32_t* cell,
                       const double* off, const double* vx, const double* vy, const double* vz,
                       const uint64_t* id) {
  if (!h || inst < 0 || inst >= h->n_inst || (species != 0 && species != 1) || n < 0)
    return fail(h, SLPIC_INVALID_ARG, "bad load arguments");
  if (n > h->inst[inst].capacity) return fail(h, SLPIC_CAPACITY_EXCEEDED, "more markers than capacity");
  if (n > 0 && (!cell || !off || !vx || !vy || !vz || !id))
    return fail(h, SLPIC_INVALID_ARG, "null marker array");
  return h->cfg.precision == 64 ? load_impl<double>(h, inst, species, n, cell, off, vx, vy, vz, id)
                                : load_impl<float>(h, inst, species, n, cell, off, vx, vy, vz, id);
}

int slpic_count(slpic_t* h, int inst, int species, int64_t* n) {
  if (!h || !n || inst < 0 || inst >= h->n_inst || (species != 0 && species != 1))
    return fail(h, SLPIC_INVALID_ARG, "bad count arguments");
  Global G;
  uint32_t slot3, bsel;
  int rc = current(h, G, slot3, bsel);
  if (rc) return rc;
  std::vector<uint32_t> c;
  rc = part_counts(h, slot3, inst, species, c);
  if (rc) return rc;
  int64_t t = 0;
  for (uint32_t v : c) t += v;
  *n = t;
  return SLPIC_OK;
}

int slpic_partitions(slpic_t* h, int inst, int species, int32_t* parts, int64_t* cap_p,
                     uint32_t* counts) {
  if (!h || !parts || !cap_p || !counts || inst < 0 || inst >= h->n_inst ||
      (species != 0 && species != 1))
    return fail(h, SLPIC_INVALID_ARG, "bad partition arguments");
  Global G;
  uint32_t slot3, bsel;
  int rc = current(h, G, slot3, bsel);
  if (rc) return rc;
  std::vector<uint32_t> c;
  rc = part_counts(h, slot3, inst, species, c);
  if (rc) return rc;
  *parts = h->ip[inst].parts;
  *cap_p = h->ip[inst].cap_p;
  for (int p = 0; p < MAX_PART; ++p) counts[p] = p < (int)c.size() ? c[p] : 0u;
  return SLPIC_OK;
}

int slpic_read_markers(slpic_t* h, int inst, int species, int64_t max_n, int64_t* n,
                       int32_t* cell, double* off, double* vx, double* vy, double* vz,
                       uint64_t* id) {
  if (!h || !n || inst < 0 || inst >= h->n_inst || (species != 0 && species != 1))
    return fail(h, SLPIC_INVALID_ARG, "bad read arguments");
  return h->cfg.precision == 64
             ? read_impl<double>(h, inst, species, max_n, n, cell, off, vx, vy, vz, id)
             : read_impl<float>(h, inst, species, max_n, n, cell, off, vx, vy, vz, id);
}

int slpic_read_weights(slpic_t* h, int inst, int species, int64_t max_n, int64_t* n,
                       double* w) {
  if (!h || !n || !w || inst < 0 || inst >= h->n_inst || (species != 0 && species != 1))
    return fail(h, SLPIC_INVALID_ARG, "bad read arguments");
  if (!splitting(&h->cfg)) return fail(h, SLPIC_INVALID_ARG, "markers carry weights only with weight splitting");
  return h->cfg.precision == 64 ? read_weights_impl<double>(h, inst, species, max_n, n, w)
                                : read_weights_impl<float>(h, inst, species, max_n, n, w);
}

int slpic_read_fields(slpic_t* h, int inst, double* rho, double* phi, double* E) {
  if (!h || inst < 0 || inst >= h->n_inst) return fail(h, SLPIC_INVALID_ARG, "bad instance");
  Global G;
  uint32_t slot3, bsel;
  int rc = current(h, G, slot3, bsel);
  if (rc) return rc;
  const size_t base = (size_t)(G.cur_gen % 2u) * h->L.total_nodes + h->ip[inst].node;
  const size_t n = (size_t)h->ip[inst].cells + 1;
  if (rho) HIPCHK(h, hipMemcpy(rho, h->ws + h->L.rho + 8 * base, 8 * n, hipMemcpyDeviceToHost));
  if (phi) HIPCHK(h, hipMemcpy(phi, h->ws + h->L.phi + 8 * base, 8 * n, hipMemcpyDeviceToHost));
  if (E) HIPCHK(h, hipMemcpy(E, h->ws + h->L.E64 + 8 * base, 8 * n, hipMemcpyDeviceToHost));
  return SLPIC_OK;
}

int slpic_read_flux(slpic_t* h, int inst, int species, double* flux, int reset) {
  if (!h || inst < 0 || inst >= h->n_inst || (species != 0 && species != 1) || !flux)
    return fail(h, SLPIC_INVALID_ARG, "bad flux arguments");
  if (!(h->cfg.flags & SLPIC_FLAG_FLUX)) return fail(h, SLPIC_INVALID_ARG, "created without SLPIC_FLAG_FLUX");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const size_t at = h->L.flux + sizeof(double) * ((size_t)species * h->L.total_nodes + h->ip[inst].node);
  const size_t n = (size_t)h->ip[inst].cells + 1;
  HIPCHK(h, hipMemcpy(flux, h->ws + at, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (reset) HIPCHK(h, hipMemset(h->ws + at, 0, sizeof(double) * n));
  return SLPIC_OK;
}

int slpic_set_source(slpic_t* h, int inst, double per_step) {
  if (!h || inst < 0 || inst >= h->n_inst) return fail(h, SLPIC_INVALID_ARG, "bad instance");
  if (!(per_step >= 0.0 && per_step <= 16777216.0))
    return fail(h, SLPIC_INVALID_ARG, "source rate outside [0, 2^24]");
  h->ip[inst].src = per_step;
  const size_t at = h->L.ip + sizeof(InstParams) * (size_t)inst + offsetof(InstParams, src);
  HIPCHK(h, hipMemcpyAsync(h->ws + at, &h->ip[inst].src, sizeof(double), hipMemcpyHostToDevice,
                           h->stream));
  return SLPIC_OK;
}

int slpic_read_stats(slpic_t* h, int inst, int64_t first_step, int n, slpic_stats* rows) {
  if (!h || inst < 0 || inst >= h->n_inst || n < 0 || (n > 0 && !rows) || first_step < 0)
    return fail(h, SLPIC_INVALID_ARG, "bad stats arguments");
  static_assert(sizeof(StatsRow) == sizeof(slpic_stats), "stats row layout");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (first_step + n > h->steps || first_step + RING < h->steps)
    return fail(h, SLPIC_INVALID_ARG, "requested steps are not in the statistics ring");
  // at most two contiguous pieces of the ring
  for (int k = 0; k < n;) {
    const int64_t slot = (first_step + k) % RING;
    const int run = (int)std::min<int64_t>(n - k, RING - slot);
    HIPCHK(h, hipMemcpy(rows + k, h->ws + h->L.ring + sizeof(StatsRow) * ((size_t)inst * RING + slot),
                        sizeof(StatsRow) * run, hipMemcpyDeviceToHost));
    k += run;
  }
  return SLPIC_OK;
}

int slpic_scalars(slpic_t* h, int inst, double* out8) {
  if (!h || !out8 || inst < 0 || inst >= h->n_inst) return fail(h, SLPIC_INVALID_ARG, "bad scalars arguments");
  Global G;
  uint32_t slot3, bsel;
  int rc = current(h, G, slot3, bsel);
  if (rc) return rc;
  InstState st;
  HIPCHK(h, hipMemcpy(&st, h->ws + h->L.st + sizeof(InstState) * ((size_t)(G.cur_gen % 2u) * h->n_inst + inst),
                      sizeof(st), hipMemcpyDeviceToHost));
  const InstParams& P = h->ip[inst];
  out8[0] = P.dx;
  out8[1] = P.dt;
  out8[2] = P.v0;
  out8[3] = P.n_g;
  out8[4] = P.nu_max_e;
  out8[5] = P.nu_max_cx;
  out8[6] = st.w_j;
  out8[7] = st.step;
  return SLPIC_OK;
}

int64_t slpic_steps_done(const slpic_t* h) { return h ? h->steps : -1; }

const char* slpic_last_error(const slpic_t* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

void slpic_destroy(slpic_t* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  release_events(h);
  if (h->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_busy[h->static_dev] = false;
  }
  delete h;
}

int slpic_philox_device(const uint32_t* ctr, uint32_t key0, uint32_t key1, int64_t n,
                        uint32_t* out, void* hip_stream) {
  if (n < 0 || (n > 0 && (!ctr || !out))) return SLPIC_INVALID_ARG;
  hipError_t e = launch_philox_test(ctr, key0, key1, n, out, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? SLPIC_OK : SLPIC_HIP_ERROR;
}

}  // extern "C"
