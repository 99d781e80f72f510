// Internal layout shared by the host side (slpic_capi.cpp) and the kernels
// (slpic_kernels.hip).  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace slpic {

constexpr int BLOCK = 256;        // threads per workgroup = markers per tile
constexpr int TBLOCK = 1024;      // threads of a tail-kernel workgroup (one per instance)
constexpr int WAVE = 64;
constexpr int MAX_INST = 1024;
constexpr int MAX_CHAN = 8;
constexpr int NEV = 11;           // event counters per tile
constexpr int RING = 4096;        // statistics rows kept per instance
constexpr int MAX_PART = 16;      // output partitions per (instance, species)
constexpr int CSTRIDE = 64;       // uint32 slots between compaction counters:
                                  // one 256-byte line each, so that the
                                  // reservations of one (instance, species)
                                  // spread over memory channels
constexpr int NSLOT = 1;          // copies of each global deposit node
constexpr int NPOOL = 8;          // claim counters of the particle kernel's
                                  // work distribution
constexpr int MAX_DEVICES = 64;   // devices a process can hold a static workspace on
constexpr int HWIN = 1856;        // nodes in a workgroup's LDS deposit window
                                  // (of the species its tile holds)
constexpr uint32_t ANCHOR_PERIOD = 16;  // steps between choices of the windows
                                  // (under 30 KB of LDS per workgroup in all,
                                  // with room for the tile offsets of 256
                                  // instances: five workgroups per CU)

// bytes of the static workspace on each device (slpic_create_static)
constexpr size_t STATIC_WS_BYTES = (size_t)64 << 20;

// Tiles an (instance, species) takes in the tile space of a step: every
// partition gets as many as the fullest one needs, so that tile j of the
// pair reads chunk j mod T of partition j / T.
__host__ __device__ inline uint32_t pair_tiles(uint32_t max_count, int parts) {
  return ((max_count + (uint32_t)BLOCK - 1u) / (uint32_t)BLOCK) * (uint32_t)parts;
}

// event counter slots (order of the public slpic_stats fields)
enum Ev {
  EV_ELASTIC = 0, EV_EXCIT, EV_IONIZ, EV_CX, EV_ABS_E_CATH, EV_ABS_E_ANODE,
  EV_ABS_I_CATH, EV_ABS_I_ANODE, EV_SEE, EV_ROULETTE, EV_SPLIT
};

// device error bits
enum Err { ERR_CAPACITY = 1, ERR_NONFINITE = 2, ERR_NU_BOUND = 4 };

// Philox stream channels: the fourth counter word is channel | sub << 8
enum Chan {
  CH_COLL = 1, CH_IONIZ = 2, CH_IONBIRTH = 3, CH_CX = 4, CH_SEE = 5,
  CH_ROULETTE = 6, CH_CHILD = 7, CH_SEED = 8, CH_INJECT = 9
};

enum PopMode { POP_NONE = 0, POP_ROULETTE = 1, POP_SPLIT = 2 };

// kernel modes of the generation kernel
enum Mode { MODE_STEP = 0, MODE_REFRESH = 1 };

// Per-instance constants.  Integer thresholds t_* turn a probability P into
// the test (r >> 9) < t on a raw 32-bit Philox word, which equals
// u < P for u = (2 (r >> 9) + 1) 2^-24.
//
// Collision strategy (Sec. III): with a split fraction s in (0, 1) a marker
// is a collision candidate with probability q = min(1, P / s) (P the
// null-collision or fixed-event candidate probability) and a colliding
// candidate moves the fraction f = max(s, P) of its flux weight into the
// collision; otherwise q = P and f = 1 (whole markers).  The candidate
// thresholds below hold q, and f_e, f_cx hold f.
struct InstParams {
  double d, dx, inv_dx, dt, V, n_g, v0, area, gamma_se;
  double nu_max_e, nu_max_cx, sigma_cx;
  double qm_e, qm_i;        // signed charge over mass [C/kg]
  double vth_i;             // sqrt(k_B T / m_Ar)
  double w_j0;
  double src;               // cathode source: markers per step at weight w_j0
  double inv_v0;            // 1 / v0 (0 for PIC)
  int64_t seg;              // first slot of the instance in each species array
  int64_t cap;              // markers per species (sum over partitions)
  int64_t cap_p;            // slots per partition: partition p of the instance
                            // holds slots [seg + p cap_p, seg + (p+1) cap_p)
  int64_t n_target;
  int32_t cells, node;      // node: first node of the instance in node arrays
  int32_t limited;          // 0: plain PIC (beta == 1)
  int32_t parts;            // partitions P, a power of two (tile j reads j mod P)
  double f_e, f_cx;          // collided fraction of a colliding candidate
  double g_e, g_cx;          // 1 - f_e, 1 - f_cx (in FP64: no cancellation in FP32)
  uint32_t t_null_e, t_null_cx, t_see;  // candidate thresholds (q), emission
  uint32_t t_cand_fixed_e;   // fixed-event electron candidate threshold (q)
  uint32_t key;             // Philox key word 1 of the instance's draws
  uint32_t t_fixed[MAX_CHAN];  // fixed events, whole markers: channel k if
                               // (r.x >> 9) < t_fixed[k]
  uint32_t t_fsplit[MAX_CHAN]; // fixed events, split: channel k of a
                               // candidate if (r.y >> 9) < t_fsplit[k]
  uint32_t t_fixed_cx;         // fixed-event charge-exchange candidate (q)
  // FP32 copies of the constants that the FP32 kernels use per marker,
  // rounded once on the host (the same rounding as a conversion on the
  // device) instead of converted at every use
  float dt_f, v0_f, inv_v0_f, dx_f, inv_dx_f, qm_e_f, qm_i_f, n_g_f, nu_max_e_f, nu_max_cx_f,
      sigma_cx_f, vth_i_f, f_e_f, g_e_f, f_cx_f, g_cx_f;
};

// Markers of one (buffer, species) in chunks of CH slots.  Within a chunk
// each field's CH entries are contiguous (cell, off, vx, vy, vz, then id), so
// one address serves every field of a slot, a wave's CH slots read or write
// one contiguous segment per field, and only the chunk array's base is a
// kernel argument.  Partitions start on chunk boundaries.
constexpr int CH = 64;  // slots per chunk (the shifts below assume 64)
template <typename R>
struct Soa {
  char* p;  // chunk 0
  static constexpr int64_t kChunk = (int64_t)CH * (4 + 4 * (int64_t)sizeof(R) + 8);
  static constexpr int64_t kOff = 4 * CH, kVx = kOff + CH * (int64_t)sizeof(R),
                           kVy = kVx + CH * (int64_t)sizeof(R), kVz = kVy + CH * (int64_t)sizeof(R),
                           kId = kVz + CH * (int64_t)sizeof(R);
  // slot indices are never negative: chunk and lane by shift and mask
  __host__ __device__ char* chunk(int64_t s) const { return p + (int64_t)((uint64_t)s >> 6) * kChunk; }
  __host__ __device__ static int64_t lane(int64_t s) { return (int64_t)((uint64_t)s & (CH - 1)); }
  __host__ __device__ int32_t& cell(int64_t s) const { return *(int32_t*)(chunk(s) + lane(s) * 4); }
  __host__ __device__ R& off(int64_t s) const { return *(R*)(chunk(s) + kOff + lane(s) * (int64_t)sizeof(R)); }
  __host__ __device__ R& vx(int64_t s) const { return *(R*)(chunk(s) + kVx + lane(s) * (int64_t)sizeof(R)); }
  __host__ __device__ R& vy(int64_t s) const { return *(R*)(chunk(s) + kVy + lane(s) * (int64_t)sizeof(R)); }
  __host__ __device__ R& vz(int64_t s) const { return *(R*)(chunk(s) + kVz + lane(s) * (int64_t)sizeof(R)); }
  __host__ __device__ uint64_t& id(int64_t s) const { return *(uint64_t*)(chunk(s) + kId + lane(s) * 8); }
};

// Slot j of one partition as byte offsets from the partition's first chunk.
// Partitions start on chunk boundaries and the host keeps a partition's
// bytes under 2^31, so the offsets fit 32 bits and the chunk base can stay
// in scalar registers (one wave works on one partition at a time).
template <typename R>
struct SlotOff {
  uint32_t o4;  // a 4-byte field's offset: chunk * kChunk + lane * 4
  uint32_t o8;  // an 8-byte field's: o4 + lane * 4
  __host__ __device__ explicit SlotOff(uint32_t j) {
    const uint32_t l4 = (j << 2) & (uint32_t)(4 * CH - 4);
    // a partition under 2^31 bytes has fewer than 2^24 chunks: a 24-bit
    // multiply-add
    o4 = ((j >> 6) & 0xffffffu) * (uint32_t)Soa<R>::kChunk + l4;
    o8 = o4 + l4;
  }
  __host__ __device__ uint32_t oR() const { return sizeof(R) == 4 ? o4 : o8; }
};

template <typename R>
struct Part {
  char* b;  // the partition's first chunk
  __host__ __device__ int32_t& cell(const SlotOff<R>& q) const { return *(int32_t*)(b + q.o4); }
  __host__ __device__ R& off(const SlotOff<R>& q) const { return *(R*)(b + Soa<R>::kOff + q.oR()); }
  __host__ __device__ R& vx(const SlotOff<R>& q) const { return *(R*)(b + Soa<R>::kVx + q.oR()); }
  __host__ __device__ R& vy(const SlotOff<R>& q) const { return *(R*)(b + Soa<R>::kVy + q.oR()); }
  __host__ __device__ R& vz(const SlotOff<R>& q) const { return *(R*)(b + Soa<R>::kVz + q.oR()); }
  __host__ __device__ uint64_t& id(const SlotOff<R>& q) const { return *(uint64_t*)(b + Soa<R>::kId + q.o8); }
};

// identical layout to the public slpic_stats
struct StatsRow {
  int64_t step, n_e, n_i, n_in;
  double w_e, w_i, w_j;
  int64_t ev[NEV];
  int64_t err;
};

struct InstState {
  double w_j;
  uint32_t step;
  int32_t popmode;
  int32_t dshift;   // fraction bits of this step's fixed-point deposit: the
                    // handle's base, raised with weight splitting by
                    // floor(-log2) of the largest marker flux weight, so
                    // that deposits keep their resolution as weights shrink
  int32_t anchor[2];  // first node of each species' deposit window for
                      // markers not in cell order: of the windows inside
                      // the gap, the one that took the species' largest
                      // deposit in the last step the tail kernel chose on
};

// Handle-wide device words.  Per-step state is buffered by generation: a
// launch pair reads generation g and writes g + 1.  The particle kernel
// reads g from cur_gen (written only by tail kernels) and passes it to the
// tail kernel in tail_gen; the tail kernel sets cur_gen to g + 1.  Launches
// therefore take no host arguments, so a captured graph can replay them.
struct Global {
  uint32_t tail_gen;    // generation the last particle kernel advanced from
  uint32_t pad;
  uint32_t cur_gen;     // generation of the current state (set by tails)
  uint32_t bufsel[2];   // particle buffer holding generation g's markers
  uint32_t err;
  // tiles claimed so far from each pool of the particle kernel's work
  // distribution, by the particle kernel of generation g in claim[g % 2]
  // (reset for g + 1 by the tail kernel of g); one 256-byte line each
  uint32_t claim[2][NPOOL][CSTRIDE];
};

template <typename R>
struct Ctx {
  const InstParams* ip;
  Soa<R> buf[2][2];          // [buffer][species]
  InstState* st;             // [2][n_inst]
  uint32_t* counts;          // [3][n_inst][2][MAX_PART], CSTRIDE apart
  unsigned long long* ev;    // [n_inst][NEV][NSLOT] event counters of a step
  unsigned long long* acc;   // [2 species][NSLOT][total_nodes] fixed-point deposit
  R* E;                      // [2][total_nodes] field in kernel precision
  double* E64;               // [2][total_nodes]
  double* phi;               // [2][total_nodes]
  double* rho;               // [2][total_nodes]
  StatsRow* ring;            // [n_inst][RING]
  uint32_t* inst_err;        // [n_inst], sticky
  Global* g;
  const R* xs_e;             // [n_grid] node energies
  const R* xs_sig;           // [n_grid][2][ncp]: each node's cross sections,
                             // then their changes to the next node (zero
                             // past n_chan and at the last node)
  const R* xs_thr;           // [MAX_CHAN] thresholds (+inf past n_chan)
  const int32_t* xs_kind;    // [MAX_CHAN]
  R log_emin, inv_dlog;      // log-uniform grid index
  R log2_ratio, ratio_m1;    // log2 of the node ratio g, and g - 1
  R e_lo, e_hi;              // first and last node energies
  double ion_B;
  int n_chan, n_grid;
  int ncp;                   // channels per table row: 4 or MAX_CHAN
  int n_inst, total_nodes, grid, max_tiles;
  int fixed;
  uint32_t flags, seed;
  int dep_shift;             // base fraction bits of the fixed-point deposit
  uint32_t* maxw;            // [n_inst] largest flux weight (float bits) among a
                             // step's outputs (weight splitting)
  int tail_lds;              // dynamic LDS bytes of the tail kernel
  int gen_lds;               // dynamic LDS bytes of the particle kernel
  uint32_t* sort_hist;       // [2][total_nodes] cell counts of the cell sort
  uint32_t* sort_cur;        // [2][total_nodes] cursors of the cell sort
  uint32_t* tiles;           // [3][n_inst][2] tiles of each (instance, species)
  int32_t* cross;            // [2][total_nodes] net upward node crossings of a step
  double* flux;              // [2][total_nodes] time-integrated flux (w_j units)
  int max_cells;             // largest cell count of the batch
  R* wt[2][2];               // [buffer][species] flux weight of each marker slot
                             // in units of w_j (weight splitting only, else NULL)
  int split;                 // weight splitting (split fraction in (0, 1))
  int dist;                  // work distribution of the particle kernel:
                             // 0 equal contiguous shares, 1 claimed runs
  int sorted;                // markers are cell-sorted now and then (resort_period > 0)
  int occ;                   // waves per SIMD of the FP32 particle kernel's
                             // launch shape (4, 5 or 6)
  int sort_lds1, sort_lds2;  // dynamic LDS bytes of the sort's count and scatter
};

}  // namespace slpic
