/*
 * slpic.h -- C ABI of the MI355X speed-limited PIC / Monte Carlo collision
 * particle step for a 1D3V electron / Ar+ cascade across a gas-filled gap.
 *
 * Method: Theis, Werner, Jenkins & Cary, "Computing the Paschen curve for
 * argon with speed-limited particle-in-cell simulation".  One call to
 * slpic_step advances every marker of every instance by one time step:
 *   - speed-limited motion, Eqs. (8)-(9) with beta(v) of Eq. (11), integrated
 *     exactly for the field gathered at the start of the step;
 *   - null-collision Monte Carlo collisions with the SLPIC rate of
 *     Eqs. (15)-(16) (elastic, excitation, ionization with new electron and
 *     ion markers; constant cross-section Ar+ charge exchange);
 *   - ion-induced secondary electron emission at the cathode (Sec. IV);
 *   - linear-weighting charge deposit with density weight w_p = beta w_j
 *     (Sec. III) and a 1D Poisson solve in FP64.
 *
 * Conventions for every entry point:
 *   - return value: SLPIC_OK (0) or a negative slpic_status; no exception
 *     crosses the ABI; slpic_last_error() gives a readable message;
 *   - "host" pointers are read (or written) before the call returns and are
 *     not retained; "device" pointers are borrowed for the handle's lifetime;
 *   - the handle is bound to one HIP stream given at create time, launches
 *     all work on it, and is not thread-safe;
 *   - units are SI except the pressure (Torr) and energies (eV);
 *   - the cathode is at x = 0 (potential 0), the anode at x = d (potential V).
 */
#ifndef SLPIC_H
#define SLPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SLPIC_ABI_VERSION 1
#define SLPIC_MAX_PARTITIONS 16
/* bytes of the per-device static workspace used by slpic_create_static */
#define SLPIC_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

typedef enum slpic_status {
  SLPIC_OK = 0,
  SLPIC_INVALID_ARG = -1,        /* a parameter is out of range */
  SLPIC_WORKSPACE_TOO_SMALL = -2,
  SLPIC_CAPACITY_EXCEEDED = -3,  /* a species outgrew its capacity; the
                                    excess markers were dropped */
  SLPIC_NONFINITE_STATE = -4,    /* a marker reached a non-finite state and
                                    was dropped */
  SLPIC_HIP_ERROR = -5,
  SLPIC_NU_BOUND_EXCEEDED = -6,  /* a collision rate exceeded the
                                    null-collision bound */
  SLPIC_NOT_BUILT = -7
} slpic_status;

/* channel kinds, seed modes, species, flags */
enum { SLPIC_ELASTIC = 0, SLPIC_EXCITATION = 1, SLPIC_IONIZATION = 2 };
enum { SLPIC_SEED_NONE = 0, SLPIC_SEED_CATHODE = 1, SLPIC_SEED_MAXWELL_CELL0 = 2 };
enum { SLPIC_ELECTRON = 0, SLPIC_ION = 1 };
/* SLPIC_FLAG_PRODUCTS_AT_REST: both electrons of an ionization leave at rest
 * (a closed-form Townsend test gas, not physical argon).
 * SLPIC_FLAG_SEE_ENERGY: an ion reaching the cathode emits an electron with
 * the probability of Eq. (17) (Sec. IV) at its impact energy,
 * 0.09 (eps/700 eV)^0.05 below 700 eV and 0.09 (eps/700 eV)^0.72 above,
 * instead of the constant gamma_se; at most one electron per ion (the yield
 * stays below 1 up to about 20 keV).
 * SLPIC_FLAG_FLUX: keep the time-integrated flux through every node for
 * slpic_read_flux (Eq. (12) and the passage after it); costs one atomic per
 * marker that changes cell. */
enum { SLPIC_FLAG_PRODUCTS_AT_REST = 1, SLPIC_FLAG_SEE_ENERGY = 2, SLPIC_FLAG_FLUX = 4 };

/* Settings shared by all instances of a handle. */
typedef struct slpic_config {
  int32_t precision;     /* 32: FP32 particles, FP64 field and totals;
                            64: FP64 throughout */
  uint32_t seed;         /* Philox key word 0 (word 1: slpic_instance.stream) */
  uint32_t flags;        /* SLPIC_FLAG_* */
  int32_t resort_period; /* cell sort of the markers before every step whose
                            count of completed steps is a multiple of it
                            (step 0 included); 0 = off (see slpic_sort) */
  double T_gas;          /* neutral temperature [K], > 0 */
  double area;           /* electrode area [m^2], > 0 */
  double w_j0;           /* initial flux weight w_j of every marker, > 0 */
  double cfl;            /* v0 dt / dx in (0, 1] when dt is derived */
  double ion_B_eV;       /* ionization energy-sharing parameter [eV] */
  double kTe_seed_eV;    /* temperature of Maxwellian seed electrons [eV] */
  double split_frac;     /* collision strategy (Sec. III), in [0, 1].  0 or 1:
                            whole markers -- a candidate collides with its
                            full flux weight, every marker of an instance
                            shares w_j.  s in (0, 1): weight splitting --
                            markers carry their own flux weight; a marker is
                            a candidate with probability q = min(1, P / s)
                            (P the null-collision, or fixed-event, candidate
                            probability) and a colliding candidate moves the
                            fraction f = max(s, P) of its weight into the
                            collision: the primary stays with 1 - f of its
                            weight, velocity and id, a new marker (id from
                            Philox channel 7, sub 2) leaves with f and the
                            scattered velocity, and ionization products
                            carry f.  The expected collided weight equals the
                            whole-marker one (q f = P).  Not available with
                            SLPIC_FLAG_FLUX. */
} slpic_config;

/* One independent gap (p, d, V). */
typedef struct slpic_instance {
  double d;          /* gap [m], > 0 */
  double p_torr;     /* neutral pressure [Torr], >= 0 */
  double V;          /* anode potential [V] */
  double gamma_se;   /* secondary electrons per ion reaching the cathode,
                        in [0, 1] */
  double v_limit;    /* speed limit v0 [m/s]; <= 0: sqrt(2 e |V| / m_Ar)
                        (Sec. IV); +INFINITY: beta == 1, plain PIC */
  double dt;         /* time step [s]; <= 0: cfl dx / v0, or for plain PIC
                        cfl dx / sqrt(2 e |V| / m_e) (Sec. IV) */
  int32_t cells;     /* >= 2 */
  int32_t seed_mode; /* SLPIC_SEED_* */
  int64_t n_seed;    /* seed electrons (ids 0 .. n_seed-1) */
  int64_t n_target;  /* population-control target; 0 = off.  Before each
                        step with N markers: N > 2 n_target keeps each output
                        marker with probability 1/2 and doubles w_j;
                        0 < N < n_target/2 clones each and halves w_j */
  int64_t capacity;  /* marker slots per species, >= n_seed; the library
                        splits them into output partitions and rounds each
                        up to whole chunks of 64 slots (slpic_partitions
                        reports the result) */
  int64_t stream;    /* Philox key word 1 of every draw of this instance
                        (seeding included), in [0, 2^32); < 0: the
                        instance's index in the batch.  Instances with equal
                        seed, stream and inputs evolve identically whatever
                        batch they are in. */
} slpic_instance;

/* Electron-neutral cross sections: piecewise linear in energy between
 * log-uniform nodes e_j = e_min (e_max/e_min)^(j/(n_grid-1)), constant
 * beyond either end, zero below the channel threshold. */
typedef struct slpic_xs {
  int32_t n_chan;               /* 0 .. 8 */
  int32_t n_grid;               /* >= 2 */
  const double* energies;       /* host [n_grid] eV, log-uniform, increasing */
  const double* sigma;          /* host [n_chan][n_grid] m^2, >= 0 */
  const double* threshold_eV;   /* host [n_chan] */
  const int32_t* kind;          /* host [n_chan] SLPIC_ELASTIC/EXCITATION/IONIZATION */
  const double* fixed_prob;     /* host [n_chan] or NULL.  If given, channel k
                                   happens with this constant per-step
                                   probability (fixed-event test mode) */
  double fixed_prob_cx;         /* fixed-event mode: per-step Ar+ charge
                                   exchange probability */
  double sigma_cx;              /* Ar+ charge exchange cross section [m^2] */
} slpic_xs;

/* Per-step statistics of one instance (one row per step). */
typedef struct slpic_stats {
  int64_t step;            /* steps completed */
  int64_t n_e, n_i;        /* markers after the step */
  int64_t n_in;            /* markers entering the step */
  double w_e, w_i;         /* sum of density weights beta w_j per species */
  double w_j;              /* flux weight after the step */
  int64_t elastic, excitation, ionization, cx;
  int64_t abs_e_cathode, abs_e_anode, abs_i_cathode, abs_i_anode;
  int64_t see;             /* secondary electrons emitted */
  int64_t roulette;        /* markers removed by population control */
  int64_t split;           /* markers cloned by population control */
  int64_t err;             /* error bits raised during the step */
} slpic_stats;

typedef struct slpic_handle slpic_t;

/* Device workspace size in bytes for the given setup, or 0 if invalid. */
size_t slpic_workspace_bytes(const slpic_config* cfg, const slpic_instance* inst,
                             int n_inst, const slpic_xs* xs);

/* Create a handle for n_inst instances (1 .. 1024).  All host arrays are
 * copied.  dev_workspace (device, >= slpic_workspace_bytes, 256-byte
 * aligned) and hip_stream (a hipStream_t, NULL = default stream) are
 * borrowed until slpic_destroy.  Seeds each instance, solves its initial
 * field and synchronizes the stream.  On failure *out is NULL.
 * SLPIC_INVALID_ARG if the device's shared memory per block cannot hold
 * 16 bytes per node of the largest instance (the per-instance field solve;
 * about 10,000 cells on a 160 KB device), or if a marker partition would
 * take 2 GiB or more (capacity above about 1.2e9 markers per instance in
 * FP32, 7.8e8 in FP64, at 16 partitions). */
int slpic_create(const slpic_config* cfg, const slpic_instance* inst, int n_inst,
                 const slpic_xs* xs, void* dev_workspace, size_t ws_bytes,
                 void* hip_stream, slpic_t** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): create a
 * handle exactly as slpic_create does, but with its device workspace in a
 * static array that the library holds on each device until the process ends,
 * SLPIC_STATIC_WORKSPACE_BYTES (64 MiB) per device.  The library allocates
 * no device memory for it, here or in any later call on the handle, and the
 * caller passes none.  The array of the current device is used; a handle
 * made this way computes exactly what an slpic_create handle of the same
 * setup computes.
 *   - SLPIC_WORKSPACE_TOO_SMALL if slpic_workspace_bytes of the setup
 *     exceeds SLPIC_STATIC_WORKSPACE_BYTES (nothing is launched);
 *   - SLPIC_INVALID_ARG while another handle made by this call on the same
 *     device is alive: the array holds one handle's state at a time, so
 *     handles on one device cannot overlap (slpic_destroy frees the array
 *     for the next create; its contents then stay as the last handle left
 *     them, and create re-initialises everything a step reads);
 *   - otherwise as slpic_create.
 * Not thread-safe with respect to other calls on the handle. */
int slpic_create_static(const slpic_config* cfg, const slpic_instance* inst, int n_inst,
                        const slpic_xs* xs, void* hip_stream, slpic_t** out);

/* Enqueue n_steps steps of every instance on the handle's stream and return
 * without waiting.  Errors raised on the device are reported by slpic_sync. */
int slpic_step(slpic_t* h, int n_steps);

/* Sort the markers of every instance and species by cell now (enqueued on the
 * handle's stream, returns without waiting).  Partition p of an (instance,
 * species) with n markers then holds the p-th run of ceil(n / partitions)
 * markers in cell order; within a cell the order is unspecified.  Results of
 * later steps do not depend on marker order.  SLPIC_INVALID_ARG if the
 * device's shared memory per block cannot hold the sort's per-cell tables
 * (about 8 bytes per cell of the largest instance). */
int slpic_sort(slpic_t* h);

/* Wait for the stream; return the first device error raised since the last
 * call (SLPIC_CAPACITY_EXCEEDED, SLPIC_NONFINITE_STATE,
 * SLPIC_NU_BOUND_EXCEEDED) or SLPIC_OK. */
int slpic_sync(slpic_t* h);

/* Use a captured HIP graph of 16 steps for slpic_step (1) or plain launches
 * (0).  Default 0.  Enabling captures the graph at once (capture runs
 * nothing), unless kernel timing is on; slpic_step replays it for every
 * whole period of its steps and launches the rest one by one. */
int slpic_use_graph(slpic_t* h, int enable);

/* Launch shape.  The particle kernel runs on a grid of workgroups that each
 * take a contiguous run of 256-marker tiles; the FP32 whole-marker kernel
 * also comes in two register budgets, compiled for 4 or 5 (the default)
 * waves per SIMD.  Results do not depend on the grid or the budget
 * (random numbers are keyed by marker id and step, deposits are exact
 * fixed-point sums), only the time does.  slpic_autotune times trial_steps
 * steps (after one untimed step) for each candidate shape -- every budget
 * with grids of a quarter, half and all of the compute units and 1 .. the
 * resident maximum workgroups per compute unit, each with both work
 * distributions (slpic_set_work_distribution) -- in three interleaved
 * rounds, keeps the candidate with the smallest median time and writes its
 * grid to *grid (host, may be NULL).  Tuning a handle per size class of
 * instances (marker count x cells) tunes each class's shape.  The trial
 * steps are ordinary steps of the simulation and count in
 * slpic_steps_done.  Synchronizes; drops a captured graph. */
int slpic_autotune(slpic_t* h, int trial_steps, int* grid);

/* Current launch shape (host outputs): the particle-kernel grid and the
 * waves per SIMD of its register budget (0 where the handle has one
 * kernel only: FP64 or weight splitting). */
int slpic_launch_shape(slpic_t* h, int* grid, int* waves_per_simd);

/* Set the launch shape (as chosen by slpic_autotune, e.g. on another handle
 * of the same size class): grid >= 1 (capped at the tile count), waves per
 * SIMD 4 or 5 for FP32 whole markers, 0 otherwise; else SLPIC_INVALID_ARG.
 * Synchronizes; drops a captured graph. */
int slpic_set_launch_shape(slpic_t* h, int grid, int waves_per_simd);

/* Work distribution of the particle kernel.  claimed == 1 (the default
 * unless markers are cell-sorted, resort_period > 0): every workgroup
 * claims runs of consecutive tiles from counters of the step, the runs
 * shrinking as the step ends, so that workgroups that draw costly tiles
 * (electrons against ions, high collision rates) do not hold the launch
 * while others idle; claimed == 0: equal contiguous shares of the tiles
 * (cell-sorted markers keep their deposits in a workgroup's LDS window
 * best this way).  Both give the same results bit for bit; slpic_autotune
 * times both.  Synchronizes; drops a captured graph.  Else
 * SLPIC_INVALID_ARG. */
int slpic_set_work_distribution(slpic_t* h, int claimed);

/* Current work distribution (host output): 1 claimed runs, 0 equal shares. */
int slpic_work_distribution(slpic_t* h, int* claimed);

/* Current particle-kernel grid (host output). */
int slpic_grid(slpic_t* h, int* grid);

/* Kernel timing.  enable != 0 starts recording HIP events on the handle's
 * stream before the particle kernel, between it and the per-instance tail
 * kernel, and after the tail kernel of every following step (steps are then
 * launched one by one, never from the graph) and clears the totals;
 * enable == 0 adds what is pending to the totals and stops.  The handle owns
 * the events.  Returns SLPIC_HIP_ERROR if events cannot be created. */
int slpic_profile(slpic_t* h, int enable);

/* Totals since profiling was last enabled: summed particle-kernel and
 * tail-kernel durations [ms] and the number of steps they cover.  Waits for
 * the recorded events.  All three outputs are host pointers and must be
 * non-NULL (else SLPIC_INVALID_ARG). */
int slpic_kernel_times(slpic_t* h, double* gen_ms, double* tail_ms, int64_t* steps);

/* Replace the markers of one species of one instance with n host-side
 * markers (x = (cell + off) dx, cell in [0, cells), off in [0, 1)), then
 * rebuild that handle's fields.  Synchronizes. */
int slpic_load_markers(slpic_t* h, int inst, int species, int64_t n,
                       const int32_t* cell, const double* off, const double* vx,
                       const double* vy, const double* vz, const uint64_t* id);

/* Number of markers of one species of one instance.  Synchronizes. */
int slpic_count(slpic_t* h, int inst, int species, int64_t* n);

/* Storage diagnostics: markers of one species of one instance are kept in
 * *parts (at most SLPIC_MAX_PARTITIONS) output partitions of *cap_p slots
 * each (the capacity split for spreading compaction counters); counts (host,
 * SLPIC_MAX_PARTITIONS entries) receives each partition's occupancy, zero
 * past *parts.  Synchronizes. */
int slpic_partitions(slpic_t* h, int inst, int species, int32_t* parts, int64_t* cap_p,
                     uint32_t* counts);

/* Copy one species of one instance to host arrays of at least max_n
 * entries (NULL to skip an array); *n receives the count.  Synchronizes. */
int slpic_read_markers(slpic_t* h, int inst, int species, int64_t max_n,
                       int64_t* n, int32_t* cell, double* off, double* vx,
                       double* vy, double* vz, uint64_t* id);

/* Flux weights (in units of the instance's w_j, as in slpic_scalars) of the
 * markers of one species of one instance, in slpic_read_markers' order:
 * host array w of at least max_n entries; *n receives the count.  Only with
 * weight splitting (split_frac in (0, 1)), else SLPIC_INVALID_ARG.
 * Synchronizes. */
int slpic_read_weights(slpic_t* h, int inst, int species, int64_t max_n, int64_t* n,
                       double* w);

/* Node arrays (cells + 1 each, host, NULL to skip) of one instance: charge
 * density [C/m^3], potential [V] and field [V/m].  Synchronizes. */
int slpic_read_fields(slpic_t* h, int inst, double* rho, double* phi, double* E);

/* Time-integrated flux through each node of one instance and species (Eq. (12)
 * and the passage after it: a marker crossing a surface carries its flux
 * weight w_j through it, whatever its speed), summed over the steps since
 * create or the last read with reset != 0: each step adds w_j times the
 * net number of markers that crossed the node in +x.  A marker crosses node
 * k upward when its cell goes from below k to k or above during the step
 * (downward likewise); a marker absorbed at the cathode (anode) ends below
 * node 0 (above node cells), so nodes 0 and cells give the electrode fluxes.
 * flux: host array of cells + 1 doubles, node 0 at the cathode.  Needs
 * SLPIC_FLAG_FLUX at create, else SLPIC_INVALID_ARG.  Synchronizes. */
int slpic_read_flux(slpic_t* h, int inst, int species, double* flux, int reset);

/* Continuous cathode source of one instance (the electrons at rest at x = 0
 * with which Sec. IV starts a run, injected every step; a steady source
 * gives the steady state in which Sec. II.B finds the speed-limited
 * equations exact).  per_step: markers per step at the initial flux weight
 * w_j0, so the physical rate per_step w_j0 / dt holds under population
 * control: at flux weight w_j a step injects per_step w_j0 / w_j markers,
 * the integer part and one more with the probability of the fraction
 * (Philox channel 9, sub 1, counter (0, 0, step)); marker k of the step has
 * the id made from channel 9, sub 0, counter (k, 0, step), with the top bit
 * set.  The electrons join the step's output (after its pushes and
 * collisions, as secondary electrons do), take part in its population
 * control and deposit their charge on node 0.  0 switches the source off.
 * Enqueued on the handle's stream: takes effect from the next step,
 * captured graphs included.  SLPIC_INVALID_ARG unless 0 <= per_step <= 2^24
 * (and finite).  A step whose injections overflow the instance's capacity
 * reports SLPIC_CAPACITY_EXCEEDED like any other overflow. */
int slpic_set_source(slpic_t* h, int inst, double per_step);

/* Statistics rows of one instance for steps first_step+1 .. first_step+n
 * (row k describes step first_step+k+1), from a ring of the last 4096 steps.
 * Synchronizes. */
int slpic_read_stats(slpic_t* h, int inst, int64_t first_step, int n,
                     slpic_stats* rows);

/* Derived scalars of one instance: dx, dt, v0, n_g, nu_max_e, nu_max_cx,
 * w_j, step (8 doubles, host).  Synchronizes. */
int slpic_scalars(slpic_t* h, int inst, double* out8);

/* Steps completed by the handle (host-side count, no synchronization). */
int64_t slpic_steps_done(const slpic_t* h);

/* Message describing the last failure on this handle (or of the last
 * create when h is NULL). */
const char* slpic_last_error(const slpic_t* h);

/* Wait for the stream and release host-side resources; the workspace stays
 * owned by the caller. */
void slpic_destroy(slpic_t* h);

/* Test hook: Philox4x32-10 on the device.  ctr is device [n][4] uint32, out
 * device [n][4]; key (key0, key1).  Enqueued on stream, not waited for. */
int slpic_philox_device(const uint32_t* ctr, uint32_t key0, uint32_t key1,
                        int64_t n, uint32_t* out, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SLPIC_H */
