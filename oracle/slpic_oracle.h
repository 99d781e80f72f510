/*
 * Oracle for the SLPIC-MCC particle step: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of one speed-limited
 * particle-in-cell step with Monte Carlo collisions, written from the paper
 * (Theis, Werner, Jenkins & Cary, "Computing the Paschen curve for argon with
 * speed-limited particle-in-cell simulation").  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the GPU library
 * never links or calls it, and it shares no code with the GPU library.
 *
 * Layout of every struct here is mirrored by ctypes in oracle/__init__.py.
 */
#ifndef SLPIC_ORACLE_H
#define SLPIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* channel kinds, seed modes (same numbering as the synthetic inputs) */
enum { OR_ELASTIC = 0, OR_EXCITATION = 1, OR_IONIZATION = 2 };
enum { OR_SEED_NONE = 0, OR_SEED_CATHODE = 1, OR_SEED_MAXWELL_CELL0 = 2 };
enum { OR_ELECTRON = 0, OR_ION = 1 };

/* Philox stream channels (fourth counter word = channel | sub << 8) */
enum {
  OR_CH_COLL = 1, OR_CH_IONIZ = 2, OR_CH_IONBIRTH = 3, OR_CH_CX = 4,
  OR_CH_SEE = 5, OR_CH_ROULETTE = 6, OR_CH_CHILD = 7, OR_CH_SEED = 8,
  OR_CH_INJECT = 9
};

/* per-step statistics row */
enum {
  OR_ST_STEP = 0, OR_ST_NE, OR_ST_NI, OR_ST_WE, OR_ST_WI, OR_ST_WJ,
  OR_ST_ELASTIC, OR_ST_EXCIT, OR_ST_IONIZ, OR_ST_CX,
  OR_ST_ABS_E_CATH, OR_ST_ABS_E_ANODE, OR_ST_ABS_I_CATH, OR_ST_ABS_I_ANODE,
  OR_ST_SEE, OR_ST_ROULETTE, OR_ST_SPLIT, OR_ST_NIN, OR_ST_ERR,
  OR_NSTAT
};

/* flags: OR_FLAG_PRODUCTS_AT_REST leaves both electrons of an ionization at
 * rest (the closed-form Townsend test gas); OR_FLAG_SEE_ENERGY takes the
 * ion-induced emission probability from the ion's impact energy by Eq. (17)
 * (Sec. IV) instead of the constant gamma_se; OR_FLAG_FLUX keeps the flux
 * through every node (Eq. (12) and the passage after it, see or_flux) */
enum { OR_FLAG_PRODUCTS_AT_REST = 1, OR_FLAG_SEE_ENERGY = 2, OR_FLAG_FLUX = 4 };

/* error bits */
enum { OR_ERR_NU_BOUND = 1, OR_ERR_NONFINITE = 2, OR_ERR_ALLOC = 4 };

typedef struct {
  /* gap instance */
  double d;          /* electrode gap [m] */
  double p_torr;     /* neutral pressure [Torr] */
  double V;          /* anode potential [V]; cathode at 0 V */
  double gamma_se;   /* secondary electrons per ion hitting the cathode, [0,1] */
  double v_limit;    /* speed limit v0 [m/s]; <= 0: sqrt(2 e V / m_Ar); +inf: PIC */
  double dt;         /* time step [s]; <= 0: cfl dx / v0 (PIC: cfl dx / v_max) */
  double T_gas;      /* neutral temperature [K] */
  double area;       /* electrode area [m^2] */
  double w_j0;       /* initial flux weight of every marker */
  double cfl;
  double ion_B_eV;   /* ionization energy-sharing parameter */
  double kTe_seed_eV;/* seed electron temperature */
  double sigma_cx;   /* Ar+ charge exchange [m^2] */
  double fixed_prob_cx;
  int64_t n_seed;
  int64_t n_target;  /* population-control target, 0 = off */
  int32_t cells;
  int32_t seed_mode;
  uint32_t seed;     /* Philox key word 0 */
  uint32_t instance; /* Philox key word 1 */
  uint32_t flags;    /* OR_FLAG_* */
  int32_t pad0;
  /* electron-neutral cross sections */
  int32_t n_chan;
  int32_t n_grid;
  const double* energies;     /* [n_grid] eV */
  const double* sigma;        /* [n_chan][n_grid] m^2 */
  const double* threshold_eV; /* [n_chan] */
  const int32_t* kind;        /* [n_chan] */
  const double* fixed_prob;   /* [n_chan] or NULL */
  /* collision strategy (Sec. III): 0 or 1 collides whole markers; s in
   * (0, 1) splits a colliding marker, moving the fraction max(s, P) of its
   * flux weight into the collision (see collide_electron) */
  double split_frac;
} or_params;

typedef struct or_sim or_sim;

or_sim* or_create(const or_params* p);
void or_destroy(or_sim* s);
/* replace one species' population (x = (cell + off) dx) and rebuild fields */
int or_load(or_sim* s, int species, int64_t n, const int32_t* cell,
            const double* off, const double* vx, const double* vy,
            const double* vz, const uint64_t* id);
int or_step(or_sim* s, int n_steps);
int64_t or_count(const or_sim* s, int species);
/* copy a species out; tie[] receives the smallest relative decision margin
 * along each marker's history (NULL to skip any output array) */
int or_read(const or_sim* s, int species, int32_t* cell, double* off,
            double* vx, double* vy, double* vz, uint64_t* id, double* tie);
/* flux weights of a species' markers in units of w_j, in or_read's order */
int or_read_weights(const or_sim* s, int species, double* w);
/* node arrays of length cells+1 (NULL to skip) */
void or_fields(const or_sim* s, double* rho, double* phi, double* E);
/* Time-integrated flux through each node (cells + 1 doubles, node 0 the
 * cathode) of one species since creation or the last or_flux_reset, with
 * OR_FLAG_FLUX: every step adds w_j times the net number of markers that
 * crossed the node in +x.  A marker crosses node k upward when
 * floor(x0/dx) < k <= floor(x1/dx) for its positions x0, x1 before and after
 * the flight, downward in the opposite case; a marker absorbed at the
 * cathode (anode) ends in cell -1 (cells). */
void or_flux(const or_sim* s, int species, double* out);
void or_flux_reset(or_sim* s);
/* Continuous cathode source: the seeding of Sec. IV (electrons at rest at
 * x = 0) repeated every step, which gives the steady state in which Sec. II.B
 * finds the speed-limited equations exact.  per_step is the number of
 * markers a step injects at the initial flux weight w_j0, so the physical
 * rate per_step w_j0 / dt stays fixed when population control changes w_j:
 * at weight w_j a step injects per_step w_j0 / w_j markers, the integer part
 * and one more with the probability of the fraction (Philox channel INJECT,
 * sub 1, counter (0, 0, step)).  Marker k of the step takes the id made from
 * Philox channel INJECT, sub 0, counter (k, 0, step).  Injected electrons
 * join the step's output as the secondary electrons do and take part in its
 * population control.  Returns -1 (and changes nothing) unless per_step is
 * finite and in [0, 2^24]; 0 switches the source off. */
int or_set_source(or_sim* s, double per_step);
/* Takes over an instance mid-run: the step counter (which keys every draw)
 * and the flux weight w_j that a run reached, then the charge density and
 * field of the markers present (as or_load leaves them).  Returns -1 (and
 * changes nothing) unless w_j is finite and positive. */
int or_set_clock(or_sim* s, uint32_t step, double w_j);
/* statistics of the last step, OR_NSTAT doubles */
void or_last_stats(const or_sim* s, double* row);
/* derived scalars: dx, dt, v0, n_g, nu_max_e, nu_max_cx, w_j, step */
void or_scalars(const or_sim* s, double* out8);
double or_min_margin(const or_sim* s);

/* building blocks exposed for the closed-form tests */
void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double or_beta(double v, double v0);
double or_sigma(const or_sim* s, int chan, double eps_eV);
/* exact speed-limited free flight for a uniform acceleration a along x:
 * returns the proper time tau and writes the displacement and new v_x */
double or_free_flight(double vx, double vperp, double a, double dt, double v0,
                      double* dx_out, double* vx_out);
void or_poisson(int n_cells, double dx, double V, const double* rho,
                double* phi, double* E);
/* scatter laws: new velocity for a given incident one and uniforms */
void or_scatter(int kind, const double v_in[3], double eps_out_eV,
                double u_chi, double u_phi, double vs_eps_eV, double v_out[3]);
double or_vs_cos_chi(double eps_eV, double u);
double or_ejected_energy(double eps_avail_eV, double B_eV, double u);
/* Eq. (17): secondary electrons per ion hitting the cathode with energy eps */
double or_see_yield(double eps_ion_eV);

#ifdef __cplusplus
}
#endif
#endif
