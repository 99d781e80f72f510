/*
 * Oracle for the SLPIC-MCC particle step.  TEST INFRASTRUCTURE ONLY: it is
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg,
 * never by the GPU library, with which it shares no code.
 *
 * Plain FP64 implementation of one speed-limited particle-in-cell step with
 * Monte Carlo collisions for a 1D3V electron / Ar+ cascade across a gap,
 * following the paper section by section:
 *
 *   speed limiter beta(v) ............ Eq. (11) (Sec. II.B)
 *   equations of motion .............. Eqs. (8)-(9); flux weight w_j = w_p/beta
 *                                      constant along orbits, Eq. (10)
 *   collision rate ................... Eqs. (15)-(16) (Sec. III): a SLPIC
 *                                      marker keeps the physical mean free
 *                                      path, rate n_g sigma |v| beta
 *   whole-marker events .............. Sec. III (colliding a fraction of pairs
 *                                      with the full weight); products carry
 *                                      the primary's flux weight (Sec. III)
 *   weight splitting ................. Sec. III (every colliding pair splits
 *                                      the primary: w_j,p0 = w_j,p1 + W_j,c),
 *                                      with per-marker flux weights, as the
 *                                      split_frac option (see collide_electron)
 *   density weight w_p = beta w_j .... after every kick or collision (Sec. III)
 *   setup ............................ Sec. IV: absorbing electrodes, cathode
 *                                      at x = 0, ion-induced secondary
 *                                      emission at the cathode, elastic
 *                                      scattering after Vahedi and Surendra,
 *                                      isotropic excitation
 *
 * Readings where the paper is silent (each restated at its function):
 *   - integrator: each step moves a marker along the exact solution of
 *     Eqs. (8)-(9) for the acceleration gathered at its start position; in
 *     proper time tau (dtau = beta dt) that orbit is the ordinary PIC
 *     parabola, and the wall-clock step satisfies
 *     dt = integral_0^tau max(1, |v|/v0) dtau';
 *   - null-collision sampling with bound nu'_max (finite-step form of
 *     Eq. (16));
 *   - ionization energy sharing after Vahedi and Surendra (the paper cites
 *     Kutasi et al. without giving the algorithm);
 *   - a 1D Poisson solve on the nodes (the paper imposes a constant field);
 *   - Ar+ charge exchange with a constant cross section (the paper has no ion
 *     collisions);
 *   - all random draws from Philox4x32-10 keyed by (seed, instance) with
 *     counter (id_lo, id_hi, step, channel | sub << 8).
 */
#include "slpic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define QE 1.602176634e-19
#define KB 1.380649e-23
#define ME 9.1093837015e-31
#define AMU 1.66053906660e-27
#define MAR (39.948 * AMU)
#define EPS0 8.8541878128e-12
#define TORR (101325.0 / 760.0)
#define TWO_PI 6.283185307179586476925286766559
#define TOP_BIT 0x8000000000000000ull

typedef struct {
  double x, vx, vy, vz, tie;
  uint64_t id;
  double w;  /* the marker's flux weight in units of the instance's w_j */
} marker;

typedef struct {
  marker* a;
  int64_t n, cap;
} mlist;

struct or_sim {
  or_params p;
  double *energies, *sigma, *thr, *fixed;
  int32_t* kind;
  double dx, dt, v0, n_g, nu_max_e, nu_max_cx, P_null_e, P_null_cx, w_j;
  double ecap_eV;
  uint32_t step;
  mlist e, i;
  double *Q, *rho, *phi, *E;
  double* cross[2];   /* net upward crossings of each node in this step, each
                        counted with the marker's relative weight */
  double* flux[2];    /* time-integrated flux through each node */
  double stats[OR_NSTAT];
  double min_margin;
  double src;         /* cathode source: markers per step at weight w_j0 */
  int err;
};

/* ------------------------------------------------------------------ */
/* Philox4xW-10 (Salmon, Moraes, Dror & Shaw, SC'11).  One body text serves
 * both word widths so that a check of the 64-bit instance against another
 * implementation also checks the round and key schedule used at 32 bits. */
#define PHILOX_BODY(UINT, WIDE, BITS, M0, M1, W0, W1)                     \
  UINT c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];                 \
  UINT k0 = key[0], k1 = key[1];                                           \
  for (int r = 0; r < 10; ++r) {                                           \
    if (r > 0) {                                                           \
      k0 += (UINT)(W0);                                                    \
      k1 += (UINT)(W1);                                                    \
    }                                                                      \
    WIDE p0 = (WIDE)(M0) * (WIDE)c0;                                       \
    WIDE p1 = (WIDE)(M1) * (WIDE)c2;                                       \
    UINT hi0 = (UINT)(p0 >> (BITS)), lo0 = (UINT)p0;                       \
    UINT hi1 = (UINT)(p1 >> (BITS)), lo1 = (UINT)p1;                       \
    c0 = hi1 ^ c1 ^ k0;                                                    \
    c1 = lo1;                                                              \
    c2 = hi0 ^ c3 ^ k1;                                                    \
    c3 = lo0;                                                              \
  }                                                                        \
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;

void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  PHILOX_BODY(uint32_t, uint64_t, 32, 0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u,
              0xBB67AE85u)
}

void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  PHILOX_BODY(uint64_t, unsigned __int128, 64, 0xD2E7470EE14C6C93ull,
              0xCA5A826395121157ull, 0x9E3779B97F4A7C15ull,
              0xBB67AE8584CAA73Bull)
}

/* uniform in (0,1): u = (2 (r >> 9) + 1) 2^-24, 23 random bits */
static double unif(uint32_t r) { return ((double)(r >> 9) * 2.0 + 1.0) * 0x1p-24; }

static void draw_raw(const or_sim* s, uint64_t id, uint32_t step, int ch, int sub,
                     uint32_t r[4]) {
  uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step,
                     (uint32_t)ch | ((uint32_t)sub << 8)};
  uint32_t key[2] = {s->p.seed, s->p.instance};
  or_philox4x32(ctr, key, r);
}

static uint64_t child_id(uint32_t lo, uint32_t hi) {
  return ((uint64_t)hi << 32 | lo) | TOP_BIT;
}

/* Box-Muller: two standard normals from two uniforms */
static void box_muller(double ua, double ub, double* z0, double* z1) {
  double r = sqrt(-2.0 * log(ua));
  *z0 = r * cos(TWO_PI * ub);
  *z1 = r * sin(TWO_PI * ub);
}

static void maxwellian(const uint32_t r[4], double sigma_v, double v[3]) {
  double z[4];
  box_muller(unif(r[0]), unif(r[1]), &z[0], &z[1]);
  box_muller(unif(r[2]), unif(r[3]), &z[2], &z[3]);
  v[0] = sigma_v * z[0];
  v[1] = sigma_v * z[1];
  v[2] = sigma_v * z[2];
}

/* ------------------------------------------------------------------ */
/* Eq. (11): beta = v0/v for v >= v0, 1 below (v0 = +inf gives PIC). */
double or_beta(double v, double v0) { return (v >= v0) ? v0 / v : 1.0; }

/* ------------------------------------------------------------------ */
/* Free flight.  Eqs. (8)-(9) with beta from Eq. (11) and a uniform
 * acceleration a along x.  With proper time dtau = beta dt they read
 * dx/dtau = v, dv/dtau = a: the PIC parabola.  The wall-clock time spent is
 * dt = integral max(1, |v(tau)|/v0) dtau, and |v(tau)|^2 = s^2 + c^2 with
 * s = v_x + a tau, c = |v_perp|.  Written in s (ds = |a| dtau after a
 * reflection that makes a > 0), |a| dt = I(s0, s1) with
 * I(p, q) = integral_p^q max(1, sqrt(u^2 + c^2)/v0) du. */

/* integral over [p, p + len] of sqrt(u^2 + c^2) du for p >= 0, len >= 0,
 * taking the length itself as the argument so that a step far below the
 * resolution of p keeps its size, and in a form free of cancellation
 * (q = p + len, W(u) = sqrt(u^2 + c^2)):
 *   q W(q) - p W(p)        = len (q+p)(q^2+p^2+c^2) / (q W(q) + p W(p))
 *   asinh(q/c) - asinh(p/c) = asinh(len (q+p) / (q W(p) + p W(q)))   */
static double sqrt_integral(double p, double len, double c) {
  if (len <= 0.0) return 0.0;
  double q = p + len, sq = p + q;
  if (c == 0.0) return 0.5 * len * sq;
  double Wp = sqrt(p * p + c * c), Wq = sqrt(q * q + c * c);
  double t1 = len * sq * (q * q + p * p + c * c) / (q * Wq + p * Wp);
  double t2 = c * c * asinh(len * sq / (q * Wp + p * Wq));
  return 0.5 * (t1 + t2);
}

/* I(a, a + len): split at 0 and at the speeds where |v| = v0 */
static double limit_integral(double a, double len, double c, double v0) {
  double ss = c < v0 ? sqrt(v0 * v0 - c * c) : 0.0; /* |v| = v0 at |s| = ss */
  double b = a + len;
  double brk[3] = {-ss, 0.0, ss};
  double start = a, total = 0.0;
  for (int k = 0; k <= 3; ++k) {
    double p = start, piece;
    if (k < 3) {
      if (!(brk[k] > start && brk[k] < b)) continue;
      piece = brk[k] - start;
      start = brk[k];
    } else {
      piece = (p == a) ? len : b - p;
    }
    double mid = p + 0.5 * piece;
    if (c < v0 && fabs(mid) < ss) total += piece;                    /* beta = 1 */
    else if (mid < 0.0) total += sqrt_integral(-(p + piece), piece, c) / v0; /* mirror */
    else total += sqrt_integral(p, piece, c) / v0;
  }
  return total;
}

/* inverse of I(0, s) for c = 0 (closed form), used for the Newton start */
static double inv_c0(double y, double v0) {
  return y <= v0 ? y : sqrt(2.0 * v0 * y - v0 * v0);
}

double or_free_flight(double vx, double vperp, double a, double dt, double v0,
                      double* dx_out, double* vx_out) {
  double c = fabs(vperp), tau;
  if (!(v0 < INFINITY)) {
    tau = dt; /* beta == 1: PIC */
  } else {
    double w0 = sqrt(vx * vx + c * c);
    double ve = vx + a * dt, we = sqrt(ve * ve + c * c);
    if (w0 <= v0 && we <= v0) {
      /* |v(tau)| is convex in tau, so it stays <= v0 and beta == 1 */
      tau = dt;
    } else if (a == 0.0) {
      tau = dt * v0 / w0;
    } else {
      /* reflect so the acceleration is positive and solve for the increment
       * delta = s1 - s0 of  I(s0, s0 + delta) = |a| dt,  0 < delta <= |a| dt */
      double sg = a > 0 ? 1.0 : -1.0, at = fabs(a), s0 = sg * vx;
      double rhs = at * dt, lo = 0.0, hi = rhs;
      double y0 = s0 >= 0 ? limit_integral(0.0, s0, 0.0, v0) : -limit_integral(s0, -s0, 0.0, v0);
      double delta;
      if (s0 >= 0) delta = inv_c0(y0 + rhs, v0) - s0;
      else delta = (y0 + rhs <= 0 ? -inv_c0(-(y0 + rhs), v0) : inv_c0(y0 + rhs, v0)) - s0;
      if (!(delta > lo && delta < hi)) {
        double h0 = w0 / v0 > 1.0 ? w0 / v0 : 1.0;
        delta = rhs / h0;
      }
      for (int it = 0; it < 200; ++it) {
        double f = limit_integral(s0, delta, c, v0) - rhs;
        if (f > 0) hi = delta;
        else if (f < 0) lo = delta;
        else break;
        double s = s0 + delta;
        double hp = sqrt(s * s + c * c) / v0;
        if (hp < 1.0) hp = 1.0;
        double step = -f / hp;
        if (fabs(step) <= 1e-16 * delta) { /* Newton has converged */
          if (delta + step > lo && delta + step < hi) delta += step;
          break;
        }
        double dn = delta + step;
        if (!(dn > lo && dn < hi)) dn = 0.5 * (lo + hi);
        if (dn == delta) break;
        delta = dn;
        if (hi - lo <= 4e-16 * hi) break;
      }
      tau = delta / at;
    }
  }
  *dx_out = vx * tau + 0.5 * a * tau * tau;
  *vx_out = vx + a * tau;
  return tau;
}

/* ------------------------------------------------------------------ */
/* Cross sections: piecewise-linear in energy between the table nodes,
 * constant beyond either end, zero below the channel threshold. */
double or_sigma(const or_sim* s, int k, double eps) {
  int n = s->p.n_grid;
  const double* e = s->energies;
  const double* sg = s->sigma + (size_t)k * n;
  if (eps < s->thr[k]) return 0.0;
  if (eps <= e[0]) return sg[0];
  if (eps >= e[n - 1]) return sg[n - 1];
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (e[mid] <= eps) lo = mid;
    else hi = mid;
  }
  double t = (eps - e[lo]) / (e[hi] - e[lo]);
  return sg[lo] + t * (sg[hi] - sg[lo]);
}

/* ------------------------------------------------------------------ */
/* Scatter laws.  Vahedi & Surendra elastic/ionization angle:
 * cos chi = (2 + eps - 2 (1+eps)^u) / eps  (eps in eV; isotropic as eps->0),
 * evaluated as 1 - 2 [(1+eps)^u - 1] / eps with the exact identity
 * (1+eps)^u - 1 = expm1(u log1p(eps)): the printed form loses all its digits
 * to cancellation for energies far below 1 eV. */
double or_vs_cos_chi(double eps, double u) {
  if (eps <= 0.0) return 1.0 - 2.0 * u;
  return 1.0 - 2.0 * expm1(u * log1p(eps)) / eps;
}

/* Vahedi & Surendra ejected-electron energy for available energy eps_av */
double or_ejected_energy(double eps_av, double B, double u) {
  return B * tan(u * atan(eps_av / (2.0 * B)));
}

/* Ion-induced secondary emission yield of Eq. (17) (Sec. IV): 0.09 at
 * 700 eV, growing as the 0.05 power of the impact energy below and as the
 * 0.72 power above. */
double or_see_yield(double eps) {
  return 0.09 * pow(eps / 700.0, eps < 700.0 ? 0.05 : 0.72);
}

/* Turn unit vector vh by polar angle chi and azimuth phi.  The azimuth is
 * measured in the frame e1 = normalize(vh x a), e2 = vh x e1, where a is the
 * coordinate axis along which |vh| has its smallest component (ties go to the
 * lower index).  Returns the margin of that choice: the gap between the two
 * smallest |components|, which rounding in another precision could close;
 * but infinity when both are exactly zero (a velocity along one axis, as an
 * electron released at rest has in the 1D field), a tie that resolves to
 * the same axis in any precision. */
static double rotate(const double vh[3], double cosx, double phi, double out[3]) {
  double a0 = fabs(vh[0]), a1 = fabs(vh[1]), a2 = fabs(vh[2]);
  int ax = 0;
  double amin = a0;
  if (a1 < amin) { ax = 1; amin = a1; }
  if (a2 < amin) { ax = 2; amin = a2; }
  double second = INFINITY;
  for (int k = 0; k < 3; ++k) {
    double ak = k == 0 ? a0 : (k == 1 ? a1 : a2);
    if (k != ax && ak < second) second = ak;
  }
  double e1[3];
  if (ax == 0) { e1[0] = 0.0; e1[1] = vh[2]; e1[2] = -vh[1]; }
  else if (ax == 1) { e1[0] = -vh[2]; e1[1] = 0.0; e1[2] = vh[0]; }
  else { e1[0] = vh[1]; e1[1] = -vh[0]; e1[2] = 0.0; }
  double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  e1[0] /= n1; e1[1] /= n1; e1[2] /= n1;
  double e2[3] = {vh[1] * e1[2] - vh[2] * e1[1], vh[2] * e1[0] - vh[0] * e1[2],
                  vh[0] * e1[1] - vh[1] * e1[0]};
  double sinx = sqrt(fmax(0.0, 1.0 - cosx * cosx));
  double cp = cos(phi), sp = sin(phi);
  for (int k = 0; k < 3; ++k) out[k] = cosx * vh[k] + sinx * (cp * e1[k] + sp * e2[k]);
  return (amin == 0.0 && second == 0.0) ? INFINITY : second - amin;
}

static void unit_of(const double v[3], double vh[3]) {
  double sp = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (sp > 0.0) { vh[0] = v[0] / sp; vh[1] = v[1] / sp; vh[2] = v[2] / sp; }
  else { vh[0] = 1.0; vh[1] = 0.0; vh[2] = 0.0; }
}

/* new electron velocity of energy eps_out, turned from v_in by chi, phi */
static double scatter_to(const double v_in[3], double eps_out, double cosx, double phi,
                         double v_out[3]) {
  double vh[3], d[3];
  unit_of(v_in, vh);
  double m = rotate(vh, cosx, phi, d);
  double sp = sqrt(2.0 * QE * fmax(eps_out, 0.0) / ME);
  for (int k = 0; k < 3; ++k) v_out[k] = sp * d[k];
  return m;
}

void or_scatter(int kind, const double v_in[3], double eps_out, double u_chi,
                double u_phi, double vs_eps, double v_out[3]) {
  double cosx = kind == OR_EXCITATION ? 1.0 - 2.0 * u_chi : or_vs_cos_chi(vs_eps, u_chi);
  scatter_to(v_in, eps_out, cosx, TWO_PI * u_phi, v_out);
}

/* ------------------------------------------------------------------ */
static int push_back(mlist* l, const marker* m) {
  if (l->n == l->cap) {
    int64_t nc = l->cap ? 2 * l->cap : 1024;
    marker* na = (marker*)realloc(l->a, (size_t)nc * sizeof(marker));
    if (!na) return -1;
    l->a = na;
    l->cap = nc;
  }
  l->a[l->n++] = *m;
  return 0;
}

static void note_margin(or_sim* s, marker* m, double margin) {
  if (margin < m->tie) m->tie = margin;
  if (margin < s->min_margin) s->min_margin = margin;
}

/* ------------------------------------------------------------------ */
/* Field: charge deposit with linear weights, density weight w_p = beta w_j
 * (Sec. III), and the Dirichlet Poisson problem phi(0) = 0, phi(d) = V. */
void or_poisson(int N, double dx, double V, const double* rho, double* phi, double* E) {
  /* Discrete Green's function of the Dirichlet problem.  By linearity
   * phi_i = V i/N + psi_i, where psi solves the same difference equation
   * with psi_0 = psi_N = 0 and the space charge as its source,
   *   -psi_{i-1} + 2 psi_i - psi_{i+1} = rho_i dx^2 / eps0,  i = 1..N-1,
   * whose solution is psi_i = (dx^2/eps0) sum_j G_ij rho_j with
   * G_ij = min(i,j) (N - max(i,j)) / N.  Differencing G over i gives the
   * field between nodes directly from sums of rho:
   *   E_{i+1/2} = -(phi_{i+1} - phi_i)/dx
   *             = -V/(N dx) - (dx/eps0) (R_i - M/N),
   *   R_i = sum_{j=i+1}^{N-1} rho_j,   M = sum_{j=1}^{N-1} j rho_j,
   * so E is not taken from differences of psi (which would cost digits on
   * long grids) and the vacuum field -V/d stays exact. */
  const double k = dx / EPS0;
  double M = 0.0;
  for (int j = 1; j < N; ++j) M += (double)j * rho[j];
  double* Eh = (double*)malloc(sizeof(double) * (size_t)N);  /* E_{i+1/2}, i = 0..N-1 */
  const double Ev = -V / ((double)N * dx);
  double R = 0.0;  /* R_i, built from the top */
  for (int i = N - 1; i >= 0; --i) {
    if (i + 1 <= N - 1) R += rho[i + 1];
    Eh[i] = Ev - k * (R - M / (double)N);
  }
  /* node fields: the central difference inside, Gauss's law over the half
   * cell at each electrode */
  for (int i = 1; i < N; ++i) E[i] = 0.5 * (Eh[i - 1] + Eh[i]);
  E[0] = Eh[0] - rho[0] * dx / (2.0 * EPS0);
  E[N] = Eh[N - 1] + rho[N] * dx / (2.0 * EPS0);
  free(Eh);
  /* potential: psi_i = (dx^2/eps0) [ (N-i)/N A_i + i/N B_i ] with
   * A_i = sum_{j=1}^{i} j rho_j and B_i = sum_{j=i+1}^{N-1} (N-j) rho_j */
  double B = 0.0;
  for (int j = 1; j < N; ++j) B += (double)(N - j) * rho[j];
  double A = 0.0;
  phi[0] = 0.0;
  for (int i = 1; i < N; ++i) {
    A += (double)i * rho[i];
    B -= (double)(N - i) * rho[i];
    const double psi = dx * k * (((double)(N - i) / N) * A + ((double)i / N) * B);
    phi[i] = V * (double)i / (double)N + psi;
  }
  phi[N] = V;
}

static void locate(const or_sim* s, double x, int* ci, double* f) {
  double g = x / s->dx;
  int i = (int)floor(g);
  double ff = g - i;
  if (i >= s->p.cells) { i = s->p.cells - 1; ff = 1.0; }
  if (i < 0) { i = 0; ff = 0.0; }
  *ci = i;
  *f = ff;
}

static void deposit_and_solve(or_sim* s) {
  int N = s->p.cells;
  memset(s->Q, 0, sizeof(double) * (N + 1));
  double we = 0.0, wi = 0.0;
  for (int sp = 0; sp < 2; ++sp) {
    const mlist* l = sp == 0 ? &s->e : &s->i;
    double q = sp == 0 ? -QE : QE;
    for (int64_t k = 0; k < l->n; ++k) {
      const marker* m = &l->a[k];
      double v = sqrt(m->vx * m->vx + m->vy * m->vy + m->vz * m->vz);
      double wp = or_beta(v, s->v0) * s->w_j * m->w; /* density weight */
      int ci;
      double f;
      locate(s, m->x, &ci, &f);
      s->Q[ci] += q * wp * (1.0 - f);
      s->Q[ci + 1] += q * wp * f;
      if (sp == 0) we += wp;
      else wi += wp;
    }
  }
  double vol = s->p.area * s->dx;
  for (int i = 0; i <= N; ++i) s->rho[i] = s->Q[i] / vol;
  s->rho[0] *= 2.0; /* half-cell volumes at the electrodes */
  s->rho[N] *= 2.0;
  or_poisson(N, s->dx, s->p.V, s->rho, s->phi, s->E);
  s->stats[OR_ST_WE] = we;
  s->stats[OR_ST_WI] = wi;
}

static double gather(const or_sim* s, double x) {
  int ci;
  double f;
  locate(s, x, &ci, &f);
  return (1.0 - f) * s->E[ci] + f * s->E[ci + 1];
}

/* ------------------------------------------------------------------ */
/* Null-collision bound for electrons: nu'(eps) = n_g sigma_T(eps) min(v, v0)
 * (Eq. 16 with beta_n = 1).  Linear interpolation keeps sigma_T on a segment
 * below the larger node value and min(v, v0) grows with energy, so each
 * segment is bounded by max(node values) * min(v(right node), v0).  Above the
 * table the cross section is constant up to the cap energy. */
static double null_bound_e(const or_sim* s) {
  int n = s->p.n_grid, nc = s->p.n_chan;
  double best = 0.0;
  for (int j = 0; j + 1 < n; ++j) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nc; ++k) {
      a += s->sigma[(size_t)k * n + j];
      b += s->sigma[(size_t)k * n + j + 1];
    }
    double v = sqrt(2.0 * QE * s->energies[j + 1] / ME);
    double term = fmax(a, b) * fmin(v, s->v0);
    if (term > best) best = term;
  }
  double tail = 0.0;
  for (int k = 0; k < nc; ++k) tail += s->sigma[(size_t)k * n + n - 1];
  double vcap = sqrt(2.0 * QE * s->ecap_eV / ME);
  if (tail * fmin(vcap, s->v0) > best) best = tail * fmin(vcap, s->v0);
  return s->n_g * best;
}

/* ------------------------------------------------------------------ */
or_sim* or_create(const or_params* p) {
  if (!(p->d > 0) || p->cells < 2 || !(p->p_torr >= 0) || !(p->cfl > 0) ||
      !(p->area > 0) || !(p->w_j0 > 0) || !(p->gamma_se >= 0 && p->gamma_se <= 1) ||
      p->n_chan < 0 || p->n_chan > 8 || p->n_grid < 2 || !(p->T_gas > 0))
    return NULL;
  or_sim* s = (or_sim*)calloc(1, sizeof(or_sim));
  if (!s) return NULL;
  s->p = *p;
  int n = p->n_grid, nc = p->n_chan;
  s->energies = (double*)malloc(sizeof(double) * n);
  s->sigma = (double*)malloc(sizeof(double) * (size_t)n * (nc > 0 ? nc : 1));
  s->thr = (double*)malloc(sizeof(double) * (nc > 0 ? nc : 1));
  s->kind = (int32_t*)malloc(sizeof(int32_t) * (nc > 0 ? nc : 1));
  memcpy(s->energies, p->energies, sizeof(double) * n);
  if (nc) {
    memcpy(s->sigma, p->sigma, sizeof(double) * (size_t)n * nc);
    memcpy(s->thr, p->threshold_eV, sizeof(double) * nc);
    memcpy(s->kind, p->kind, sizeof(int32_t) * nc);
  }
  if (p->fixed_prob) {
    s->fixed = (double*)malloc(sizeof(double) * (nc > 0 ? nc : 1));
    if (nc) memcpy(s->fixed, p->fixed_prob, sizeof(double) * nc);
  }
  s->p.energies = s->energies;
  s->p.sigma = s->sigma;
  s->p.threshold_eV = s->thr;
  s->p.kind = s->kind;
  s->p.fixed_prob = s->fixed;

  int N = p->cells;
  s->dx = p->d / N;
  if (p->v_limit == INFINITY) s->v0 = INFINITY;
  else if (p->v_limit > 0) s->v0 = p->v_limit;
  else s->v0 = sqrt(2.0 * QE * fabs(p->V) / MAR); /* Sec. IV speed limit */
  if (!(s->v0 > 0)) { or_destroy(s); return NULL; }
  if (p->dt > 0) s->dt = p->dt;
  else if (s->v0 < INFINITY) s->dt = p->cfl * s->dx / s->v0;
  else s->dt = p->cfl * s->dx / sqrt(2.0 * QE * fabs(p->V) / ME);
  if (!(s->dt > 0 && s->dt < INFINITY)) { or_destroy(s); return NULL; }
  s->n_g = p->p_torr * TORR / (KB * p->T_gas);
  s->ecap_eV = fmax(s->energies[n - 1], 2.0 * fabs(p->V) + 100.0);
  s->nu_max_e = null_bound_e(s);
  double vcap_i = sqrt(2.0 * QE * s->ecap_eV / MAR);
  s->nu_max_cx = s->n_g * p->sigma_cx * fmin(s->v0, vcap_i);
  s->P_null_e = -expm1(-s->nu_max_e * s->dt);
  s->P_null_cx = -expm1(-s->nu_max_cx * s->dt);
  s->w_j = p->w_j0;
  s->min_margin = INFINITY;
  s->Q = (double*)calloc(N + 1, sizeof(double));
  s->rho = (double*)calloc(N + 1, sizeof(double));
  s->phi = (double*)calloc(N + 1, sizeof(double));
  s->E = (double*)calloc(N + 1, sizeof(double));
  for (int sp = 0; sp < 2; ++sp) {
    s->cross[sp] = (double*)calloc(N + 1, sizeof(double));
    s->flux[sp] = (double*)calloc(N + 1, sizeof(double));
  }

  /* seeding (Sec. IV injects electrons at rest on the cathode) */
  for (int64_t k = 0; k < p->n_seed && p->seed_mode != OR_SEED_NONE; ++k) {
    marker m = {0};
    m.id = (uint64_t)k;
    m.tie = INFINITY;
    m.w = 1.0;
    if (p->seed_mode == OR_SEED_MAXWELL_CELL0) {
      uint32_t r[4];
      double v[3];
      draw_raw(s, m.id, 0, OR_CH_SEED, 0, r);
      m.x = unif(r[0]) * s->dx;
      draw_raw(s, m.id, 0, OR_CH_SEED, 1, r);
      maxwellian(r, sqrt(QE * p->kTe_seed_eV / ME), v);
      m.vx = v[0]; m.vy = v[1]; m.vz = v[2];
    }
    if (push_back(&s->e, &m)) { or_destroy(s); return NULL; }
  }
  deposit_and_solve(s);
  return s;
}

void or_destroy(or_sim* s) {
  if (!s) return;
  free(s->energies); free(s->sigma); free(s->thr); free(s->kind); free(s->fixed);
  free(s->e.a); free(s->i.a);
  free(s->Q); free(s->rho); free(s->phi); free(s->E);
  for (int sp = 0; sp < 2; ++sp) { free(s->cross[sp]); free(s->flux[sp]); }
  free(s);
}

int or_load(or_sim* s, int species, int64_t n, const int32_t* cell, const double* off,
            const double* vx, const double* vy, const double* vz, const uint64_t* id) {
  mlist* l = species == OR_ELECTRON ? &s->e : &s->i;
  l->n = 0;
  for (int64_t k = 0; k < n; ++k) {
    marker m;
    m.x = ((double)cell[k] + off[k]) * s->dx;
    m.vx = vx[k]; m.vy = vy[k]; m.vz = vz[k];
    m.id = id[k];
    m.tie = INFINITY;
    m.w = 1.0;
    if (push_back(l, &m)) return -1;
  }
  deposit_and_solve(s);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Collision strategy (Sec. III).  The paper notes that Monte Carlo
 * strategies which give the same expected number of collisions W_c are
 * interchangeable: split every colliding primary (w_j,p0 = w_j,p1 + W_j,c,
 * the collided part W_j,c carrying the products), or collide a fraction of
 * the pairs with the primary's whole weight.  Both are written here through
 * one split fraction s:
 *   - a marker becomes a collision candidate with probability
 *     q = min(1, P/s), P the per-step candidate probability (the
 *     null-collision probability, or the fixed-event total);
 *   - a candidate that collides moves the fraction f = max(s, P) of its flux
 *     weight into the collision: q f = P, so the expected collided weight is
 *     that of every candidate colliding whole with probability P;
 *   - s = 1 (or s <= 0) is the whole-marker strategy (q = P, f = 1); with
 *     f < 1 the primary keeps w (1 - f) and its velocity and id as the
 *     uncollided part, and a new marker of weight w f (id from channel
 *     CHILD, sub 2) leaves with the scattered velocity; ionization products
 *     carry w f.
 * Flux weights are conserved in every event (Sec. III). */
static double split_frac(const or_sim* s) {
  const double sf = s->p.split_frac;
  return (sf > 0.0 && sf < 1.0) ? sf : 1.0;
}

/* the uncollided part stays as m (weight w (1 - f)); the scattered part is
 * returned in *sc with the new velocity and weight w f and a new id */
static void split_off(or_sim* s, marker* m, double f, const double v_new[3], marker* sc) {
  uint32_t r[4];
  draw_raw(s, m->id, s->step, OR_CH_CHILD, 2, r);
  *sc = *m;
  sc->vx = v_new[0];
  sc->vy = v_new[1];
  sc->vz = v_new[2];
  sc->id = child_id(r[0], r[1]);
  sc->w = m->w * f;
  m->w = m->w * (1.0 - f);
}

/* Electron-neutral collision (Sec. III and Sec. IV).  The marker's channel is
 * drawn with per-step probability P_null nu'_k / nu'_max, the finite-step
 * form of Eq. (16), split as above. */
static int collide_electron(or_sim* s, marker* m, mlist* born_e, mlist* born_i) {
  uint32_t step = s->step;
  uint32_t r[4];
  draw_raw(s, m->id, step, OR_CH_COLL, 0, r);
  double u0 = unif(r[0]), u1 = unif(r[1]);
  double v[3] = {m->vx, m->vy, m->vz};
  double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  double speed = sqrt(v2);
  double eps = 0.5 * ME * v2 / QE;
  int nc = s->p.n_chan, ch = -1;
  const double sf = split_frac(s);
  double f = 1.0;
  if (s->fixed) {
    double tot = 0.0;
    for (int k = 0; k < nc; ++k) tot += s->fixed[k];
    if (sf >= 1.0) {
      double cum = 0.0;
      for (int k = 0; k < nc; ++k) {
        cum += s->fixed[k];
        if (ch < 0 && u0 < cum) ch = k;
      }
    } else {
      if (!(u0 < fmin(1.0, tot / sf))) return 0;
      f = fmax(sf, tot);
      /* channel k of a candidate with probability fixed_k / tot */
      double cum = 0.0;
      for (int k = 0; k < nc; ++k) {
        cum += s->fixed[k];
        if (ch < 0 && u1 < cum / tot) ch = k;
      }
    }
  } else {
    if (!(u0 < (sf >= 1.0 ? s->P_null_e : fmin(1.0, s->P_null_e / sf)))) return 0;
    if (sf < 1.0) f = fmax(sf, s->P_null_e);
    double slow = fmin(speed, s->v0);
    double target = u1 * s->nu_max_e, cum = 0.0, margin = INFINITY;
    for (int k = 0; k < nc; ++k) {
      cum += s->n_g * or_sigma(s, k, eps) * slow;
      double mk = fabs(target - cum) / s->nu_max_e;
      if (mk < margin) margin = mk;
      if (ch < 0 && target < cum) ch = k;
    }
    note_margin(s, m, margin);
    if (cum > s->nu_max_e * (1.0 + 1e-12)) s->err |= OR_ERR_NU_BOUND;
  }
  if (ch < 0) return 0;
  int kind = s->kind[ch];
  double thr = s->thr[ch], vout[3], mrot;
  const double w_coll = m->w * (f < 1.0 ? f : 1.0);  /* weight of the collided part */
  if (kind == OR_ELASTIC) {
    double cosx = or_vs_cos_chi(eps, unif(r[2]));
    double eps1 = eps * (1.0 - 2.0 * ME / MAR * (1.0 - cosx));
    mrot = scatter_to(v, eps1, cosx, TWO_PI * unif(r[3]), vout);
    s->stats[OR_ST_ELASTIC] += 1;
  } else if (kind == OR_EXCITATION) {
    double eps1 = fmax(eps - thr, 0.0);
    mrot = scatter_to(v, eps1, 1.0 - 2.0 * unif(r[2]), TWO_PI * unif(r[3]), vout);
    s->stats[OR_ST_EXCIT] += 1;
  } else {
    /* ionization: the primary and the ejected electron share eps - I;
     * a new Ar+ appears at the primary's position with a thermal velocity */
    uint32_t q[4], b[4], c[4];
    draw_raw(s, m->id, step, OR_CH_IONIZ, 0, q);
    draw_raw(s, m->id, step, OR_CH_IONBIRTH, 0, b);
    draw_raw(s, m->id, step, OR_CH_CHILD, 0, c);
    double eps_av = fmax(eps - thr, 0.0);
    double eps_ej = or_ejected_energy(eps_av, s->p.ion_B_eV, unif(q[0]));
    double eps_sc = eps_av - eps_ej;
    if (s->p.flags & OR_FLAG_PRODUCTS_AT_REST) eps_ej = eps_sc = 0.0;
    double vej[3], vi[3];
    mrot = scatter_to(v, eps_sc, or_vs_cos_chi(eps_sc, unif(r[2])), TWO_PI * unif(r[3]),
                      vout);
    double m2 = scatter_to(v, eps_ej, or_vs_cos_chi(eps_ej, unif(q[1])),
                           TWO_PI * unif(q[2]), vej);
    if (m2 < mrot) mrot = m2;
    maxwellian(b, sqrt(KB * s->p.T_gas / MAR), vi);
    marker ne = {m->x, vej[0], vej[1], vej[2], m->tie, child_id(c[0], c[1]), w_coll};
    marker ni = {m->x, vi[0], vi[1], vi[2], m->tie, child_id(c[2], c[3]), w_coll};
    note_margin(s, &ne, mrot);
    note_margin(s, &ni, mrot);
    if (push_back(born_e, &ne) || push_back(born_i, &ni)) return -1;
    s->stats[OR_ST_IONIZ] += 1;
  }
  if (f < 1.0) {
    marker sc;
    split_off(s, m, f, vout, &sc);
    note_margin(s, &sc, mrot);
    return push_back(born_e, &sc);
  }
  note_margin(s, m, mrot);
  m->vx = vout[0];
  m->vy = vout[1];
  m->vz = vout[2];
  return 0;
}

/* Ar+ charge exchange: the ion leaves with a neutral's thermal velocity
 * (split as above). */
static int collide_ion(or_sim* s, marker* m, mlist* born_i) {
  uint32_t r[4];
  draw_raw(s, m->id, s->step, OR_CH_CX, 0, r);
  double u0 = unif(r[0]), u1 = unif(r[1]);
  const double sf = split_frac(s);
  double f = 1.0;
  int hit;
  if (s->fixed) {
    const double P = s->p.fixed_prob_cx;
    if (sf >= 1.0) {
      hit = u0 < P;
    } else {
      hit = u0 < fmin(1.0, P / sf);
      f = fmax(sf, P);
    }
  } else {
    if (!(s->p.sigma_cx > 0)) return 0;
    if (!(u0 < (sf >= 1.0 ? s->P_null_cx : fmin(1.0, s->P_null_cx / sf)))) return 0;
    if (sf < 1.0) f = fmax(sf, s->P_null_cx);
    double speed = sqrt(m->vx * m->vx + m->vy * m->vy + m->vz * m->vz);
    double nu = s->n_g * s->p.sigma_cx * fmin(speed, s->v0);
    if (nu > s->nu_max_cx * (1.0 + 1e-12)) s->err |= OR_ERR_NU_BOUND;
    double target = u1 * s->nu_max_cx;
    note_margin(s, m, fabs(target - nu) / s->nu_max_cx);
    hit = target < nu;
  }
  if (!hit) return 0;
  uint32_t b[4];
  double vi[3];
  draw_raw(s, m->id, s->step, OR_CH_CX, 1, b);
  maxwellian(b, sqrt(KB * s->p.T_gas / MAR), vi);
  s->stats[OR_ST_CX] += 1;
  if (f < 1.0) {
    marker sc;
    split_off(s, m, f, vi, &sc);
    return push_back(born_i, &sc);
  }
  m->vx = vi[0]; m->vy = vi[1]; m->vz = vi[2];
  return 0;
}

/* Push one marker; returns 0 inside, 1 absorbed at the cathode, 2 at the anode.
 * The wall test uses the whole flight: the lowest and highest x reached. */
static int push(or_sim* s, marker* m, double qm) {
  double a = qm * gather(s, m->x);
  double vperp = sqrt(m->vy * m->vy + m->vz * m->vz);
  double ddx, vx1;
  double tau = or_free_flight(m->vx, vperp, a, s->dt, s->v0, &ddx, &vx1);
  double x0 = m->x, x1 = x0 + ddx;
  double xlo = fmin(x0, x1), xhi = fmax(x0, x1);
  /* the start point was inside already; the margin looks at the new points */
  double nlo = x1, nhi = x1;
  if (m->vx * a < 0.0 && -m->vx / a < tau) { /* turning point inside the flight */
    double xt = x0 - m->vx * m->vx / (2.0 * a);
    xlo = fmin(xlo, xt);
    xhi = fmax(xhi, xt);
    nlo = fmin(nlo, xt);
    nhi = fmax(nhi, xt);
  }
  m->x = x1;
  m->vx = vx1;
  double margin = fmin(fabs(nlo), fabs(s->p.d - nhi)) / s->dx;
  note_margin(s, m, margin);
  if (!isfinite(x1) || !isfinite(vx1)) s->err |= OR_ERR_NONFINITE;
  if (xlo < 0.0) return 1;
  if (xhi >= s->p.d) return 2;
  return 0;
}

/* Flux through surfaces (Eq. (12) and the passage after it): a marker that
 * crosses a surface carries w_j physical particles through it, whatever its
 * speed.  Net crossings of the nodes between the cells before and after the
 * flight; absorbed markers end in cell -1 (cathode, w == 1) or cells (anode,
 * w == 2). */
static void note_crossings(or_sim* s, int sp, double x0, double x1, int w, double wt) {
  if (!(s->p.flags & OR_FLAG_FLUX)) return;
  if (w == 0 && !isfinite(x1)) return;  /* a non-finite state is an error, not a crossing */
  const int64_t N = s->p.cells;
  int64_t c0 = (int64_t)floor(x0 / s->dx);
  c0 = c0 < 0 ? 0 : (c0 > N - 1 ? N - 1 : c0);
  int64_t c1;
  if (w == 1) c1 = -1;
  else if (w == 2) c1 = N;
  else {
    c1 = (int64_t)floor(x1 / s->dx);
    c1 = c1 < 0 ? 0 : (c1 > N - 1 ? N - 1 : c1);
  }
  for (int64_t k = c0 + 1; k <= c1; ++k) s->cross[sp][k] += wt;
  for (int64_t k = c1 + 1; k <= c0; ++k) s->cross[sp][k] -= wt;
}

static int one_step(or_sim* s) {
  memset(s->stats, 0, sizeof(s->stats));
  uint32_t step = s->step;
  const double w_step = s->w_j;  /* the flux weight of the markers this step */
  int64_t nin = s->e.n + s->i.n;
  /* population control decided from the integer counts entering the step */
  int mode = 0;
  if (s->p.n_target > 0) {
    if (nin > 2 * s->p.n_target) mode = 1;                 /* roulette */
    else if (nin > 0 && 2 * nin < s->p.n_target) mode = 2; /* split */
  }
  mlist born_e = {0}, born_i = {0}, out_e = {0}, out_i = {0};
  int rc = 0;
  for (int64_t k = 0; k < s->e.n && !rc; ++k) {
    marker m = s->e.a[k];
    const double xe0 = m.x;
    int w = push(s, &m, -QE / ME);
    note_crossings(s, OR_ELECTRON, xe0, m.x, w, m.w);
    if (w == 1) { s->stats[OR_ST_ABS_E_CATH] += 1; continue; }
    if (w == 2) { s->stats[OR_ST_ABS_E_ANODE] += 1; continue; }
    rc = collide_electron(s, &m, &born_e, &born_i);
    if (!rc) rc = push_back(&out_e, &m);
  }
  for (int64_t k = 0; k < s->i.n && !rc; ++k) {
    marker m = s->i.a[k];
    const double x0 = m.x, vx0 = m.vx, a0 = QE / MAR * gather(s, m.x);
    int w = push(s, &m, QE / MAR);
    note_crossings(s, OR_ION, x0, m.x, w, m.w);
    if (w == 1) {
      /* ion-induced secondary emission at the cathode (Sec. IV): an electron
       * at rest at x = 0 with probability gamma_se, or with the yield of
       * Eq. (17) at the impact energy.  v_x^2 - 2 a x is constant along the
       * flight (in proper time the orbit is the PIC parabola), so the ion
       * reaches x = 0 with v_x^2 = vx0^2 - 2 a x0. */
      s->stats[OR_ST_ABS_I_CATH] += 1;
      uint32_t r[4];
      draw_raw(s, m.id, step, OR_CH_SEE, 0, r);
      double gam = s->p.gamma_se;
      if (s->p.flags & OR_FLAG_SEE_ENERGY) {
        const double vx2 = fmax(vx0 * vx0 - 2.0 * a0 * x0, 0.0);
        gam = or_see_yield(0.5 * MAR * (vx2 + m.vy * m.vy + m.vz * m.vz) / QE);
        note_margin(s, &m, fabs(unif(r[0]) - gam));
      }
      if (unif(r[0]) < gam) {
        marker ne = {0.0, 0.0, 0.0, 0.0, m.tie, child_id(r[2], r[3]), m.w};
        rc = push_back(&born_e, &ne);
        s->stats[OR_ST_SEE] += 1;
      }
      continue;
    }
    if (w == 2) { s->stats[OR_ST_ABS_I_ANODE] += 1; continue; }
    rc = collide_ion(s, &m, &born_i);
    if (!rc) rc = push_back(&out_i, &m);
  }
  /* continuous cathode source (or_set_source): electrons at rest at x = 0,
   * as many as keep the physical rate at the step's flux weight */
  if (s->src > 0 && !rc) {
    const double want = s->src * (s->p.w_j0 / w_step);
    int64_t n = (int64_t)floor(want);
    uint32_t r[4];
    draw_raw(s, 0, step, OR_CH_INJECT, 1, r);
    if (unif(r[0]) < want - floor(want)) n += 1;
    for (int64_t k = 0; k < n && !rc; ++k) {
      draw_raw(s, (uint64_t)k, step, OR_CH_INJECT, 0, r);
      marker ne = {0.0, 0.0, 0.0, 0.0, INFINITY, child_id(r[0], r[1]), 1.0};
      rc = push_back(&born_e, &ne);
    }
  }
  for (int64_t k = 0; k < born_e.n && !rc; ++k) rc = push_back(&out_e, &born_e.a[k]);
  for (int64_t k = 0; k < born_i.n && !rc; ++k) rc = push_back(&out_i, &born_i.a[k]);
  free(born_e.a);
  free(born_i.a);
  /* population control on the step's output */
  if (mode && !rc) {
    for (int sp = 0; sp < 2 && !rc; ++sp) {
      mlist* src = sp == 0 ? &out_e : &out_i;
      mlist dst = {0};
      for (int64_t k = 0; k < src->n && !rc; ++k) {
        marker m = src->a[k];
        uint32_t r[4];
        if (mode == 1) {
          draw_raw(s, m.id, step, OR_CH_ROULETTE, 0, r);
          if (unif(r[0]) < 0.5) rc = push_back(&dst, &m);
          else s->stats[OR_ST_ROULETTE] += 1;
        } else {
          draw_raw(s, m.id, step, OR_CH_CHILD, 1, r);
          marker c = m;
          c.id = child_id(r[0], r[1]);
          rc = push_back(&dst, &m);
          if (!rc) rc = push_back(&dst, &c);
          s->stats[OR_ST_SPLIT] += 1;
        }
      }
      free(src->a);
      *src = dst;
    }
    s->w_j *= (mode == 1) ? 2.0 : 0.5;
  }
  free(s->e.a);
  free(s->i.a);
  s->e = out_e;
  s->i = out_i;
  if (rc) { s->err |= OR_ERR_ALLOC; return -1; }
  if (s->p.flags & OR_FLAG_FLUX)
    for (int sp = 0; sp < 2; ++sp)
      for (int k = 0; k <= s->p.cells; ++k) {
        s->flux[sp][k] += w_step * s->cross[sp][k];
        s->cross[sp][k] = 0;
      }
  deposit_and_solve(s);
  s->step = step + 1;
  s->stats[OR_ST_STEP] = s->step;
  s->stats[OR_ST_NE] = (double)s->e.n;
  s->stats[OR_ST_NI] = (double)s->i.n;
  s->stats[OR_ST_WJ] = s->w_j;
  s->stats[OR_ST_NIN] = (double)nin;
  s->stats[OR_ST_ERR] = s->err;
  return 0;
}

int or_step(or_sim* s, int n_steps) {
  for (int k = 0; k < n_steps; ++k)
    if (one_step(s)) return -1;
  return s->err ? -2 : 0;
}

int64_t or_count(const or_sim* s, int species) {
  return species == OR_ELECTRON ? s->e.n : s->i.n;
}

int or_read(const or_sim* s, int species, int32_t* cell, double* off, double* vx,
            double* vy, double* vz, uint64_t* id, double* tie) {
  const mlist* l = species == OR_ELECTRON ? &s->e : &s->i;
  for (int64_t k = 0; k < l->n; ++k) {
    const marker* m = &l->a[k];
    double g = m->x / s->dx;
    int ci = (int)floor(g);
    if (cell) cell[k] = ci;
    if (off) off[k] = g - ci;
    if (vx) vx[k] = m->vx;
    if (vy) vy[k] = m->vy;
    if (vz) vz[k] = m->vz;
    if (id) id[k] = m->id;
    if (tie) tie[k] = m->tie;
  }
  return 0;
}

int or_read_weights(const or_sim* s, int species, double* w) {
  const mlist* l = species == OR_ELECTRON ? &s->e : &s->i;
  for (int64_t k = 0; k < l->n; ++k) w[k] = l->a[k].w;
  return 0;
}

void or_fields(const or_sim* s, double* rho, double* phi, double* E) {
  size_t n = (size_t)s->p.cells + 1;
  if (rho) memcpy(rho, s->rho, n * sizeof(double));
  if (phi) memcpy(phi, s->phi, n * sizeof(double));
  if (E) memcpy(E, s->E, n * sizeof(double));
}

void or_flux(const or_sim* s, int species, double* out) {
  memcpy(out, s->flux[species == OR_ELECTRON ? 0 : 1], ((size_t)s->p.cells + 1) * sizeof(double));
}

int or_set_source(or_sim* s, double per_step) {
  if (!(per_step >= 0.0 && per_step <= 16777216.0)) return -1;
  s->src = per_step;
  return 0;
}

int or_set_clock(or_sim* s, uint32_t step, double w_j) {
  if (!(w_j > 0.0 && w_j < INFINITY)) return -1;
  s->step = step;
  s->w_j = w_j;
  deposit_and_solve(s);
  return 0;
}

void or_flux_reset(or_sim* s) {
  for (int sp = 0; sp < 2; ++sp)
    memset(s->flux[sp], 0, ((size_t)s->p.cells + 1) * sizeof(double));
}

void or_last_stats(const or_sim* s, double* row) {
  memcpy(row, s->stats, sizeof(s->stats));
}

void or_scalars(const or_sim* s, double* out) {
  out[0] = s->dx; out[1] = s->dt; out[2] = s->v0; out[3] = s->n_g;
  out[4] = s->nu_max_e; out[5] = s->nu_max_cx; out[6] = s->w_j; out[7] = s->step;
}

double or_min_margin(const or_sim* s) { return s->min_margin; }
