// HIP kernels (gfx950) of the speed-limited PIC / Monte Carlo collision step.
//
// A step is two launches.  k_gen<R, MODE_STEP> advances every marker of
// every instance: gather, speed-limited free flight (Eqs. 8-9 with beta of
// Eq. 11, solved exactly for the gathered field), wall absorption and
// ion-induced secondary emission, null-collision MCC with the SLPIC rate of
// Eqs. (15)-(16), population control, stream compaction of survivors and new
// markers, and the linear charge deposit in fixed point.  k_tail, one
// workgroup per instance, then turns the deposit into the charge density,
// solves the instance's Poisson problem in FP64, writes its statistics row,
// decides the next step's population control, injects the cathode source,
// picks the deposit windows of the next steps (every ANCHOR_PERIOD steps)
// and advances the generation.
//
// Memory layout: markers (int32 cell, R offset in the cell, R v_x, v_y, v_z,
// uint64 id) in chunks of 64 slots, each field contiguous within a chunk, in
// two ping-pong buffers per species; each instance owns a segment of output
// partitions.  Work unit: a tile of 256 markers of one (instance, species),
// one marker per lane of four waves; each workgroup takes a contiguous run
// of tiles.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "slpic_internal.hpp"

namespace slpic {

// ---------------------------------------------------------------- math
__device__ __forceinline__ float m_atan(float x) { return atanf(x); }
__device__ __forceinline__ double m_atan(double x) { return atan(x); }
__device__ __forceinline__ float m_tan(float x) { return tanf(x); }
__device__ __forceinline__ double m_tan(double x) { return tan(x); }
__device__ __forceinline__ float m_floor(float x) { return floorf(x); }
__device__ __forceinline__ double m_floor(double x) { return floor(x); }
__device__ __forceinline__ bool m_finite(float x) { return isfinite(x); }
__device__ __forceinline__ bool m_finite(double x) { return isfinite(x); }
template <typename R> __device__ __forceinline__ R one_below();
template <> __device__ __forceinline__ float one_below<float>() { return 0x1.fffffep-1f; }
template <> __device__ __forceinline__ double one_below<double>() { return 0x1.fffffffffffffp-1; }

// physical constants (SI)
constexpr double QE = 1.602176634e-19;
constexpr double ME = 9.1093837015e-31;
constexpr double MAR = 39.948 * 1.66053906660e-27;

// Arithmetic of the particle kernels.  The FP64 instantiation uses the
// correctly rounded library functions and true division.  The FP32 one uses
// the hardware square root, reciprocal, base-2 logarithm and exponential and
// sine/cosine (about one ulp each; sine and cosine take revolutions), with
// short Taylor series where a hardware form would lose relative accuracy
// (log1p and expm1 of small arguments, asinh near 0).  That keeps every
// FP32 quantity within a few 1e-7 relative of its exact value, far inside
// the FP32 budget of 1e-5.
template <typename R> struct Fm;
template <> struct Fm<double> {
  static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double div(double x, double y) { return x / y; }
  static __device__ __forceinline__ double asinh(double x) { return ::asinh(x); }
  static __device__ __forceinline__ double log(double x) { return ::log(x); }
  static __device__ __forceinline__ double log1p(double x) { return ::log1p(x); }
  static __device__ __forceinline__ double expm1(double x) { return ::expm1(x); }
  static __device__ __forceinline__ double pow(double x, double y) { return ::pow(x, y); }
  // sin and cos of 2 pi u
  static __device__ __forceinline__ void sincos2pi(double u, double* s, double* c) {
    ::sincospi(2.0 * u, s, c);
  }
};
template <> struct Fm<float> {
  static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float div(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }
  static __device__ __forceinline__ float log(float x) { return __builtin_amdgcn_logf(x) * 0.69314718f; }
  // asinh for x >= 0: series below 1/16, else ln 2 * log2(x + sqrt(x^2 + 1))
  static __device__ __forceinline__ float asinh(float x) {
    if (x < 0.0625f) {
      const float x2 = x * x;
      return x * (1.0f - x2 * (0.16666667f - x2 * 0.075f));
    }
    return 0.69314718f * __builtin_amdgcn_logf(x + __builtin_amdgcn_sqrtf(x * x + 1.0f));
  }
  // log(1 + x) for x >= 0: series below 2^-5 (truncation below 1e-8
  // relative), else the logarithm of the rounded 1 + x (2e-6 at most)
  static __device__ __forceinline__ float log1p(float x) {
    if (x < 0.03125f)
      return x * (1.0f - x * (0.5f - x * (0.33333334f - x * (0.25f - x * 0.2f))));
    return log(1.0f + x);
  }
  // exp(y) - 1: series for |y| below 2^-5, else exp(y) - 1 (the result is
  // then at least 0.03 in magnitude: 2e-6 relative at most)
  static __device__ __forceinline__ float expm1(float y) {
    if (__builtin_fabsf(y) < 0.03125f)
      return y * (1.0f + y * 0.5f * (1.0f + y * 0.33333334f * (1.0f + y * 0.25f * (1.0f + y * 0.2f))));
    return __builtin_amdgcn_exp2f(y * 1.44269504f) - 1.0f;
  }
  // x^y = 2^(y log2 x) for x > 0 (relative error ~1e-7 for |y log2 x| < 10)
  static __device__ __forceinline__ float pow(float x, float y) {
    return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
  }
  static __device__ __forceinline__ void sincos2pi(float u, float* s, float* c) {
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
  }
};

// Per-instance parameters do not change while a kernel runs: reading them
// through the constant address space lets the compiler use scalar loads
// (held in scalar registers, reloaded cheaply) instead of vector loads.
using IP = const __attribute__((address_space(4))) InstParams;
__device__ __forceinline__ IP& param(const InstParams* ip, int i) { return ((IP*)ip)[i]; }

// A per-instance constant in kernel precision: the FP64 field, or its FP32
// copy rounded on the host.
template <typename R> __device__ __forceinline__ R pr(double d, float f);
template <> __device__ __forceinline__ double pr<double>(double d, float) { return d; }
template <> __device__ __forceinline__ float pr<float>(double, float f) { return f; }
#define PR(P, name) pr<R>((P).name, (P).name##_f)

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplies on words 0 and 2, with the Weyl-sequence key schedule.
struct U4 {
  uint32_t x, y, z, w;
};

// a ^ b ^ c in one instruction: gfx950's three-input bitwise operation
// with the truth table of XOR (0x96 for the operand bytes 0xf0, 0xcc, 0xaa)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    c0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    c2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// stream of one marker: key (seed, instance), counter (id, step, channel)
__device__ __forceinline__ U4 draw(uint64_t id, uint32_t step, uint32_t ch, uint32_t seed,
                                   uint32_t inst) {
  return philox((uint32_t)id, (uint32_t)(id >> 32), step, ch, seed, inst);
}

// the same stream out of line, for draws on rare paths (population
// control, emission, ionization products, charge exchange): keeps one copy
// of the ten rounds in the code instead of one per call site
__device__ __noinline__ U4 draw_cold(uint64_t id, uint32_t step, uint32_t ch, uint32_t seed,
                                     uint32_t inst) {
  return draw(id, step, ch, seed, inst);
}

// u = (2 (r >> 9) + 1) 2^-24: exact in FP32 and FP64, never 0 or 1
template <typename R>
__device__ __forceinline__ R unif(uint32_t r) {
  return (R)(((r >> 9) << 1) | 1u) * (R)5.9604644775390625e-08;
}

__device__ __forceinline__ uint64_t child(uint32_t lo, uint32_t hi) {
  return ((uint64_t)hi << 32 | lo) | 0x8000000000000000ull;
}

// three normals (Box-Muller on two pairs) scaled by sigma
template <typename R>
__device__ __forceinline__ void normals3(U4 r, R sigma, R& a, R& b, R& c) {
  R s0, c0, s1, c1;
  const R r0 = Fm<R>::sqrt(R(-2) * Fm<R>::log(unif<R>(r.x)));
  const R r1 = Fm<R>::sqrt(R(-2) * Fm<R>::log(unif<R>(r.z)));
  Fm<R>::sincos2pi(unif<R>(r.y), &s0, &c0);
  Fm<R>::sincos2pi(unif<R>(r.w), &s1, &c1);
  a = sigma * r0 * c0;
  b = sigma * r0 * s0;
  c = sigma * r1 * c1;
}

// ---------------------------------------------------------------- flight
// Integral of sqrt(u^2 + c^2) over [p, p + len], p >= 0, in a form without
// cancellation for short intervals (q = p + len, W(u) = sqrt(u^2 + c^2)):
//   q W(q) - p W(p) = len (q + p)(q^2 + p^2 + c^2) / (q W(q) + p W(p)),
//   asinh(q/c) - asinh(p/c) = asinh(len (q + p) / (q W(p) + p W(q))).
// Wp = W(p) and Wq = W(q) come from the caller: the span ends are the
// flight's ends, 0 or the speed-limit point, whose W are known there.
template <typename R>
__device__ __forceinline__ R sqrt_span(R p, R len, R c, R Wp, R Wq) {
  const R q = p + len, sq = p + q;
  const R c2 = c * c;
  const R den1 = q * Wq + p * Wp, den2 = q * Wp + p * Wq;
  const bool empty = !(len > R(0)) || !(den1 > R(0));
  const R t1 = empty ? R(0) : Fm<R>::div(len * sq * (q * q + p * p + c2), den1);
  const R t2 = (empty || c2 == R(0)) ? R(0) : c2 * Fm<R>::asinh(Fm<R>::div(len * sq, den2));
  return R(0.5) * (t1 + t2);
}

// Integral of max(1, W(u)/v0) over [p, p + len] for p >= 0, where |v| < v0
// (beta = 1) below u = ss: a linear part and one square-root part.  Wp and
// Wq are W(p) and W(p + len); W(ss) = v0.
template <typename R>
__device__ __forceinline__ R half_span(R p, R len, R c, R inv_v0, R ss, R v0, R Wp, R Wq) {
  const R q = p + len;
  const bool split = p < ss;
  const R e = q < ss ? q : ss;                 // end of the linear part
  const R lin = split ? e - p : R(0);
  const R start = split ? e : p;
  R rest = split ? q - e : len;                // keeps len exact when unsplit
  rest = rest > R(0) ? rest : R(0);            // (zero when q < ss)
  return lin + sqrt_span(start, rest, c, split ? v0 : Wp, Wq) * inv_v0;
}

// Wall-clock time (times |a|) for s to move from s0 to s0 + len: the
// integral of max(1, |v|/v0) ds, split at s = 0 by symmetry.  The second
// half span is taken only when s crosses 0 (rare; it would add +0).  w0 and
// w1 are |v| at the two ends, W(s0) and W(s0 + len); W(0) = c.
template <typename R>
__device__ __forceinline__ R time_span(R s0, R len, R c, R inv_v0, R ss, R v0, R w0, R w1) {
  const R s1 = s0 + len;
  const bool pos = s0 >= R(0), neg = !(s1 > R(0));
  const R p1 = pos ? s0 : (neg ? -s1 : R(0));
  const R l1 = (pos || neg) ? len : -s0;
  R t = half_span(p1, l1, c, inv_v0, ss, v0, pos ? w0 : (neg ? w1 : c), pos ? w1 : w0);
  if (!(pos || neg)) t += half_span(R(0), s1, c, inv_v0, ss, v0, c, w1);
  return t;
}

// Exact speed-limited flight over dt in the uniform acceleration a along x
// (inv_v0 = 1 / v0, precomputed per instance).  Returns the displacement, the
// new v_x and, when v_x changes sign inside the flight, the displacement of
// the turning point.
template <typename R>
__device__ void flight(R vx, R c2, R a, R dt, R v0, R inv_v0, int limited, R& disp, R& vx1,
                       bool& turns, R& turn_disp) {
  R dv;  // change of v_x (= a tau)
  R tau;
  // c = |v_perp| from c2 = v_y^2 + v_z^2: FP64 takes it at once (and c^2
  // as c c); FP32 only where the iteration needs it, c^2 being c2
  const R c64 = sizeof(R) == 8 ? Fm<R>::sqrt(c2) : R(0);
  const R cc = sizeof(R) == 8 ? c64 * c64 : c2;
  const R w0sq = vx * vx + cc;
  const R ve = vx + a * dt;
  if (!limited || (w0sq <= v0 * v0 && ve * ve + cc <= v0 * v0)) {
    tau = dt;  // beta == 1 along the whole flight
    dv = a * dt;
  } else if (a == R(0)) {
    tau = Fm<R>::div(dt * v0, Fm<R>::sqrt(w0sq));
    dv = R(0);
  } else {
    // reflect so that a > 0, unknown delta = s1 - s0 in (0, |a| dt]:
    //   time_span(s0, delta) = |a| dt
    const R sg = a > R(0) ? R(1) : R(-1);
    const R at = a * sg, s0 = sg * vx;
    const R rhs = at * dt;
    // |v| at the start and, in FP32, its reciprocal by one reciprocal
    // square root
    const R iw32 = sizeof(R) == 4 ? (R)__builtin_amdgcn_rsqf((float)w0sq) : R(0);
    const R w0 = sizeof(R) == 4 ? w0sq * iw32 : Fm<R>::sqrt(w0sq);
    R delta = R(0);
    bool solved = false;
    if (sizeof(R) == 4) {
      // Fully speed-limited flight (|v| > v0 all along, as for nearly every
      // limited electron): the path length in s is w0^2 F(delta / w0) with
      // F(r) = int_0^r sqrt(1 + 2 p u + u^2) du, p = s0 / w0, q = c / w0,
      // and F(r) = R = v0 |a| dt / w0^2.  The Taylor coefficients of the
      // integrand are the Gegenbauer polynomials C_n^(-1/2)(-p): g_0 = 1,
      // g_1 = p, g_2 = q^2 / 2 and n g_n = -(2n - 3) p g_(n-1) - (n - 3)
      // g_(n-2), each at most 2 / (2n - 1) in magnitude, so for r <= 0.2
      // eight terms of F leave under 1e-7 of it.  The guess is the series
      // reversion to fourth order, r = R - (p/2) R^2 + (p^2/2 - q^2/6) R^3 +
      // (13 p q^2 / 24 - 5 p^3 / 8) R^4 (within 2e-3 for R < 0.25); with
      // F' = sqrt(1 + 2 p r + r^2) and F'' = (p + r) / F' in closed form,
      // one Halley step then reaches FP32 rounding, without square roots or
      // logarithms of the spans.  A step larger than the guess's error
      // (0.4 %) sends the marker to the iteration below, as does a flight
      // that would reach |v| <= v0 (a 1 % margin on the guess covers its
      // error).  The choice is the marker's own, never its wave's: a result
      // must not depend on which markers share a wave.  A wave whose lanes
      // all qualify skips the iteration.
      const R iw = iw32;
      const R p = s0 * iw, q2 = cc * iw * iw;
      const R Rt = v0 * rhs * iw * iw;
      const R b2 = R(-0.5) * p, b3 = R(0.5) * p * p - q2 * R(1.0 / 6.0);
      const R b4 = p * (q2 * R(13.0 / 24.0) - p * p * R(5.0 / 8.0));
      const R r0 = Rt * (R(1) + Rt * (b2 + Rt * (b3 + Rt * b4)));
      const R sN = s0 + R(1.01) * r0 * w0;
      const bool ok = w0 > v0 && Rt < R(0.25) && r0 > R(0) && r0 < R(0.2) &&
                      sN * sN + cc > v0 * v0 && !(s0 < R(0) && sN > R(0) && !(cc > v0 * v0));
      if (ok) {
        constexpr int NT = 8;
        R gn[NT];
        gn[0] = R(1);
        gn[1] = p;
        gn[2] = R(0.5) * q2;
#pragma unroll
        for (int n = 3; n < NT; ++n)
          gn[n] = R(-(2.0 * n - 3.0) / n) * p * gn[n - 1] - R((n - 3.0) / n) * gn[n - 2];
        R F = gn[NT - 1] * R(1.0 / NT);
#pragma unroll
        for (int n = NT - 2; n >= 0; --n) F = F * r0 + gn[n] * R(1.0 / (n + 1));
        F *= r0;
        const R S = Fm<R>::sqrt(R(1) + r0 * (R(2) * p + r0));  // F'(r0)
        const R f = F - Rt;
        // Halley: -2 f F' / (2 F'^2 - f F''), over F'
        const R step = Fm<R>::div(R(2) * f * S * S, R(2) * S * S * S - f * (p + r0));
        if ((step < R(0) ? -step : step) <= R(4e-3) * r0) {
          delta = (r0 - step) * w0;
          solved = true;
        }
      }
    }
    if (!solved) {
      const R c = sizeof(R) == 8 ? c64 : Fm<R>::sqrt(c2);
      const R ss = c < v0 ? Fm<R>::sqrt(v0 * v0 - c * c) : R(0);
      R lo = R(0), hi = rhs;
      if (w0 > v0) {
        // speed-limited start: the path length in s, integral of W = |v|
        // over [s0, s0 + d], is w0 d + s0 d^2 / (2 w0) + c^2 d^3 / (6 w0^3)
        // + ...; solve the quadratic, then one Newton step adds the cubic
        // term
        const R disc = w0 * w0 + R(2) * s0 * v0 * Fm<R>::div(rhs, w0);
        delta = disc > R(0) ? Fm<R>::div(R(2) * v0 * rhs, w0 + Fm<R>::sqrt(disc)) : R(-1);
        const R iw = Fm<R>::div(R(1), w0);
        const R cub = c * c * iw * iw * iw * (R(1) / R(6)) * delta * delta * delta;
        delta -= Fm<R>::div(cub, w0 + s0 * iw * delta);
      } else {
        // slow start: the c = 0 motion (beta = 1 up to v0, then v0 ds = s ds)
        const R as = s0 < R(0) ? -s0 : s0;
        R y = as <= v0 ? as : (as * as + v0 * v0) * R(0.5) * inv_v0;
        y = (s0 < R(0) ? -y : y) + rhs;
        const R ay = y < R(0) ? -y : y;
        const R sy = ay <= v0 ? ay : Fm<R>::sqrt(R(2) * v0 * ay - v0 * v0);
        delta = (y < R(0) ? -sy : sy) - s0;
      }
      if (!(delta > lo && delta < hi)) delta = rhs * (w0 > v0 ? v0 / w0 : R(1));
      // Halley iteration on f(delta) = time_span - rhs, f' = max(1, W/v0),
      // f'' = s / (v0 W) where W > v0, kept inside the bracket [lo, hi]
      const R tol = sizeof(R) == 4 ? R(1e-7) : R(1e-16);
      // a Halley step of relative size e leaves an error of order e^3
      const R quick = sizeof(R) == 4 ? R(2e-3) : R(1e-8);
      for (int it = 0; it < 40; ++it) {
        const R s = s0 + delta;
        const R W = Fm<R>::sqrt(s * s + c * c);  // |v| at the end of the flight
        const R f = time_span(s0, delta, c, inv_v0, ss, v0, w0, W) - rhs;
        if (f > R(0)) hi = delta;
        else if (f < R(0)) lo = delta;
        else break;
        R step;
        if (W > v0) {
          // -2 f f' / (2 f'^2 - f f'') with f'' = s / (v0 W), over W
          const R hp = W * inv_v0;
          step = Fm<R>::div(R(-2) * f * hp * W, R(2) * hp * hp * W - f * s * inv_v0);
        } else {
          step = -f;
        }
        R dn = delta + step;
        const R astep = step < R(0) ? -step : step;
        if (astep <= quick * delta) {
          // converged to within step^2: take the step unless it leaves the
          // bracket (possible when it is below the resolution of delta)
          if (dn > lo && dn < hi) delta = dn;
          break;
        }
        if (!(dn > lo && dn < hi)) dn = R(0.5) * (lo + hi);
        delta = dn;
        if (hi - lo <= tol * hi) break;
      }
    }
    tau = Fm<R>::div(delta, at);
    dv = sg * delta;
  }
  disp = tau * (vx + R(0.5) * dv);
  vx1 = vx + dv;
  turns = (vx * dv < R(0)) && ((vx < R(0) ? -vx : vx) < (dv < R(0) ? -dv : dv));
  turn_disp = turns ? Fm<R>::div(-vx * vx, R(2) * a) : R(0);
}

// secondary electrons per ion reaching the cathode with energy eps [eV],
// Eq. (17) (Sec. IV)
template <typename R>
__device__ __forceinline__ R see_yield(R eps) {
  return R(0.09) * Fm<R>::pow(eps * R(1.0 / 700.0), eps < R(700) ? R(0.05) : R(0.72));
}

// Eq. (17) yield of an ion that reaches the cathode during this step from
// its state m at the start of the step: v_x^2 - 2 a x is constant along the
// flight, so at x = 0, v_x^2 = vx^2 - 2 a x with a gathered at x (the
// field is gathered again here, out of line on this rare path, so that the
// particle kernel keeps no extra registers for it)
template <typename R>
struct Mk;
template <typename R>
__device__ __noinline__ R impact_yield(const R* E, R qm, R dx, const Mk<R> m) {
  const R a = qm * (E[m.cell] + m.off * (E[m.cell + 1] - E[m.cell]));
  const R x0 = ((R)m.cell + m.off) * dx;
  R vx2 = m.vx * m.vx - R(2) * a * x0;
  vx2 = vx2 > R(0) ? vx2 : R(0);
  return see_yield<R>(R(0.5 * MAR / QE) * (vx2 + m.vy * m.vy + m.vz * m.vz));
}

// beta of Eq. (11) as min(1, v0/|v|) (deposit weights)
template <typename R>
__device__ __forceinline__ R beta_fast(R v2, R v0, int limited) {
  if (!limited) return R(1);
  const R v = Fm<R>::sqrt(v2);
  return v > v0 ? Fm<R>::div(v0, v) : R(1);
}
// FP32: one reciprocal square root instead of a square root and a
// reciprocal
__device__ __forceinline__ float beta_fast(float v2, float v0, int limited) {
  if (!limited) return 1.0f;
  return v2 > v0 * v0 ? v0 * __builtin_amdgcn_rsqf(v2) : 1.0f;
}

// ---------------------------------------------------------------- collisions
// A scattering angle as 1 - cos chi and 1 + cos chi, each formed without
// cancellation, so that sin chi = sqrt((1 - cos chi)(1 + cos chi)) keeps its
// relative accuracy at forward and backward angles alike.
template <typename R>
struct Chi {
  R omc, opc;
};

// Vahedi-Surendra angle law, cos chi = (2 + eps - 2 (1 + eps)^u) / eps:
//   1 - cos chi = 2 expm1(u L) / eps,
//   1 + cos chi = -2 (1 + eps) expm1(-(1 - u) L) / eps,   L = log1p(eps);
// eps -> 0 gives the isotropic law.  1 - u is exact for the uniforms used.
template <typename R>
__device__ __forceinline__ Chi<R> vs_angle(R eps, R u) {
  if (!(eps > R(0))) return Chi<R>{R(2) * u, R(2) * (R(1) - u)};
  const R L = Fm<R>::log1p(eps);
  const R k = Fm<R>::div(R(2), eps);
  return Chi<R>{k * Fm<R>::expm1(u * L), -(k + R(2)) * Fm<R>::expm1(-(R(1) - u) * L)};
}

// isotropic scattering: cos chi = 1 - 2u
template <typename R>
__device__ __forceinline__ Chi<R> iso_angle(R u) {
  return Chi<R>{R(2) * u, R(2) * (R(1) - u)};
}

// Turn unit vector (hx, hy, hz) by the angle chi and azimuth 2 pi u; the
// azimuth is measured from e1 = normalize(h x a), a the axis of the smallest
// |component| of h (ties to the lower index), e2 = h x e1.
template <typename R>
__device__ __forceinline__ void turn(R hx, R hy, R hz, Chi<R> chi, R u, R& ox, R& oy, R& oz) {
  const R ax = hx < R(0) ? -hx : hx, ay = hy < R(0) ? -hy : hy, az = hz < R(0) ? -hz : hz;
  R e1x, e1y, e1z;
  if (ay < ax && ay <= az) { e1x = -hz; e1y = R(0); e1z = hx; }       // axis y
  else if (az < ax && az < ay) { e1x = hy; e1y = -hx; e1z = R(0); }  // axis z
  else { e1x = R(0); e1y = hz; e1z = -hy; }                          // axis x
  const R n = Fm<R>::sqrt(e1x * e1x + e1y * e1y + e1z * e1z);
  e1x = Fm<R>::div(e1x, n); e1y = Fm<R>::div(e1y, n); e1z = Fm<R>::div(e1z, n);
  const R e2x = hy * e1z - hz * e1y, e2y = hz * e1x - hx * e1z, e2z = hx * e1y - hy * e1x;
  const R cosx = chi.omc <= R(1) ? R(1) - chi.omc : chi.opc - R(1);
  R sn = chi.omc * chi.opc;
  sn = sn > R(0) ? Fm<R>::sqrt(sn) : R(0);
  R sp, cp;
  Fm<R>::sincos2pi(u, &sp, &cp);
  ox = cosx * hx + sn * (cp * e1x + sp * e2x);
  oy = cosx * hy + sn * (cp * e1y + sp * e2y);
  oz = cosx * hz + sn * (cp * e1z + sp * e2z);
}

template <typename R>
__device__ __forceinline__ void unit3(R vx, R vy, R vz, R& hx, R& hy, R& hz) {
  const R s = Fm<R>::sqrt(vx * vx + vy * vy + vz * vz);
  if (s > R(0)) { hx = Fm<R>::div(vx, s); hy = Fm<R>::div(vy, s); hz = Fm<R>::div(vz, s); }
  else { hx = R(1); hy = R(0); hz = R(0); }
}

// Entry k of a per-channel table that no kernel writes, for a wave-uniform
// k: a scalar load through the constant address space.
template <typename T>
__device__ __forceinline__ T chan_entry(const T* table, int k) {
  using CT = const __attribute__((address_space(4))) T;
  return ((CT*)table)[k];
}

// Running sum over the NB channels of a table row (loaded at once, so
// that the collision waits for one memory access rather than one per
// channel); also picks the kind and threshold of the chosen channel from
// the uniform per-channel entries.  target_of() gives the target: it runs
// after the row's loads are issued, so that work it does (the candidate's
// draw) overlaps them.
template <typename R, int NB, typename F>
__device__ __forceinline__ int sum_channels(const Ctx<R>& C, const R* row, R eps, R t, R scale,
                                            F target_of, R& cum, int& kind, R& thr) {
  R a[NB], d[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    a[k] = row[k];
    d[k] = row[NB + k];
  }
  __builtin_amdgcn_sched_barrier(0);
  const R target = target_of();
  int ch = -1;
  R sum = R(0);
  kind = 0;
  thr = R(0);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const R tk = chan_entry(C.xs_thr, k);
    const R v = eps < tk ? R(0) : a[k] + t * d[k];
    sum += scale * v;
    if (ch < 0 && target < sum) {
      ch = k;
      kind = chan_entry(C.xs_kind, k);
      thr = tk;
    }
  }
  cum = sum;
  return ch;
}

// Channel choice of a collision candidate: the first channel k with
// target < sum_{q<=k} n_g sigma_q(eps) slow, where sigma_q is interpolated
// linearly between log-uniform nodes and is zero below the channel's
// threshold.  Returns -1 for a null collision; cum receives the full sum,
// kind and thr the chosen channel's kind and threshold.  target() returns
// the target (called once, after the table row is requested).
template <typename R, typename F>
__device__ __forceinline__ int select_channel(const Ctx<R>& C, R eps, R scale, F target, R& cum,
                                              int& kind, R& thr) {
  const int n = C.n_grid;
  // segment [i, i+1] holding eps, and the position t in it
  int i;
  R t;
  if (!(eps > C.e_lo)) { i = 0; t = R(0); }
  else if (!(eps < C.e_hi)) { i = n - 2; t = R(1); }
  else if (sizeof(R) == 4) {
    // FP32: the node energies of the log-uniform grid are e_lo g^i, g the
    // node ratio, computed rather than loaded, so that the cross sections
    // are the only dependent loads.  Within a few 1e-5 of a node the FP32
    // estimate of i may be the neighbouring segment; t, clamped to [0, 1],
    // then gives the node's value, a few 1e-5 of a segment's change away
    // from the interpolant (which is continuous at nodes).
    int ic = (int)((Fm<R>::log(eps) - C.log_emin) * C.inv_dlog);
    ic = ic < 0 ? 0 : (ic > n - 2 ? n - 2 : ic);
    const R e0 = C.e_lo * __builtin_amdgcn_exp2f((float)ic * (float)C.log2_ratio);
    i = ic;
    t = Fm<R>::div(eps - e0, e0 * C.ratio_m1);
    t = t < R(0) ? R(0) : (t > R(1) ? R(1) : t);
  } else {
    // FP64: the log-uniform estimate ic is off by at most one node, so the
    // energies of nodes ic-1 .. ic+2 are loaded together and the segment
    // holding eps is picked from them (as the table lookup of the oracle)
    int ic = (int)((Fm<R>::log(eps) - C.log_emin) * C.inv_dlog);
    ic = ic < 0 ? 0 : (ic > n - 2 ? n - 2 : ic);
    const int im = ic > 0 ? ic - 1 : 0, ip = ic + 2 < n ? ic + 2 : n - 1;
    const R em = C.xs_e[im], e0 = C.xs_e[ic], e1 = C.xs_e[ic + 1], ep = C.xs_e[ip];
    R el = e0, eh = e1;
    i = ic;
    if (eps < e0 && ic > 0) { i = ic - 1; el = em; eh = e0; }
    else if (!(eps < e1) && ic < n - 2) { i = ic + 1; el = e1; eh = ep; }
    t = Fm<R>::div(eps - el, eh - el);
  }
  // the node's row: values, then changes to the next node (padding
  // channels have zero cross sections and an infinite threshold)
  if (C.ncp == 4) return sum_channels<R, 4>(C, C.xs_sig + (size_t)i * 8, eps, t, scale, target, cum, kind, thr);
  return sum_channels<R, MAX_CHAN>(C, C.xs_sig + (size_t)i * (2 * MAX_CHAN), eps, t, scale, target,
                                   cum, kind, thr);
}

template <typename R>
struct Mk {  // one marker's state
  int32_t cell;
  R off, vx, vy, vz;
  uint64_t id;
  R w;       // flux weight in units of the instance's w_j (weight splitting)
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t gen_slot3(uint32_t g, uint32_t k) { return (g + k) % 3u; }

template <typename R>
__device__ __forceinline__ unsigned long long fixed_pt(R w, int shift);
// w in [0, 1] -> round(w 2^shift); FP32 uses shift <= 31 so one
// conversion to a 32-bit integer suffices
template <>
__device__ __forceinline__ unsigned long long fixed_pt<float>(float w, int shift) {
  return (unsigned long long)__float2uint_rn(__builtin_ldexpf(w, shift));
}
template <>
__device__ __forceinline__ unsigned long long fixed_pt<double>(double w, int shift) {
  return (unsigned long long)(__builtin_ldexp(w, shift) + 0.5);
}

// ---------------------------------------------------------------- tail
// Poisson problem of one instance on its N+1 nodes (phi_0 = 0, phi_N = V),
// solved as two prefix sums:
//   E_{k+1/2} = E_{1/2} + (dx/eps0) S_k,   S_k = sum_{j=1..k} rho_j,
//   E_{1/2} fixed by sum_k E_{k+1/2} dx = -V,
//   phi_i = -dx (i E_{1/2} + (dx/eps0) U_i),  U_i = sum_{k<i} S_k,
// with node fields E_i = (E_{i-1/2} + E_{i+1/2}) / 2 inside and Gauss's law
// over the half cell at each electrode.
constexpr double EPS0 = 8.8541878128e-12;


__device__ __forceinline__ size_t cidx(int n_inst, uint32_t slot, int inst, int sp, int p) {
  return ((((size_t)slot * n_inst + inst) * 2 + sp) * MAX_PART + p) * CSTRIDE;
}

// Marker chunks of one (buffer, species) as seen by a kernel: the base goes
// through the global address space, so that loads and stores of marker
// fields are global (not flat) accesses.
template <typename R>
__device__ __forceinline__ Soa<R> gbuf(const Ctx<R>& C, uint32_t b, int sp) {
  using GC = __attribute__((address_space(1))) char;
  return Soa<R>{(char*)(GC*)C.buf[b][sp].p};
}

// The partition of buffer S that starts at slot first (a multiple of CH),
// seen from one wave: its first chunk, the same for every lane, goes to
// scalar registers, so that slot accesses are a scalar base plus a 32-bit
// lane offset.
template <typename R>
__device__ __forceinline__ Part<R> part_of(const Soa<R>& S, int64_t first) {
  using GC = __attribute__((address_space(1))) char;
  const uint64_t a = (uint64_t)S.chunk(first);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return Part<R>{(char*)(GC*)(((uint64_t)hi << 32) | lo)};
}

// Marker count of an input partition of generation g.  Nothing writes the
// input slot of the count ring while the particle kernel runs (reservations
// go to slot g + 1), so it is read through the constant address space, with
// a scalar load.
__device__ __forceinline__ uint32_t count_in(const uint32_t* counts, int n_inst, uint32_t g,
                                             int inst, int sp, int p) {
  using CU = const __attribute__((address_space(4))) uint32_t;
  return ((CU*)counts)[cidx(n_inst, g % 3u, inst, sp, p)];
}

// Exclusive prefix sums of NV values over the NW waves of a workgroup:
// wave-level shuffles, then the first wave scans the wave totals (sh holds
// (NW + 1) NV doubles: each wave's prefix, then the sums).  ex[] receives
// the prefixes, tot[] the sums.
template <int NV, int NW = BLOCK / WAVE>
__device__ __forceinline__ void block_scan(const double (&v)[NV], double (&ex)[NV],
                                           double (&tot)[NV], double* sh) {
  static_assert(NW <= WAVE, "one wave scans the wave totals");
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  double inc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) inc[k] = v[k];
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double u = __shfl_up(inc[k], d);
      if (lane >= d) inc[k] += u;
    }
  }
  if (lane == WAVE - 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wave * NV + k] = inc[k];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double x = lane < NW ? sh[lane * NV + k] : 0.0;
      double w = x;
#pragma unroll
      for (int d = 1; d < NW; d <<= 1) {
        const double u = __shfl_up(w, d);
        if (lane >= d) w += u;
      }
      if (lane < NW) sh[lane * NV + k] = w - x;
      if (lane == NW - 1) sh[NW * NV + k] = w;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double prev = __shfl_up(inc[k], 1);
    ex[k] = sh[wave * NV + k] + (lane == 0 ? 0.0 : prev);
    tot[k] = sh[NW * NV + k];
  }
  __syncthreads();
}

// Continuous cathode source of a tail kernel (MODE_STEP): electrons at rest
// at x = 0, per_step w_j0 / w_j of them at the step's flux weight w_j (the
// integer part, and one more when a draw falls below the fraction), with
// ids from the INJECT channel and the step's population control.  The
// outputs follow the particle kernel's in the electron partitions, dealt
// round-robin; partition counts, the fullest count, the electron total and
// the event slots are updated.  Returns the fixed-point charge to add at
// node 0 (each kept marker has beta = 1 and offset 0).  Called by all
// threads (block-wide scans); pc holds the partition counts on entry.
template <typename R>
__device__ double inject(const Ctx<R>& C, IP& P, int inst, const InstState& cur, uint32_t g,
                         uint32_t bout, uint32_t* pc, double* sh, unsigned long long* ev,
                         uint32_t* n_e, uint32_t* mx_e, uint32_t* err) {
  const int t = threadIdx.x;
  const uint32_t step = cur.step;
  const double want = P.src * (P.w_j0 / cur.w_j);
  const double fl = floor(want);
  const U4 rf = draw(0, step, CH_INJECT | (1u << 8), C.seed, P.key);
  int64_t n = (int64_t)fl + (unif<double>(rf.x) < want - fl ? 1 : 0);
  if (n > P.cap) {  // more than the instance holds: an error, as in any overflow
    n = P.cap;
    if (t == 0) {
      atomicOr(C.inst_err + inst, (uint32_t)ERR_CAPACITY);
      atomicOr(err, (uint32_t)ERR_CAPACITY);
    }
  }
  const int parts = P.parts, pop = cur.popmode;
  const Soa<R> out = gbuf(C, bout, 0);
  int64_t base = 0;  // outputs of the earlier rounds
  for (int64_t k0 = 0; k0 < n; k0 += TBLOCK) {
    const int64_t k = k0 + t;
    uint64_t id[2] = {0, 0};
    int m = 0;
    if (k < n) {
      const U4 r = draw((uint64_t)k, step, CH_INJECT, C.seed, P.key);
      id[0] = child(r.x, r.y);
      m = 1;
      if (pop == POP_ROULETTE) {
        const U4 q = draw(id[0], step, CH_ROULETTE, C.seed, P.key);
        m = (q.x >> 9) < (1u << 22) ? 1 : 0;
      } else if (pop == POP_SPLIT) {
        const U4 q = draw(id[0], step, CH_CHILD | (1u << 8), C.seed, P.key);
        id[1] = child(q.x, q.y);
        m = 2;
      }
    }
    double v[1] = {(double)m}, ex[1], tot[1];
    block_scan<1, TBLOCK / WAVE>(v, ex, tot, sh);
    for (int j = 0; j < m; ++j) {
      const int64_t o = base + (int64_t)ex[0] + j;
      const int p = (int)(o % parts);
      const int64_t at = (int64_t)pc[p] + o / parts;
      if (at < P.cap_p) {
        const int64_t sl = P.seg + p * P.cap_p + at;
        out.cell(sl) = 0;
        out.off(sl) = R(0);
        out.vx(sl) = R(0);
        out.vy(sl) = R(0);
        out.vz(sl) = R(0);
        out.id(sl) = id[j];
        if (C.split) C.wt[bout][0][sl] = R(1);
      }
    }
    base += (int64_t)tot[0];
  }
  if (t == 0) {
    if (pop == POP_ROULETTE) ev[EV_ROULETTE] += (unsigned long long)(n - base);
    if (pop == POP_SPLIT) ev[EV_SPLIT] += (unsigned long long)n;
  }
  // partition p received the outputs o = p, p + parts, ...
  int64_t kept = 0;
  if (t < parts) {
    const int64_t add = base > t ? (base - t - 1) / parts + 1 : 0;
    int64_t c = (int64_t)pc[t] + add;
    if (c > P.cap_p) {
      c = P.cap_p;
      atomicOr(C.inst_err + inst, (uint32_t)ERR_CAPACITY);
      atomicOr(err, (uint32_t)ERR_CAPACITY);
    }
    kept = c - (int64_t)pc[t];
    C.counts[cidx(C.n_inst, (g + 1) % 3u, inst, 0, t)] = (uint32_t)c;
    atomicAdd(n_e, (uint32_t)kept);
    atomicMax(mx_e, (uint32_t)c);
  }
  double vk[1] = {(double)kept}, exk[1], totk[1];
  block_scan<1, TBLOCK / WAVE>(vk, exk, totk, sh);
  return __builtin_ldexp(totk[0], cur.dshift);
}

// One workgroup of TBLOCK threads per instance, launched after the particle
// kernel: charge density from the fixed-point deposit, Poisson solve,
// statistics row, population-control decision for the next step, the next
// deposit windows (every ANCHOR_PERIOD steps) and the generation switch.
// Every global load is issued up front; the prefix sums
// run in LDS (dynamic shared memory: max_cells + 1 doubles, then two rows
// of max_cells + 2 floats).
template <typename R, int MODE>
__global__ void __launch_bounds__(TBLOCK) k_tail(Ctx<R> C) {
  extern __shared__ double s_S[];          // rho, then S
  // [species][max_cells + 2]: deposit per node, then its prefix sums
  float* s_D = (float*)(s_S + C.max_cells + 1);
  const int DS = C.max_cells + 2;
  __shared__ double sh[(TBLOCK / WAVE + 1) * 5];
  __shared__ unsigned long long s_ev[NEV];
  __shared__ uint32_t s_cnt[2][2];         // [in, out][species]
  __shared__ uint32_t s_mx[2];             // fullest output partition per species
  __shared__ uint32_t s_err;               // capacity errors found here
  __shared__ uint32_t s_pc[MAX_PART];      // electron output partition counts
  __shared__ InstState s_cur;
  __shared__ uint32_t s_bs;
  // the next step's deposit windows: (float bits of the deposit) << 32 | first node
  __shared__ unsigned long long s_best[2];
  const int inst = blockIdx.x, t = threadIdx.x;
  IP& P = param(C.ip, inst);
  const int N = P.cells, node = P.node;
  // The generation, and what this kernel reads at an index that depends on
  // it: the state of both generations, both buffer selectors and this
  // thread's partition count in all three ring slots.  The particle kernel
  // has finished and nothing writes them before this kernel does, so they
  // go out first, with the deposit's loads, and are picked once the
  // generation is known.
  const uint32_t g = C.g->tail_gen;
  InstState st_a, st_b;
  uint32_t bs_a = 0u, bs_b = 0u, err0 = 0u;
  if (t == 0) {
    st_a = C.st[inst];
    st_b = C.st[C.n_inst + inst];
    bs_a = C.g->bufsel[0];
    bs_b = C.g->bufsel[1];
    err0 = C.inst_err[inst];
  }
  const int csp = t / MAX_PART, cpart = t % MAX_PART;
  const bool cown = t < 2 * MAX_PART && cpart < P.parts;
  uint32_t cnt3[3] = {0u, 0u, 0u};
  if (cown) {
#pragma unroll
    for (int s = 0; s < 3; ++s) cnt3[s] = C.counts[cidx(C.n_inst, (uint32_t)s, inst, csp, cpart)];
  }
  if (t < NEV) s_ev[t] = 0ull;
  if (t < 4) s_cnt[t / 2][t % 2] = 0u;
  if (t < 2) s_mx[t] = 0u;
  if (t == 0) {
    s_err = 0u;
    s_best[0] = s_best[1] = 0ull;
  }
  __syncthreads();

  // The loads that do not need the generation go first, so that they
  // overlap the loads that do: the deposit slots (each of the NSLOT copies
  // read with consecutive threads on consecutive nodes, UN nodes per thread
  // in flight together, then cleared) as raw fixed-point differences in
  // LDS with the species totals, and the step's event slots.
  double se = 0.0, si = 0.0;
  const size_t tn = (size_t)C.total_nodes;
  {
    unsigned long long* acc_e = C.acc + node;
    unsigned long long* acc_i = C.acc + (size_t)NSLOT * tn + node;
    constexpr int UN = 5;  // a 4096-cell gap in one round
    for (int i0 = t; i0 <= N; i0 += UN * TBLOCK) {
      unsigned long long ae[UN], ai[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        // past the last node, read the last node again (no branch around
        // the loads) and drop the sum
        const int i = min(i0 + u * TBLOCK, N);
        ae[u] = ai[u] = 0ull;
#pragma unroll
        for (int q = 0; q < NSLOT; ++q) {
          ae[u] += acc_e[q * tn + i];
          ai[u] += acc_i[q * tn + i];
        }
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int i = i0 + u * TBLOCK;
        if (i > N) break;
#pragma unroll
        for (int q = 0; q < NSLOT; ++q) {
          acc_e[q * tn + i] = 0ull;
          acc_i[q * tn + i] = 0ull;
        }
        se += (double)ae[u];
        si += (double)ai[u];
        s_S[i] = (double)ai[u] - (double)ae[u];
        s_D[i] = (float)(double)ae[u];
        s_D[DS + i] = (float)(double)ai[u];
      }
    }
    if (t < NEV * NSLOT) {
      unsigned long long* e = C.ev + (size_t)inst * NEV * NSLOT + t;
      const unsigned long long v = *e;
      *e = 0ull;
      if (v) atomicAdd(&s_ev[t / NSLOT], v);
    }
  }
  // the generation, then the state, buffer choice and partition counts
  const uint32_t sn = (g + 1) % 2u;
  if (t == 0) {
    // field by field (a select of whole records goes through memory)
    const bool odd = (g & 1u) != 0u;
    s_cur.w_j = odd ? st_b.w_j : st_a.w_j;
    s_cur.step = odd ? st_b.step : st_a.step;
    s_cur.popmode = odd ? st_b.popmode : st_a.popmode;
    s_cur.dshift = odd ? st_b.dshift : st_a.dshift;
    s_cur.anchor[0] = odd ? st_b.anchor[0] : st_a.anchor[0];
    s_cur.anchor[1] = odd ? st_b.anchor[1] : st_a.anchor[1];
    s_bs = odd ? bs_b : bs_a;
  }
  if (cown) {
    const int sp = csp, p = cpart;
    {
      const uint32_t g3 = g % 3u;
      uint32_t* co = C.counts + cidx(C.n_inst, (g + 1) % 3u, inst, sp, p);
      uint32_t* cf = C.counts + cidx(C.n_inst, (g + 2) % 3u, inst, sp, p);
      const uint32_t cin = g3 == 0u ? cnt3[0] : (g3 == 1u ? cnt3[1] : cnt3[2]);
      const uint32_t cout = g3 == 0u ? cnt3[1] : (g3 == 1u ? cnt3[2] : cnt3[0]);
      uint32_t c = MODE == MODE_STEP ? cout : cin;
      if (c > (uint32_t)P.cap_p) {
        atomicOr(C.inst_err + inst, (uint32_t)ERR_CAPACITY);
        atomicOr(&s_err, (uint32_t)ERR_CAPACITY);
        c = (uint32_t)P.cap_p;
      }
      *co = c;
      *cf = 0u;
      if (sp == 0) s_pc[p] = c;
      atomicAdd(&s_cnt[0][sp], cin);
      atomicAdd(&s_cnt[1][sp], c);
      atomicMax(&s_mx[sp], c);
    }
  }
  __syncthreads();
  const InstState cur = s_cur;
  if (MODE == MODE_STEP && P.src > 0.0) {
    const double q = inject(C, P, inst, cur, g, 1u - s_bs, s_pc, sh, s_ev, &s_cnt[1][0], &s_mx[0], &s_err);
    if (t == 0) {
      s_S[0] -= q;
      se += q;
    }
  }
  const double factor = MODE == MODE_STEP
                            ? (cur.popmode == POP_ROULETTE ? 2.0 : (cur.popmode == POP_SPLIT ? 0.5 : 1.0))
                            : 1.0;
  const double wj = cur.w_j * factor;
  // the shift this step's deposits used, and the next step's: with weight
  // splitting the base raised by floor(-log2) of the largest output flux
  // weight (an active source injects weight 1)
  const int dsh = MODE == MODE_STEP ? cur.dshift : C.dep_shift;
  const double unit = __builtin_ldexp(1.0, -dsh);
  int next_dsh = C.dep_shift;
  if (MODE == MODE_STEP && C.split) {
    float mw = __uint_as_float(C.maxw[inst]);
    if (P.src > 0.0) mw = 1.0f;
    if (mw > 0.0f && mw < 1.0f) {
      int e;
      (void)frexpf(mw, &e);  // mw in [2^(e-1), 2^e)
      next_dsh += -e;        // floor(-log2 mw) >= -e
    }
  }
  const double qvol = QE * wj * unit / (P.area * P.dx);
  // charge density at the nodes this thread read (half cells at the
  // electrodes); with the flux diagnostic, the step's node crossings times
  // the flux weight the markers had in it
  {
    double* rho = C.rho + (size_t)sn * C.total_nodes + node;
    const bool flux = MODE == MODE_STEP && (C.flags & 4u);
    for (int i = t; i <= N; i += TBLOCK) {
      double r = s_S[i] * qvol;
      if (i == 0 || i == N) r *= 2.0;
      rho[i] = r;
      s_S[i] = r;
      if (flux) {
        for (int sp = 0; sp < 2; ++sp) {
          const size_t at = (size_t)sp * tn + node + i;
          const int32_t c = C.cross[at];
          if (c) {
            C.flux[at] += cur.w_j * (double)c;
            C.cross[at] = 0;
          }
        }
      }
    }
  }
  __syncthreads();

  // S_i = sum_{j=1..i} rho_j for i < N (S_0 = 0), then U_i = sum_{k<i} S_k,
  // both over contiguous chunks per thread
  const int chunk = (N + 1 + TBLOCK - 1) / TBLOCK;
  const int i0 = t * chunk, i1 = min(i0 + chunk, N + 1);
  const double rho0 = s_S[0], rhoN = s_S[N];
  // the deposit windows of the next step are chosen every ANCHOR_PERIOD
  // steps (the dense regions move slowly) and carried over in between
  const bool choose = MODE == MODE_REFRESH || cur.step % ANCHOR_PERIOD == 0u;
  double wtot[2];  // species totals (fixed point)
  double usum = 0.0;
  // the pass, with (D) or without the deposit's prefix sums
  auto s_pass = [&](auto with_d) {
    constexpr bool D = decltype(with_d)::value;
    constexpr int NV = D ? 5 : 3;
    double v[NV], ex[NV], tot[NV];
    double loc = 0.0, dle = 0.0, dli = 0.0;
    for (int i = i0; i < i1; ++i) {
      if (i >= 1 && i <= N - 1) loc += s_S[i];
      if (D) {
        dle += (double)s_D[i];
        dli += (double)s_D[DS + i];
      }
    }
    v[0] = loc;
    v[1] = se;
    v[2] = si;
    if (D) {
      v[NV - 2] = dle;
      v[NV - 1] = dli;
    }
    block_scan<NV, TBLOCK / WAVE>(v, ex, tot, sh);
    double run = ex[0], drun_e = D ? ex[NV - 2] : 0.0, drun_i = D ? ex[NV - 1] : 0.0;
    for (int i = i0; i < i1; ++i) {
      if (i >= 1 && i <= N - 1) run += s_S[i];
      const double sv = (i == 0) ? 0.0 : (i <= N - 1 ? run : 0.0);
      s_S[i] = sv;
      if (i <= N - 1) usum += sv;
      if (D) {
        // deposit of the nodes before i (rounding keeps the sums ordered)
        const double de = (double)s_D[i], di = (double)s_D[DS + i];
        s_D[i] = (float)drun_e;
        s_D[DS + i] = (float)drun_i;
        drun_e += de;
        drun_i += di;
      }
    }
    if (D && t == 0) {
      s_D[N + 1] = (float)tot[NV - 2];
      s_D[DS + N + 1] = (float)tot[NV - 1];
    }
    wtot[0] = tot[1];
    wtot[1] = tot[2];
  };
  if (choose) s_pass(std::true_type{});
  else s_pass(std::false_type{});
  double v1[1] = {usum}, ex1[1], tot1[1];
  block_scan<1, TBLOCK / WAVE>(v1, ex1, tot1, sh);  // its barriers also publish s_S and s_D
  const double T = tot1[0];
  const double dx = P.dx, k = dx / EPS0;
  const double Ehalf = (-P.V / dx - k * T) / (double)N;
  double* phi = C.phi + (size_t)sn * C.total_nodes + node;
  double* E64 = C.E64 + (size_t)sn * C.total_nodes + node;
  R* ER = C.E + (size_t)sn * C.total_nodes + node;
  double U = ex1[0];
  for (int i = i0; i < i1; ++i) {
    double e;
    if (i == 0) e = Ehalf - rho0 * dx / (2.0 * EPS0);
    else if (i == N) e = Ehalf + k * s_S[N - 1] + rhoN * dx / (2.0 * EPS0);
    else e = Ehalf + k * 0.5 * (s_S[i - 1] + s_S[i]);
    phi[i] = (i == N) ? P.V : -dx * ((double)i * Ehalf + k * U);
    E64[i] = e;
    ER[i] = (R)e;
    if (i <= N - 1) U += s_S[i];
  }
  if (choose) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      // the next step's deposit window of each species: of the HWIN-node
      // windows inside the gap, the one that took the species' largest
      // deposit in this step (nonnegative floats order as their bit patterns)
      const float* D = s_D + sp * DS;
      unsigned long long best = 0ull;
      const int top = min(i1 - 1, N + 1 - HWIN);
      for (int a = i0; a <= top; ++a) {
        const float w = D[a + HWIN] - D[a];
        const unsigned long long key =
            (unsigned long long)__float_as_uint(w) << 32 | (unsigned long long)(uint32_t)a;
        best = key > best ? key : best;
      }
#pragma unroll
      for (int d = 1; d < WAVE; d <<= 1) {
        const unsigned long long o = __shfl_xor(best, d);
        best = o > best ? o : best;
      }
      if ((t & (WAVE - 1)) == 0 && best) atomicMax(&s_best[sp], best);
    }
    __syncthreads();
  }

  if (t == 0) {
    const int64_t n[2] = {(int64_t)s_cnt[1][0], (int64_t)s_cnt[1][1]};
    const int64_t nin = (int64_t)s_cnt[0][0] + s_cnt[0][1];
    const int64_t nout = n[0] + n[1];
    int32_t pm = POP_NONE;
    if (P.n_target > 0) {
      if (nout > 2 * P.n_target) pm = POP_ROULETTE;
      else if (nout > 0 && 2 * nout < P.n_target) pm = POP_SPLIT;
    }
    InstState nx;
    nx.w_j = wj;
    nx.step = cur.step + (MODE == MODE_STEP ? 1u : 0u);
    nx.popmode = pm;
    nx.dshift = next_dsh;
    // 0 where the gap fits one window
    nx.anchor[0] = choose ? (int)(uint32_t)s_best[0] : cur.anchor[0];
    nx.anchor[1] = choose ? (int)(uint32_t)s_best[1] : cur.anchor[1];
    if (C.split) C.maxw[inst] = 0u;
    C.st[sn * C.n_inst + inst] = nx;
    if (MODE == MODE_STEP) {
      // field by field, so that the row is never held in registers
      StatsRow& row = C.ring[(size_t)inst * RING + (nx.step - 1) % RING];
      row.step = nx.step;
      row.n_e = n[0];
      row.n_i = n[1];
      row.n_in = nin;
      row.w_e = wtot[0] * unit * wj;
      row.w_i = wtot[1] * unit * wj;
      row.w_j = wj;
      for (int q = 0; q < NEV; ++q) row.ev[q] = (int64_t)s_ev[q];
      row.err = err0 | s_err;
    }
    for (int sp = 0; sp < 2; ++sp)
      C.tiles[(size_t)((g + 1) % 3u) * 2 * C.n_inst + 2 * inst + sp] = pair_tiles(s_mx[sp], P.parts);
    C.g->bufsel[(g + 1) % 2u] = MODE == MODE_STEP ? 1u - s_bs : s_bs;
    if (inst == 0)  // the next particle kernel's claims
      for (int p = 0; p < NPOOL; ++p) C.g->claim[(g + 1) % 2u][p][0] = 0u;
    C.g->cur_gen = g + 1;
  }
}

// ---------------------------------------------------------------- deposit
// A workgroup accumulates its markers' fixed-point weights in an LDS window
// of HWIN nodes (the whole grid when it fits) for the (instance, species) of
// its tiles, and adds the window to global memory each time it moves on to
// another (instance, species), into one of NSLOT copies of each node picked
// by the workgroup index: the tail kernel sums the copies.  Nodes outside
// the window, and the few products of the other species (ions from
// ionization in electron tiles, secondary electrons in ion tiles), go to
// global memory directly.
struct DepWin {
  int inst, sp, anchor;
};

__device__ __forceinline__ void dep_add(unsigned long long* acc, unsigned long long* hist,
                                        const DepWin& w, int sp, int node0, int total_nodes,
                                        int cell, unsigned long long lo, unsigned long long hi) {
  const int r = cell - w.anchor;
  if (sp == w.sp && r >= 0 && r + 1 < HWIN) {
    if (lo) atomicAdd(&hist[r], lo);
    if (hi) atomicAdd(&hist[r + 1], hi);
  } else {
    // the accumulators are global memory: global (not flat) atomics
    using GU = __attribute__((address_space(1))) unsigned long long;
    const int slot = blockIdx.x % NSLOT;
    unsigned long long* a =
        (unsigned long long*)((GU*)acc + ((size_t)sp * NSLOT + slot) * total_nodes + node0 + cell);
    if (lo) atomicAdd(a, lo);
    if (hi) atomicAdd(a + 1, hi);
  }
}

// Adds the window and the event counts gathered since the last flush (one
// LDS row per wave) to global memory.  Called by all threads.
template <typename R>
__device__ __forceinline__ void dep_flush(const Ctx<R>& C, unsigned long long* hist,
                                          const DepWin& w, uint32_t (*evw)[NEV]) {
  __syncthreads();
  const int slot = blockIdx.x % NSLOT;
  if (threadIdx.x < NEV) {
    uint32_t v = 0u;
#pragma unroll
    for (int q = 0; q < BLOCK / WAVE; ++q) {
      v += evw[q][threadIdx.x];
      evw[q][threadIdx.x] = 0u;
    }
    if (v) atomicAdd(C.ev + ((size_t)w.inst * NEV + threadIdx.x) * NSLOT + slot,
                     (unsigned long long)v);
  }
  IP& P = param(C.ip, w.inst);
  const int nn = min(HWIN, P.cells + 1 - w.anchor);
  using GU = __attribute__((address_space(1))) unsigned long long;
  unsigned long long* dst = (unsigned long long*)((GU*)C.acc +
                                                  ((size_t)w.sp * NSLOT + slot) * C.total_nodes +
                                                  P.node + w.anchor);
  for (int i = threadIdx.x; i < nn; i += BLOCK) {
    const unsigned long long v = hist[i];
    if (v) {
      atomicAdd(dst + i, v);
      hist[i] = 0ull;
    }
  }
  __syncthreads();
}

// Tile space of generation g: the electrons of instance 0, 1, ..., then the
// ions of instance 0, 1, ... (a workgroup's run of tiles then changes
// species at most once per step, and its deposit window with it); an
// (instance, species) with P partitions gets P * T tiles, T = max_p
// ceil(n_p / BLOCK), and tile j reads chunk j mod T of partition j / T
// (partitions in order, so that the tiles of a cell-sorted (instance,
// species) follow its cells).  Fills s_prefix[q] with the first tile of
// position q (q = 0 .. 2 n_inst; pair_at gives its instance and species).
// Called by all threads; ends with a barrier.
__device__ __forceinline__ void pair_at(int q, int n_inst, int& inst, int& sp) {
  sp = q >= n_inst ? 1 : 0;
  inst = q - sp * n_inst;
}

// Thread t owns positions t * per + j, j < per = ceil(2 n_inst / BLOCK) <=
// MAXPER; count_of(j, k) gives the tile count of its j-th position k.
constexpr int MAXPER = (2 * MAX_INST + BLOCK - 1) / BLOCK;

template <typename R, typename F>
__device__ void tile_prefix_of(const Ctx<R>& C, uint32_t* s_prefix, double* s_scan, F count_of) {
  const int tid = threadIdx.x, nk = 2 * C.n_inst;
  const int per = (nk + BLOCK - 1) / BLOCK;
  uint32_t loc = 0;
#pragma unroll
  for (int j = 0; j < MAXPER; ++j) {
    const int k = tid * per + j;
    if (j < per && k < nk) {
      const uint32_t tl = count_of(j, k);
      s_prefix[k + 1] = tl;
      loc += tl;
    }
  }
  double v1[1] = {(double)loc}, ex1[1], tot1[1];
  block_scan<1>(v1, ex1, tot1, s_scan);
  uint32_t run = (uint32_t)ex1[0];
  if (tid == 0) s_prefix[0] = 0;
  __syncthreads();
  for (int k = tid * per; k < min(nk, (tid + 1) * per); ++k) {
    run += s_prefix[k + 1];
    s_prefix[k + 1] = run;
  }
  __syncthreads();
}

// per (instance, species): its tile count, set with the partition counts
// (by the tail kernel, the cell sort or the host) at 2 instance + species
// of ring slot g mod 3
template <typename R>
__device__ __forceinline__ const uint32_t* tile_counts(const Ctx<R>& C, uint32_t slot, int k) {
  int inst, sp;
  pair_at(k, C.n_inst, inst, sp);
  return C.tiles + (size_t)slot * 2 * C.n_inst + 2 * inst + sp;
}

template <typename R>
__device__ void tile_prefix(const Ctx<R>& C, uint32_t g, uint32_t* s_prefix, double* s_scan) {
  tile_prefix_of(C, s_prefix, s_scan, [&](int, int k) { return *tile_counts(C, g % 3u, k); });
}

// Position of tiles in the tile space: a cursor that finds its first tile by
// bisection and then only moves forward.  For tile t it gives the pair k,
// the tile's partition, and the first marker slot of its chunk.
struct TileCursor {
  int kc = -1;
  uint32_t kbeg = 0, kend = 0;
  uint32_t next = 0xffffffffu;  // tile whose place is in (part, chunk)
  uint32_t per_part = 0, chunk = 0;
  int part = 0;
  __device__ void locate(const uint32_t* s_prefix, int nk, uint32_t t) {
    if (kc < 0) {
      int lo = 0, hi = nk;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_prefix[mid] <= t) lo = mid;
        else hi = mid;
      }
      kc = lo;
      kbeg = s_prefix[kc];
      kend = s_prefix[kc + 1];
      // a new run can begin on the tile after the last run's end, in
      // another pair: the place then has to be computed afresh
      next = 0xffffffffu;
    }
    while (t >= kend) {
      ++kc;
      kbeg = kend;
      kend = s_prefix[kc + 1];
      next = 0xffffffffu;
    }
  }
  // partition and first slot of tile t (after locate(t)) for P partitions,
  // P a power of two.  A workgroup walks its tiles in order, so the place of
  // the next tile follows from this one's; the division runs only on the
  // first tile of a pair.
  __device__ void place(uint32_t t, int parts, int& part_out, uint32_t& first) {
    if (t != next) {
      per_part = (kend - kbeg) >> __builtin_ctz((uint32_t)parts);  // tiles per partition
      const uint32_t j = t - kbeg;
      part = (int)(j / per_part);
      chunk = j - (uint32_t)part * per_part;
    }
    part_out = part;
    first = chunk * BLOCK;
    next = t + 1u;
    if (++chunk == per_part) {
      chunk = 0;
      ++part;
    }
  }
};

// ---------------------------------------------------------------- main kernel
template <typename R, bool WS>
struct LaneOut {
  // electrons produced by this lane (before population control): the marker
  // or its emitted electron, an ionization's ejected electron and, with
  // weight splitting, the scattered part of a split primary
  static constexpr int NE = WS ? 3 : 2;
  // ions: the marker or an ionization's new ion, and with weight splitting
  // the scattered part of a split charge exchange
  static constexpr int NI = WS ? 2 : 1;
  Mk<R> e[NE];
  Mk<R> i[NI];
  uint32_t me, mi;   // which slots of e[] and i[] are set (bit j: slot j)
};

constexpr int NWAVE = BLOCK / WAVE;
// collision-queue slots per wave: fewer than WAVE wait between tiles, and a
// tile adds at most WAVE
constexpr int QW = 2 * WAVE;

// a wave-uniform or lane ring position a + b for a, b < QW
__device__ __forceinline__ uint32_t ring(uint32_t a, uint32_t b) {
  const uint32_t s = a + b;
  return s >= (uint32_t)QW ? s - (uint32_t)QW : s;
}

// What a wave is working on: one (instance, species), and the output
// partition of its next emit.
struct Work {
  int inst, sp, part;
  uint32_t step;
  int pop;
  int dshift;        // fraction bits of this step's fixed-point deposit
  int64_t pbase;
  uint32_t emits;
};

// Output partition of a wave's next emit: an integer hash of (wave, emit
// number, step), so that each partition receives an equal share of a step's
// output in expectation whatever partition the markers came from, and no
// fixed stride between tiles can map one input partition to one output
// partition step after step.
__device__ __forceinline__ void next_output(Work& W, IP& P) {
  const uint32_t wid = blockIdx.x * (uint32_t)NWAVE + threadIdx.x / WAVE;
  uint32_t h = wid * 0x9E3779B1u ^ (W.emits * 0x85EBCA77u + W.step * 0xC2B2AE3Du);
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  h *= 0x846CA68Bu;
  h ^= h >> 16;
  W.part = (int)(h & (uint32_t)(P.parts - 1));  // parts is a power of two
  W.pbase = P.seg + (int64_t)W.part * P.cap_p;
  ++W.emits;
}

// Population control, charge deposit, event counts and stream compaction of
// the markers each lane of one wave produced.  Called by all lanes of the
// wave, independently of the other waves.  QUEUE: outputs of collided
// candidates (collision events) rather than of a tile (wall and emission
// events).  Event counts go to the wave's row evw of LDS counters.  WS: the
// markers carry flux weights (weight splitting), which scale their deposit
// and are stored with them.
template <typename R, int MODE, bool QUEUE, bool WS>
__device__ __forceinline__ void emit(const Ctx<R>& C, const Work& W, const DepWin& win,
                                     unsigned long long* hist, const LaneOut<R, WS>& o,
                                     uint32_t ev, uint32_t err, uint32_t g, uint32_t bsel,
                                     uint32_t* evw) {
  constexpr int NE = LaneOut<R, WS>::NE, NI = LaneOut<R, WS>::NI;
  const int lane = threadIdx.x & (WAVE - 1);
  IP& P = param(C.ip, W.inst);
  const int inst = W.inst, pop = W.pop;
  const uint32_t step = W.step;
  const R v0 = PR(P, v0);
  const int limited = P.limited;

  // population control: each output is kept (roulette) or doubled (split)
  uint32_t keep_e = 0, keep_i = 0;
  uint64_t clone_e[NE], clone_i[NI];
  int cnt_e = 0, cnt_i = 0;
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    clone_e[j] = 0;
    if (!(o.me >> j & 1u)) continue;
    if (pop == POP_ROULETTE) {
      const U4 r = draw_cold(o.e[j].id, step, CH_ROULETTE, C.seed, P.key);
      if ((r.x >> 9) < (1u << 22)) { keep_e |= 1u << j; ++cnt_e; }
    } else {
      keep_e |= 1u << j;
      ++cnt_e;
      if (pop == POP_SPLIT) {
        const U4 r = draw_cold(o.e[j].id, step, CH_CHILD | (1u << 8), C.seed, P.key);
        clone_e[j] = child(r.x, r.y);
        ++cnt_e;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    clone_i[j] = 0;
    if (!(o.mi >> j & 1u)) continue;
    if (pop == POP_ROULETTE) {
      const U4 r = draw_cold(o.i[j].id, step, CH_ROULETTE, C.seed, P.key);
      if ((r.x >> 9) < (1u << 22)) { keep_i |= 1u << j; ++cnt_i; }
    } else {
      keep_i |= 1u << j;
      ++cnt_i;
      if (pop == POP_SPLIT) {
        const U4 r = draw_cold(o.i[j].id, step, CH_CHILD | (1u << 8), C.seed, P.key);
        clone_i[j] = child(r.x, r.y);
        ++cnt_i;
      }
    }
  }
  // at most NE + NI outputs per lane (one from a tile; three, or five with
  // weight splitting, from a collision)
  const int n_out = __popc(o.me) + __popc(o.mi);
  const int removed = pop == POP_ROULETTE ? n_out - (cnt_e + cnt_i) : 0;
  const int split_added = pop == POP_SPLIT ? n_out : 0;

  // compaction: prefix within the wave by bit-sliced ballots (cnt_e in
  // 0..2 NE, cnt_i in 0..2 NI), one reservation per wave and species on the
  // partition's counter.  The reservations go out before the deposit and the
  // event counts, which run while they return.
  constexpr bool E3 = QUEUE || WS;   // cnt_e can reach 4
  constexpr bool I3 = QUEUE && WS;   // cnt_i can reach 4
  const unsigned long long lt = (1ull << lane) - 1ull;
  const unsigned long long be0 = __ballot(cnt_e & 1), be1 = __ballot(cnt_e & 2),
                           be2 = E3 ? __ballot(cnt_e & 4) : 0ull;
  const unsigned long long bi0 = __ballot(cnt_i & 1), bi1 = __ballot(cnt_i & 2),
                           bi2 = I3 ? __ballot(cnt_i & 4) : 0ull;
  const uint32_t pre_e = __popcll(be0 & lt) + 2 * __popcll(be1 & lt) + 4 * __popcll(be2 & lt);
  const uint32_t pre_i = __popcll(bi0 & lt) + 2 * __popcll(bi1 & lt) + 4 * __popcll(bi2 & lt);
  const uint32_t te = __popcll(be0) + 2 * __popcll(be1) + 4 * __popcll(be2);
  const uint32_t ti = __popcll(bi0) + 2 * __popcll(bi1) + 4 * __popcll(bi2);
  uint32_t base_e = 0u, base_i = 0u;
  if (MODE == MODE_STEP && lane == 0) {
    if (te) base_e = atomicAdd(C.counts + cidx(C.n_inst, (g + 1) % 3u, inst, 0, W.part), te);
    if (ti) base_i = atomicAdd(C.counts + cidx(C.n_inst, (g + 1) % 3u, inst, 1, W.part), ti);
  }
  // deposit (fixed point, units of q w_j): every kept marker adds its two
  // linear weights, times its flux weight with weight splitting, to the LDS
  // window (clones count twice: one bit more)
  {
    // whole markers always use the base shift
    const int shift = WS ? W.dshift : C.dep_shift;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      if (!(keep_e >> q & 1u)) continue;
      const Mk<R>& e = o.e[q];
      R b = beta_fast(e.vx * e.vx + e.vy * e.vy + e.vz * e.vz, v0, limited);
      if (WS) b *= e.w;
      const uint32_t dbl = clone_e[q] ? 1u : 0u;
      dep_add(C.acc, hist, win, 0, P.node, C.total_nodes, e.cell,
              fixed_pt<R>(b * (R(1) - e.off), shift) << dbl, fixed_pt<R>(b * e.off, shift) << dbl);
    }
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      if (!(keep_i >> q & 1u)) continue;
      const Mk<R>& e = o.i[q];
      R b = beta_fast(e.vx * e.vx + e.vy * e.vy + e.vz * e.vz, v0, limited);
      if (WS) b *= e.w;
      const uint32_t dbl = clone_i[q] ? 1u : 0u;
      dep_add(C.acc, hist, win, 1, P.node, C.total_nodes, e.cell,
              fixed_pt<R>(b * (R(1) - e.off), shift) << dbl, fixed_pt<R>(b * e.off, shift) << dbl);
    }
  }

  // events: wave totals by ballot; removed and split_added are in 0..NE+NI
  if (QUEUE) {
    if (__ballot(ev != 0u)) {
#pragma unroll
      for (int q = EV_ELASTIC; q < EV_ABS_E_CATH; ++q) {
        const uint32_t n = (uint32_t)__popcll(__ballot((ev >> q) & 1u));
        if (lane == 0 && n) atomicAdd(&evw[q], n);
      }
    }
  } else {
    // wall and emission events are rare: the lanes that have one count it
    uint32_t b = ev;
    while (b) {
      const int q = __builtin_ctz(b);
      atomicAdd(&evw[q], 1u);
      b &= b - 1u;
    }
  }
  if (pop != POP_NONE) {
    const int x = pop == POP_ROULETTE ? removed : split_added;
    const uint32_t n = (uint32_t)(__popcll(__ballot(x & 1)) + 2 * __popcll(__ballot(x & 2)) +
                                  4 * __popcll(__ballot(x & 4)));
    if (lane == 0 && n) atomicAdd(&evw[pop == POP_ROULETTE ? EV_ROULETTE : EV_SPLIT], n);
  }
  if (err) atomicOr(C.inst_err + inst, err);

  if (MODE != MODE_STEP) return;
  if (WS) {
    // the largest flux weight among the wave's outputs, for the next
    // step's deposit shift (positive floats order as their bit patterns)
    float mw = 0.0f;
#pragma unroll
    for (int j = 0; j < NE; ++j)
      if (keep_e >> j & 1u) mw = fmaxf(mw, (float)o.e[j].w);
#pragma unroll
    for (int j = 0; j < NI; ++j)
      if (keep_i >> j & 1u) mw = fmaxf(mw, (float)o.i[j].w);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mw = fmaxf(mw, __shfl_xor(mw, d));
    if (lane == 0 && mw > 0.0f) atomicMax(C.maxw + inst, __float_as_uint(mw));
  }
  const Part<R> oe = part_of(gbuf(C, 1 - bsel, 0), W.pbase), oi = part_of(gbuf(C, 1 - bsel, 1), W.pbase);
  R* const we = WS ? C.wt[1 - bsel][0] : nullptr;
  R* const wi = WS ? C.wt[1 - bsel][1] : nullptr;
  uint32_t pe = __builtin_amdgcn_readfirstlane(base_e) + pre_e;
  uint32_t pi = __builtin_amdgcn_readfirstlane(base_i) + pre_i;
  uint32_t werr = 0;
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    if (!(keep_e >> j & 1u)) continue;
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      if (rep == 1 && !clone_e[j]) continue;
      if (pe < (uint32_t)P.cap_p) {
        const SlotOff<R> q(pe);
        oe.cell(q) = o.e[j].cell;
        oe.off(q) = o.e[j].off;
        oe.vx(q) = o.e[j].vx;
        oe.vy(q) = o.e[j].vy;
        oe.vz(q) = o.e[j].vz;
        oe.id(q) = rep ? clone_e[j] : o.e[j].id;
        if (WS) we[W.pbase + pe] = o.e[j].w;
      } else {
        werr |= ERR_CAPACITY;
      }
      ++pe;
    }
  }
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    if (!(keep_i >> j & 1u)) continue;
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      if (rep == 1 && !clone_i[j]) continue;
      if (pi < (uint32_t)P.cap_p) {
        const SlotOff<R> q(pi);
        oi.cell(q) = o.i[j].cell;
        oi.off(q) = o.i[j].off;
        oi.vx(q) = o.i[j].vx;
        oi.vy(q) = o.i[j].vy;
        oi.vz(q) = o.i[j].vz;
        oi.id(q) = rep ? clone_i[j] : o.i[j].id;
        if (WS) wi[W.pbase + pi] = o.i[j].w;
      } else {
        werr |= ERR_CAPACITY;
      }
      ++pi;
    }
  }
  if (werr) atomicOr(C.inst_err + inst, werr);
}

// Electron-neutral collision of a candidate (Sec. III, Sec. IV): channel by
// the SLPIC rate of Eq. (16) or the fixed-event thresholds, then the scatter
// law of the channel; ionization spawns an electron and an ion.  With weight
// splitting (WS and f_e < 1) the primary stays as the uncollided part with
// the fraction 1 - f_e of its flux weight and its velocity, and the
// scattered part and the products carry f_e (Sec. III: w_j,p0 = w_j,p1 +
// W_j,c); the scattered part's id comes from channel CHILD, sub 2.
template <typename R, bool WS>
__device__ void collide_electron(const Ctx<R>& C, IP& P, int inst, uint32_t step,
                                 Mk<R>& m, LaneOut<R, WS>& o, uint32_t& ev, uint32_t& err) {
  U4 r;
  const R v2 = m.vx * m.vx + m.vy * m.vy + m.vz * m.vz;
  const R eps = v2 * (R)(0.5 * ME / QE);
  const bool split = WS && P.f_e < 1.0;
  int ch = -1, kind = 0;
  R thr = R(0);
  if (C.fixed) {
    r = draw(m.id, step, CH_COLL, C.seed, P.key);
    // whole markers: channel from the candidate's own word; split: from
    // the second word, with probability fixed_k / (their sum)
    const uint32_t u = (split ? r.y : r.x) >> 9;
    for (int q = 0; q < C.n_chan; ++q)
      if (ch < 0 && u < (split ? P.t_fsplit[q] : P.t_fixed[q])) ch = q;
    // its kind and threshold, picked from the uniform per-channel entries
    // (no dependent per-lane load)
    for (int q = 0; q < C.n_chan; ++q) {
      const int kq = chan_entry(C.xs_kind, q);
      const R tq = chan_entry(C.xs_thr, q);
      kind = q == ch ? kq : kind;
      thr = q == ch ? tq : thr;
    }
  } else {
    const R sp0 = Fm<R>::sqrt(v2);
    const R v0 = PR(P, v0);
    const R slow = P.limited ? (sp0 < v0 ? sp0 : v0) : sp0;
    const R numax = PR(P, nu_max_e);
    R cum;
    // the draw runs while the cross-section row is loaded
    auto target = [&]() {
      r = draw(m.id, step, CH_COLL, C.seed, P.key);
      return unif<R>(r.y) * numax;
    };
    ch = select_channel(C, eps, PR(P, n_g) * slow, target, cum, kind, thr);
    if (cum > numax * R(1.000001)) err |= ERR_NU_BOUND;
  }
  o.e[0] = m;
  o.me = 1u;
  if (ch >= 0) {
    R hx, hy, hz, ox, oy, oz;
    unit3(m.vx, m.vy, m.vz, hx, hy, hz);
    // ionization: share eps - I between the scattered and the ejected
    // electron (only ionizing lanes draw)
    const bool ioniz = kind == 2;
    R eej = R(0), esc = R(0);
    U4 q = U4{0u, 0u, 0u, 0u};
    if (ioniz) {
      q = draw_cold(m.id, step, CH_IONIZ, C.seed, P.key);
      R eav = eps - thr;
      eav = eav > R(0) ? eav : R(0);
      const R B = (R)C.ion_B;
      eej = B * m_tan(unif<R>(q.x) * m_atan(eav / (R(2) * B)));
      esc = eav - eej;
      if (C.flags & 1u) { eej = R(0); esc = R(0); }
    }
    // the primary leaves by one rotation whatever the channel: the
    // Vahedi-Surendra angle at its energy for elastic scattering and
    // ionization, isotropic for excitation
    const Chi<R> chi = kind == 1 ? iso_angle(unif<R>(r.z)) : vs_angle(kind == 0 ? eps : esc, unif<R>(r.z));
    R e1;
    if (kind == 0) e1 = eps * (R(1) - R(2.0 * ME / MAR) * chi.omc);
    else if (kind == 1) e1 = eps - thr > R(0) ? eps - thr : R(0);
    else e1 = esc;
    turn(hx, hy, hz, chi, unif<R>(r.w), ox, oy, oz);
    const R sp1 = Fm<R>::sqrt(e1 * (R)(2.0 * QE / ME));
    // the collided part: the marker itself, or with weight splitting a new
    // marker beside the uncollided remainder
    Mk<R> sc = m;
    sc.vx = sp1 * ox; sc.vy = sp1 * oy; sc.vz = sp1 * oz;
    if (split) {
      const R f = PR(P, f_e);
      const U4 sid = draw_cold(m.id, step, CH_CHILD | (2u << 8), C.seed, P.key);
      sc.id = child(sid.x, sid.y);
      sc.w = m.w * f;
      o.e[0].w = m.w * PR(P, g_e);
      o.e[1] = sc;
      o.me = 3u;
    } else {
      o.e[0] = sc;
    }
    ev |= 1u << (kind == 0 ? EV_ELASTIC : (kind == 1 ? EV_EXCIT : EV_IONIZ));
    if (ioniz) {
      // the ejected electron and the ion at the primary's position
      const U4 b = draw_cold(m.id, step, CH_IONBIRTH, C.seed, P.key);
      const U4 cid = draw_cold(m.id, step, CH_CHILD, C.seed, P.key);
      R jx, jy, jz;
      turn(hx, hy, hz, vs_angle(eej, unif<R>(q.y)), unif<R>(q.z), jx, jy, jz);
      const R spj = Fm<R>::sqrt(eej * (R)(2.0 * QE / ME));
      Mk<R> e2 = m;
      e2.vx = spj * jx; e2.vy = spj * jy; e2.vz = spj * jz;
      e2.id = child(cid.x, cid.y);
      e2.w = sc.w;
      Mk<R> i2 = m;
      normals3<R>(b, PR(P, vth_i), i2.vx, i2.vy, i2.vz);
      i2.id = child(cid.z, cid.w);
      i2.w = sc.w;
      if (split) {
        o.e[LaneOut<R, WS>::NE - 1] = e2;
        o.me |= 4u;
      } else {
        o.e[1] = e2;
        o.me |= 2u;
      }
      o.i[0] = i2;
      o.mi = 1u;
    }
  }
}

// Ar+ charge exchange of a candidate: the ion takes a neutral's thermal
// velocity (with weight splitting, a new ion of the fraction f_cx of its
// flux weight does, beside the uncollided remainder).
template <typename R, bool WS>
__device__ void collide_ion(const Ctx<R>& C, IP& P, int inst, uint32_t step,
                            Mk<R>& m, LaneOut<R, WS>& o, uint32_t& ev, uint32_t& err) {
  bool hit = true;  // fixed-event candidates always exchange
  if (!C.fixed) {
    const U4 r = draw(m.id, step, CH_CX, C.seed, P.key);
    const R v2 = m.vx * m.vx + m.vy * m.vy + m.vz * m.vz;
    const R sp1 = Fm<R>::sqrt(v2);
    const R v0 = PR(P, v0);
    const R slow = P.limited ? (sp1 < v0 ? sp1 : v0) : sp1;
    const R nu = PR(P, n_g) * PR(P, sigma_cx) * slow;
    const R numax = PR(P, nu_max_cx);
    if (nu > numax * R(1.000001)) err |= ERR_NU_BOUND;
    hit = unif<R>(r.y) * numax < nu;
  }
  o.i[0] = m;
  o.mi = 1u;
  if (hit) {
    const U4 b = draw_cold(m.id, step, CH_CX | (1u << 8), C.seed, P.key);
    Mk<R> sc = m;
    normals3<R>(b, PR(P, vth_i), sc.vx, sc.vy, sc.vz);
    if (WS && P.f_cx < 1.0) {
      const R f = PR(P, f_cx);
      const U4 sid = draw_cold(m.id, step, CH_CHILD | (2u << 8), C.seed, P.key);
      sc.id = child(sid.x, sid.y);
      sc.w = m.w * f;
      o.i[0].w = m.w * PR(P, g_cx);
      o.i[WS ? 1 : 0] = sc;
      o.mi = 3u;
    } else {
      o.i[0] = sc;
    }
    ev |= 1u << EV_CX;
  }
}

// One marker of a tile: gather at x^n, null-collision draw, flight, walls
// and emission.  A collision candidate sets cand and produces nothing yet;
// otherwise the marker, or the electron its cathode impact emits, becomes
// the lane's output.
template <typename R, int MODE, bool WS>
__device__ __forceinline__ void advance(const Ctx<R>& C, IP& P, int inst, int sp,
                                        uint32_t g, uint32_t step, bool valid, Mk<R>& m,
                                        LaneOut<R, WS>& o, uint32_t& ev, uint32_t& err, bool& cand) {
  if (!valid) return;
  if (MODE == MODE_REFRESH) {
    if (sp == 0) { o.e[0] = m; o.me = 1u; }
    else { o.i[0] = m; o.mi = 1u; }
    return;
  }
  // the null-collision draw does not depend on the field and overlaps the
  // gather
  const R* E = C.E + (size_t)(g % 2u) * C.total_nodes + P.node;
  const R e0 = E[m.cell], e1 = E[m.cell + 1];
  __builtin_amdgcn_sched_barrier(0);  // the gather goes out before the draw
  const U4 rn = draw(m.id, step, sp == 0 ? (uint32_t)CH_COLL : (uint32_t)CH_CX, C.seed, P.key);
  // only the first word is used, at the end of the step; the empty asm
  // keeps the compiler from sinking the ten rounds there, after the flight
  uint32_t rnx = rn.x;
  asm volatile("" : "+v"(rnx));
  const R Ep = e0 + m.off * (e1 - e0);
  const R a = (sp == 0 ? PR(P, qm_e) : PR(P, qm_i)) * Ep;
  const R c2 = m.vy * m.vy + m.vz * m.vz;
  R disp, vx1, tdisp;
  bool turns;
  flight<R>(m.vx, c2, a, PR(P, dt), PR(P, v0), PR(P, inv_v0), P.limited, disp, vx1, turns, tdisp);
  const R inv_dx = PR(P, inv_dx);
  R f = m.off + disp * inv_dx;
  const R fl = m_floor(f);
  int cell = m.cell + (int)fl;
  f -= fl;
  if (f >= R(1)) f = one_below<R>();
  bool out_lo = cell < 0, out_hi = cell >= P.cells;
  if (turns) {
    const R ft = m.off + tdisp * inv_dx;
    const int ct = m.cell + (int)m_floor(ft);
    out_lo = out_lo || ct < 0;
    out_hi = out_hi || ct >= P.cells;
  }
  const bool finite = m_finite(f) && m_finite(vx1);
  if ((C.flags & 4u) && finite) {
    // flux diagnostic (Eq. (12) and the passage after it): the net
    // crossings of the nodes between the cells before and after the flight,
    // an absorbed marker ending below node 0 or above node cells
    const int c0 = m.cell, c1 = out_lo ? -1 : (out_hi ? P.cells : cell);
    int32_t* cr = C.cross + (size_t)sp * C.total_nodes + P.node;
    for (int k = c0 + 1; k <= c1; ++k) atomicAdd(cr + k, 1);
    for (int k = c1 + 1; k <= c0; ++k) atomicAdd(cr + k, -1);
  }
  if (!finite) {
    err |= ERR_NONFINITE;
  } else if (out_lo) {
    ev |= 1u << (sp == 0 ? EV_ABS_E_CATH : EV_ABS_I_CATH);
    if (sp == 1) {
      // ion-induced secondary emission (Sec. IV): an electron at rest at
      // the cathode with probability gamma_se, or with the yield of
      // Eq. (17) at the impact energy; v_x^2 - 2 a x is constant along
      // the flight, so the ion reaches x = 0 with v_x^2 = vx^2 - 2 a x
      const U4 r = draw_cold(m.id, step, CH_SEE, C.seed, P.key);
      const bool see = (C.flags & 2u)
                           ? unif<R>(r.x) < impact_yield<R>(E, PR(P, qm_i), PR(P, dx), m)
                           : (r.x >> 9) < P.t_see;
      if (see) {
        ev |= 1u << EV_SEE;
        Mk<R> e;
        e.cell = 0;
        e.off = R(0);
        e.vx = e.vy = e.vz = R(0);
        e.id = child(r.z, r.w);
        e.w = m.w;  // the ion's flux weight (Sec. III: products carry it)
        o.e[0] = e;
        o.me = 1u;
      }
    }
  } else if (out_hi) {
    ev |= 1u << (sp == 0 ? EV_ABS_E_ANODE : EV_ABS_I_ANODE);
  } else {
    m.cell = cell;
    m.off = f;
    m.vx = vx1;
    // null-collision test: candidates go to the queue
    const uint32_t u = rnx >> 9;
    uint32_t tcand;
    if (C.fixed) tcand = sp == 0 ? P.t_cand_fixed_e : P.t_fixed_cx;
    else tcand = sp == 0 ? P.t_null_e : (P.sigma_cx > 0.0 ? P.t_null_cx : 0u);
    cand = u < tcand;
    if (!cand) {
      if (sp == 0) { o.e[0] = m; o.me = 1u; }
      else { o.i[0] = m; o.mi = 1u; }
    }
  }
}

// The particle kernel reads its argument through the kernel-argument
// segment (constant, invariant memory): the compiler then reloads fields
// with scalar loads instead of keeping them all in scalar registers.
__device__ __forceinline__ const void* kernarg_base() {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_kernarg_segment_ptr();
#else
  return nullptr;
#endif
}

// OCC: waves per SIMD the FP32 kernel is compiled for (its register budget:
// 4 or 5; the LDS of a workgroup allows at most 5 per compute unit), one of
// the launch shapes an autotuner chooses between.  Results do not depend on
// it, only the register allocation does.
template <typename R, int MODE, bool WS, int OCC>
__global__ void __launch_bounds__(BLOCK, sizeof(R) == 4 ? OCC : 1) k_gen(Ctx<R> C_arg) {
  (void)C_arg;
  const Ctx<R>& C = *reinterpret_cast<const Ctx<R>*>(kernarg_base());
  extern __shared__ uint32_t s_prefix[];  // 2 n_inst + 1 tile offsets (dynamic)
  __shared__ unsigned long long s_hist[HWIN];
  __shared__ uint32_t s_gen;
  __shared__ uint32_t s_run[2];
  __shared__ uint32_t s_claim[7];  // pool, its tiles left and when, the claim's offset and
                                   // size, the workgroup's start and tiles taken
  __shared__ uint32_t s_dist[3];   // first tile of the pools, first-run size, workgroups per pool
  __shared__ uint32_t s_evw[NWAVE][NEV];
  __shared__ double s_scan[NWAVE + 1];
  // collision queues (rings), one per wave: candidates of the wave's
  // current (instance, species)
  __shared__ int32_t q_cell[NWAVE][QW];
  __shared__ R q_off[NWAVE][QW], q_vx[NWAVE][QW], q_vy[NWAVE][QW], q_vz[NWAVE][QW];
  __shared__ uint64_t q_id[NWAVE][QW];
  __shared__ R q_w[WS ? NWAVE : 1][WS ? QW : 1];  // flux weights (weight splitting)

  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int nk = 2 * C.n_inst;
  // The tile counts of this thread's positions in all three ring slots (for
  // up to PREPER positions a thread, 256 instances), and both buffer
  // selectors: nothing writes them while this kernel runs, so they go out
  // with the generation's load and are picked once it is known (one memory
  // round trip instead of three before the first claim).
  constexpr int PREPER = 2;
  const int per = (nk + BLOCK - 1) / BLOCK;
  uint32_t pre[3][PREPER];
#pragma unroll
  for (int j = 0; j < PREPER; ++j) {
    const int k = tid * per + j;
#pragma unroll
    for (int s = 0; s < 3; ++s)
      pre[s][j] = per <= PREPER && j < per && k < nk ? *tile_counts(C, (uint32_t)s, k) : 0u;
  }
  const uint32_t bs0 = C.g->bufsel[0], bs1 = C.g->bufsel[1];
  // the generation to advance from: set by the previous tail kernel, and
  // handed to the next one through tail_gen (tail workgroups cannot read
  // cur_gen, which the first of them to finish moves on)
  if (tid == 0) {
    const uint32_t gg = C.g->cur_gen;
    s_gen = gg;
    if (blockIdx.x == 0) C.g->tail_gen = gg;
  }
  if (tid < NWAVE * NEV) s_evw[tid / NEV][tid % NEV] = 0u;
  for (int i = tid; i < HWIN; i += BLOCK) s_hist[i] = 0ull;
  __syncthreads();
  const uint32_t g = s_gen;

  const uint32_t g3 = g % 3u;
  tile_prefix_of(C, s_prefix, s_scan, [&](int j, int k) {
    if (j < PREPER && per <= PREPER) return g3 == 0u ? pre[0][j] : (g3 == 1u ? pre[1][j] : pre[2][j]);
    return *tile_counts(C, g3, k);
  });
  const uint32_t n_tiles = s_prefix[nk];
  const uint32_t bsel = g % 2u ? bs1 : bs0;

  // Work distribution.  Tile costs differ widely (electron tiles against ion
  // tiles, collision rates from instance to instance), so equal shares of
  // tiles leave much of the grid idle while the costliest shares finish.
  // The tiles form NPOOL pools of consecutive tiles, each with a claim
  // counter of the step on a line of its own.  Workgroup b claims runs of
  // consecutive tiles from pool b mod NPOOL, each as large as the pool's
  // unclaimed tiles over twice its share of the grid (at most
  // n_tiles / (2 grid), at least one), so that runs shrink as the step
  // ends, and moves on to the pool with the most tiles
  // left when its pool is exhausted.  Claiming from the start, rather than
  // taking a fixed first share, keeps a workgroup that starts late (when
  // the grid exceeds what stays resident) from ending late.  Runs are
  // contiguous, so that (for markers in cell order) deposits stay inside
  // one LDS window.  A claim goes out at the start of a run's last tile and
  // is read at its end; the first lane of the workgroup keeps the claims in
  // LDS.  With fewer than four tiles per workgroup the claims would cost
  // more than they balance: equal contiguous shares, no claims, as with
  // the static distribution (C.dist == 0), which suits markers in cell
  // order, whose contiguous shares keep their deposits in the window.  The claim
  // logic reads its constants from LDS (s_dist), so that they hold no scalar
  // registers in the tile loop.
  uint32_t run_b, run_e;
  {
    const uint32_t grid = gridDim.x;
    const bool pooled = C.dist && n_tiles >= 4u * grid;
    const uint32_t per = (n_tiles + grid - 1u) / grid;
    run_b = pooled ? 0u : (uint32_t)min((uint64_t)n_tiles, (uint64_t)blockIdx.x * per);
    run_e = pooled ? 0u : min(n_tiles, run_b + per);
    if (tid == 0) {
      const uint32_t home = blockIdx.x % (uint32_t)NPOOL;
      const uint32_t now = (uint32_t)__builtin_amdgcn_s_memrealtime();
      s_dist[0] = pooled ? 0u : n_tiles;              // first tile of the pools
      s_dist[1] = max(1u, n_tiles / (2u * grid));     // largest run
      s_dist[2] = max(1u, grid / (uint32_t)NPOOL);    // workgroups per pool
      s_claim[0] = home;                              // pool
      s_claim[1] = (uint32_t)(((uint64_t)n_tiles * (home + 1u)) / (uint32_t)NPOOL -
                              ((uint64_t)n_tiles * home) / (uint32_t)NPOOL);  // its tiles left
      s_claim[2] = now;                               // as of this time
      s_claim[5] = now;                               // start of the workgroup
      s_claim[6] = 0u;                                // tiles it has taken
    }
  }
  // tiles [pool_lo(p), pool_lo(p + 1)) form pool p
  auto pool_lo = [&](uint32_t p) {
    const uint32_t base = s_dist[0];
    return base + (uint32_t)(((uint64_t)(n_tiles - base) * p) / (uint32_t)NPOOL);
  };
  // thread 0: claim a run from the current pool (its offset in the pool in
  // s_claim[3], its size in s_claim[4]) when there are pools.  The pool's
  // tiles left are estimated from the count at the last claim, less what
  // the pool's workgroups have taken since at this workgroup's own rate
  // (the real-time counter, no memory access).
  auto claim = [&]() {
    if (s_dist[0] >= n_tiles) {
      s_claim[3] = 0u;
      s_claim[4] = 0u;
      return;
    }
    const uint32_t p = s_claim[0], now = (uint32_t)__builtin_amdgcn_s_memrealtime();
    const float rate = (float)s_claim[6] / (float)max(1u, now - s_claim[5]);  // tiles per tick
    const float left =
        (float)s_claim[1] - rate * (float)(now - s_claim[2]) * (float)s_dist[2];
    const uint32_t rem = left > 0.0f ? (uint32_t)left : 0u;
    const uint32_t kk = min(s_dist[1], max(1u, rem / (2u * s_dist[2])));
    s_claim[3] = atomicAdd(&C.g->claim[g % 2u][p][0], kk);
    s_claim[4] = kk;
    s_claim[2] = now;
  };
  // wave 0, at the end of a run: the claimed run into s_run, or, when the
  // claim found its pool exhausted, a claim from the pool with the most
  // tiles left (the lanes read every pool's counter at once), until every
  // pool is exhausted (s_run empty)
  auto resolve = [&]() {
    for (;;) {
      const uint32_t p = s_claim[0], at = s_claim[3], kk = s_claim[4];
      if (kk == 0u) {
        if (lane == 0) s_run[0] = s_run[1] = n_tiles;
        return;
      }
      const uint32_t lo = pool_lo(p), size = pool_lo(p + 1) - lo;
      if (at < size) {
        if (lane == 0) {
          const uint32_t end = min(at + kk, size);
          s_claim[1] = size - end;   // tiles left at the claim
          s_claim[6] += end - at;
          s_run[0] = lo + at;
          s_run[1] = lo + end;
        }
        return;
      }
      unsigned long long key = 0ull;  // tiles left << 8 | pool
      if (lane < NPOOL) {
        const uint32_t c = __hip_atomic_load(&C.g->claim[g % 2u][lane][0], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t sz = pool_lo((uint32_t)lane + 1u) - pool_lo((uint32_t)lane);
        key = (unsigned long long)(sz > c ? sz - c : 0u) << 8 | (unsigned long long)lane;
      }
#pragma unroll
      for (int d = 1; d < NPOOL; d <<= 1) {
        const unsigned long long o = __shfl_xor(key, d);
        key = o > key ? o : key;
      }
      if ((key >> 8) == 0ull) {
        if (lane == 0) s_run[0] = s_run[1] = n_tiles;
        return;
      }
      if (lane == 0) {
        s_claim[0] = (uint32_t)(key & 0xffu);
        s_claim[1] = (uint32_t)(key >> 8);
        s_claim[2] = (uint32_t)__builtin_amdgcn_s_memrealtime();
        claim();
      }
    }
  };
  DepWin win{-1, 0, 0};
  Work W{-1, -1, 0, 0u, POP_NONE, 0, 0, 0u};
  uint32_t q_head = 0, q_count = 0;  // uniform over the wave
  uint32_t* evw = s_evw[wv];          // event counts of this wave since the last flush
  const unsigned long long lt = (1ull << lane) - 1ull;

  // collide up to WAVE queued candidates and emit the results
  auto run_queue = [&](uint32_t n) {
    LaneOut<R, WS> o;
    o.me = o.mi = 0u;
    uint32_t ev = 0, err = 0;
    // the batch's output partition, ahead of the collisions (see the tile's)
    next_output(W, param(C.ip, W.inst));
    // the appends of other lanes land before these reads (one wave: LDS
    // operations complete in order; the fence keeps the compiler's order)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if ((uint32_t)lane < n) {
      const uint32_t s = ring(q_head, (uint32_t)lane);
      Mk<R> m;
      m.cell = q_cell[wv][s];
      m.off = q_off[wv][s];
      m.vx = q_vx[wv][s];
      m.vy = q_vy[wv][s];
      m.vz = q_vz[wv][s];
      m.id = q_id[wv][s];
      m.w = WS ? q_w[WS ? wv : 0][WS ? s : 0] : R(1);
      IP& P = param(C.ip, W.inst);
      if (W.sp == 0) collide_electron(C, P, W.inst, W.step, m, o, ev, err);
      else collide_ion(C, P, W.inst, W.step, m, o, ev, err);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // reads before reuse
    q_head = ring(q_head, n);
    q_count -= n;
    emit<R, MODE, true, WS>(C, W, win, s_hist, o, ev, err, g, bsel, evw);
  };
  // append marker m to the queue at offset off (< QW) past its head
  auto q_put = [&](const Mk<R>& m, uint32_t off) {
    const uint32_t s = ring(q_head, off);
    q_cell[wv][s] = m.cell;
    q_off[wv][s] = m.off;
    q_vx[wv][s] = m.vx;
    q_vy[wv][s] = m.vy;
    q_vz[wv][s] = m.vz;
    q_id[wv][s] = m.id;
    if (WS) q_w[WS ? wv : 0][WS ? s : 0] = m.w;
  };

  // One tile at a time, one marker per lane: a single marker's registers
  // leave room for five waves per SIMD, which hide more of the load and
  // atomic latency than two markers per lane at four waves did.
  TileCursor cur;
  for (;;) {
  if (tid == 0 && run_b == run_e) claim();  // nothing in this run: claim at once
  cur.kc = -1;  // a run can start anywhere: find its pair by bisection
  for (uint32_t t = run_b; t < run_e; ++t) {
    if (tid == 0 && t + 1u == run_e) claim();
    cur.locate(s_prefix, nk, t);
    int inst, sp;
    pair_at(cur.kc, C.n_inst, inst, sp);
    IP& P = param(C.ip, inst);
    int part;
    uint32_t first;
    cur.place(t, P.parts, part, first);
    const uint32_t n = count_in(C.counts, C.n_inst, g, inst, sp, part);
    const uint32_t idx = first + (uint32_t)tid;
    const int64_t pb = P.seg + (int64_t)part * P.cap_p;
    if (inst != W.inst || sp != W.sp) {
      // new (instance, species): collide what is queued for the old one
      while (q_count > 0) run_queue(q_count < (uint32_t)WAVE ? q_count : (uint32_t)WAVE);
      // the state of generation g: written by the last tail kernel, read
      // only while this kernel runs (scalar loads)
      using CS = const __attribute__((address_space(4))) InstState;
      CS& S0 = ((CS*)C.st)[(g % 2u) * C.n_inst + inst];
      {
        // flush the old deposit window and anchor the new one: for
        // cell-sorted markers a quarter window below the tile's first
        // marker (a run's markers follow the cells); otherwise the tail
        // kernel's choice, where the species deposited most in the last
        // step it chose on (every ANCHOR_PERIOD steps), which a marker of
        // any tile is likely to hit
        if (win.inst >= 0) dep_flush(C, s_hist, win, s_evw);
        int anchor = S0.anchor[sp];
        if (C.sorted) {
          const int c0 = first < n ? gbuf(C, bsel, sp).cell(pb + first) : 0;
          anchor = c0 - HWIN / 4;
        }
        const int top = P.cells + 1 - HWIN;
        anchor = anchor > top ? top : anchor;
        win.anchor = anchor < 0 ? 0 : anchor;
        win.inst = inst;
        win.sp = sp;
      }
      W.inst = inst;
      W.sp = sp;
      W.step = S0.step;
      W.pop = MODE == MODE_STEP ? S0.popmode : POP_NONE;
      if (WS) W.dshift = MODE == MODE_STEP ? S0.dshift : C.dep_shift;
    }
    const Part<R> in = part_of(gbuf(C, bsel, sp), pb);

    // loads inside the partition need not wait for its count
    Mk<R> m;
    if (idx < (uint32_t)P.cap_p) {
      const SlotOff<R> q(idx);
      m.cell = in.cell(q);
      m.off = in.off(q);
      m.vx = in.vx(q);
      m.vy = in.vy(q);
      m.vz = in.vz(q);
      m.id = in.id(q);
      m.w = WS ? C.wt[bsel][sp][pb + idx] : R(1);
    }
    // this tile's output partition: its hash runs while the loads are in
    // flight rather than between the flight and the reservation
    next_output(W, P);
    LaneOut<R, WS> o;
    o.me = o.mi = 0u;
    uint32_t ev = 0, err = 0;
    bool cand = false;
    advance<R, MODE, WS>(C, P, inst, sp, g, W.step, idx < n, m, o, ev, err, cand);
    if (MODE == MODE_STEP) {
      // append the wave's candidates to its queue (fewer than WAVE wait)
      const unsigned long long b = __ballot(cand);
      if (cand) q_put(m, q_count + (uint32_t)__popcll(b & lt));
      q_count += (uint32_t)__popcll(b);
    }
    emit<R, MODE, false, WS>(C, W, win, s_hist, o, ev, err, g, bsel, evw);
    while (MODE == MODE_STEP && q_count >= (uint32_t)WAVE) run_queue((uint32_t)WAVE);
  }
  if (wv == 0) resolve();
  __syncthreads();
  // the same for every lane: kept in scalar registers
  run_b = __builtin_amdgcn_readfirstlane(s_run[0]);
  run_e = __builtin_amdgcn_readfirstlane(s_run[1]);
  __syncthreads();  // read before thread 0 writes the next run
  if (run_b >= run_e) break;
  }
  while (q_count > 0) run_queue(q_count < (uint32_t)WAVE ? q_count : (uint32_t)WAVE);
  if (win.inst >= 0) dep_flush(C, s_hist, win, s_evw);
}

// ---------------------------------------------------------------- cell sort
// Counting sort of every (instance, species) by cell, between two steps.
// It moves markers without changing them, and nothing in a step depends on
// the order of the markers (random draws are keyed by marker id and step,
// deposits are exact fixed-point sums), so a sorted run equals an unsorted
// one bit for bit.  Markers go to the other buffer in cell order: partition
// p of a pair with n markers takes ranks [p q, (p + 1) q), q = ceil(n / P),
// so the partition-ordered tiles of the next step follow the cells.  Within
// a cell the order is that of the atomic cursors (the sort is not stable).
//
// Dynamic LDS of the three tile-walking kernels: the tile offsets, then one
// (count) or two (scatter) arrays of max_cells words.

// generation and buffer of the state the sort works on (set by the tail)
template <typename R>
__device__ __forceinline__ void sort_state(const Ctx<R>& C, uint32_t& g, uint32_t& bsel) {
  g = C.g->cur_gen;
  bsel = C.g->bufsel[g % 2u];
}

template <typename R>
__device__ __forceinline__ uint32_t pair_count(const Ctx<R>& C, uint32_t g, int inst, int sp) {
  uint32_t n = 0;
  for (int p = 0; p < param(C.ip, inst).parts; ++p) n += C.counts[cidx(C.n_inst, g % 3u, inst, sp, p)];
  return n;
}

// 1: per-cell marker counts of every pair, in LDS per workgroup and pair
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_sort_count(Ctx<R> C) {
  extern __shared__ uint32_t s_dyn[];
  __shared__ double s_scan[NWAVE + 1];
  const int nk = 2 * C.n_inst, tid = threadIdx.x;
  uint32_t* s_prefix = s_dyn;
  uint32_t* s_hist = s_dyn + ((nk + 1 + 3) & ~3);
  uint32_t g, bsel;
  sort_state(C, g, bsel);
  for (int i = tid; i < C.max_cells; i += BLOCK) s_hist[i] = 0u;
  tile_prefix(C, g, s_prefix, s_scan);
  const uint32_t n_tiles = s_prefix[nk];
  const uint32_t per = (n_tiles + (uint32_t)C.grid - 1) / (uint32_t)C.grid;
  const uint32_t t_begin = blockIdx.x * per, t_end = min(n_tiles, t_begin + per);
  TileCursor cur;
  int k_open = -1;
  auto flush = [&]() {
    __syncthreads();
    int oi, os;
    pair_at(k_open, C.n_inst, oi, os);
    IP& P = param(C.ip, oi);
    uint32_t* dst = C.sort_hist + (size_t)os * C.total_nodes + P.node;
    for (int c = tid; c < P.cells; c += BLOCK) {
      const uint32_t v = s_hist[c];
      if (v) {
        atomicAdd(dst + c, v);
        s_hist[c] = 0u;
      }
    }
    __syncthreads();
  };
  for (uint32_t t = t_begin; t < t_end; ++t) {
    cur.locate(s_prefix, nk, t);
    if (cur.kc != k_open) {
      if (k_open >= 0) flush();
      k_open = cur.kc;
    }
    int inst, sp;
    pair_at(cur.kc, C.n_inst, inst, sp);
    IP& P = param(C.ip, inst);
    int part;
    uint32_t first;
    cur.place(t, P.parts, part, first);
    const uint32_t idx = first + (uint32_t)tid;
    if (idx < C.counts[cidx(C.n_inst, g % 3u, inst, sp, part)])
      atomicAdd(&s_hist[gbuf(C, bsel, sp).cell(P.seg + (int64_t)part * P.cap_p + idx)], 1u);
  }
  if (k_open >= 0) flush();
}

// 2: one workgroup per pair: exclusive prefix sums of the counts become the
// cursors of the scatter; the counts are cleared for the next sort
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_sort_scan(Ctx<R> C) {
  __shared__ double s_scan[NWAVE + 1];
  const int k = blockIdx.x, inst = k >> 1, sp = k & 1, tid = threadIdx.x;
  IP& P = param(C.ip, inst);
  uint32_t* hist = C.sort_hist + (size_t)sp * C.total_nodes + P.node;
  uint32_t* cursor = C.sort_cur + (size_t)sp * C.total_nodes + P.node;
  const int chunk = (P.cells + BLOCK - 1) / BLOCK;
  const int c0 = tid * chunk, c1 = min(P.cells, c0 + chunk);
  uint32_t loc = 0;
  for (int c = c0; c < c1; ++c) loc += hist[c];
  double v1[1] = {(double)loc}, ex1[1], tot1[1];
  block_scan<1>(v1, ex1, tot1, s_scan);
  uint32_t run = (uint32_t)ex1[0];
  for (int c = c0; c < c1; ++c) {
    const uint32_t v = hist[c];
    cursor[c] = run;
    run += v;
    hist[c] = 0u;
  }
}

// 3: each workgroup counts its markers of a pair per cell, reserves one
// range per cell on the pair's cursors, then places every marker at
// rank = reserved start + local order, in the other buffer
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_sort_scatter(Ctx<R> C) {
  extern __shared__ uint32_t s_dyn[];
  __shared__ double s_scan[NWAVE + 1];
  const int nk = 2 * C.n_inst, tid = threadIdx.x;
  uint32_t* s_prefix = s_dyn;
  uint32_t* s_cnt = s_dyn + ((nk + 1 + 3) & ~3);
  uint32_t* s_base = s_cnt + C.max_cells;
  uint32_t g, bsel;
  sort_state(C, g, bsel);
  for (int i = tid; i < C.max_cells; i += BLOCK) s_cnt[i] = 0u;
  tile_prefix(C, g, s_prefix, s_scan);
  const uint32_t n_tiles = s_prefix[nk];
  const uint32_t per = (n_tiles + (uint32_t)C.grid - 1) / (uint32_t)C.grid;
  const uint32_t t_begin = blockIdx.x * per, t_end = min(n_tiles, t_begin + per);
  // the workgroup's tiles, one pair at a time
  uint32_t t = t_begin;
  while (t < t_end) {
    TileCursor cur;
    cur.locate(s_prefix, nk, t);
    int inst, sp;
    pair_at(cur.kc, C.n_inst, inst, sp);
    const uint32_t run_end = min(t_end, cur.kend);
    IP& P = param(C.ip, inst);
    const Soa<R> in = gbuf(C, bsel, sp), out = gbuf(C, 1u - bsel, sp);
    const uint32_t n = pair_count(C, g, inst, sp);
    const uint32_t q = (n + (uint32_t)P.parts - 1) / (uint32_t)P.parts;
    // pass A: counts per cell
    for (uint32_t u = t; u < run_end; ++u) {
      int part;
      uint32_t first;
      cur.place(u, P.parts, part, first);
      const uint32_t idx = first + (uint32_t)tid;
      if (idx < C.counts[cidx(C.n_inst, g % 3u, inst, sp, part)])
        atomicAdd(&s_cnt[in.cell(P.seg + (int64_t)part * P.cap_p + idx)], 1u);
    }
    __syncthreads();
    uint32_t* cursor = C.sort_cur + (size_t)sp * C.total_nodes + P.node;
    for (int c = tid; c < P.cells; c += BLOCK) {
      const uint32_t v = s_cnt[c];
      if (v) s_base[c] = atomicAdd(cursor + c, v);
      s_cnt[c] = 0u;
    }
    __syncthreads();
    // pass B: place
    for (uint32_t u = t; u < run_end; ++u) {
      int part;
      uint32_t first;
      cur.place(u, P.parts, part, first);
      const uint32_t idx = first + (uint32_t)tid;
      if (idx < C.counts[cidx(C.n_inst, g % 3u, inst, sp, part)]) {
        const int64_t s = P.seg + (int64_t)part * P.cap_p + idx;
        const int32_t cell = in.cell(s);
        const uint32_t rank = s_base[cell] + atomicAdd(&s_cnt[cell], 1u);
        const int64_t d = P.seg + (int64_t)(rank / q) * P.cap_p + rank % q;
        out.cell(d) = cell;
        out.off(d) = in.off(s);
        out.vx(d) = in.vx(s);
        out.vy(d) = in.vy(s);
        out.vz(d) = in.vz(s);
        out.id(d) = in.id(s);
        if (C.split) C.wt[1u - bsel][sp][d] = C.wt[bsel][sp][s];
      }
    }
    __syncthreads();
    for (int c = tid; c < P.cells; c += BLOCK) s_cnt[c] = 0u;
    __syncthreads();
    t = run_end;
  }
}

// 4: one thread per pair: the new partition counts, then the buffer switch
template <typename R>
__global__ void k_sort_commit(Ctx<R> C) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t g, bsel;
  sort_state(C, g, bsel);
  if (k < 2 * C.n_inst) {
    const int inst = k >> 1, sp = k & 1;
    IP& P = param(C.ip, inst);
    const uint32_t n = pair_count(C, g, inst, sp);
    const uint32_t q = (n + (uint32_t)P.parts - 1) / (uint32_t)P.parts;
    for (int p = 0; p < P.parts; ++p) {
      const uint32_t lo = (uint32_t)p * q;
      C.counts[cidx(C.n_inst, g % 3u, inst, sp, p)] = lo < n ? min(q, n - lo) : 0u;
    }
    C.tiles[(size_t)(g % 3u) * 2 * C.n_inst + k] = pair_tiles(min(q, n), P.parts);
  }
  // every thread has read the counts above before one of them switches the
  // buffer: the switch is made by a second launch (see launch_sort)
}

template <typename R>
__global__ void k_sort_switch(Ctx<R> C) {
  uint32_t g, bsel;
  sort_state(C, g, bsel);
  C.g->bufsel[g % 2u] = 1u - bsel;
}

// ---------------------------------------------------------------- seeding
template <typename R>
__global__ void k_seed(Ctx<R> C, int inst, int mode, int64_t n, double sigma_v, uint32_t bsel) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  IP& P = param(C.ip, inst);
  const Soa<R> o = gbuf(C, bsel, 0);
  // seed k goes to partition k mod P, slot k / P
  const int64_t s = P.seg + (k % P.parts) * P.cap_p + k / P.parts;
  o.id(s) = (uint64_t)k;
  o.cell(s) = 0;
  if (C.split) C.wt[bsel][0][s] = R(1);
  if (mode == 2) {
    const U4 r0 = draw((uint64_t)k, 0u, CH_SEED, C.seed, P.key);
    const U4 r1 = draw((uint64_t)k, 0u, CH_SEED | (1u << 8), C.seed, P.key);
    o.off(s) = unif<R>(r0.x);
    R a, b, c;
    normals3<R>(r1, (R)sigma_v, a, b, c);
    o.vx(s) = a;
    o.vy(s) = b;
    o.vz(s) = c;
  } else {
    o.off(s) = R(0);
    o.vx(s) = R(0);
    o.vy(s) = R(0);
    o.vz(s) = R(0);
  }
}

__global__ void k_philox_test(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n,
                              uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const U4 r = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

// ---------------------------------------------------------------- launchers
template <typename R>
hipError_t launch_particles(const Ctx<R>& C, int mode, hipStream_t s) {
  const dim3 g(C.grid), b(BLOCK);
  if (C.split) {
    if (mode == MODE_STEP)
      hipLaunchKernelGGL((k_gen<R, MODE_STEP, true, 5>), g, b, C.gen_lds, s, C);
    else
      hipLaunchKernelGGL((k_gen<R, MODE_REFRESH, true, 5>), g, b, C.gen_lds, s, C);
  } else if (mode != MODE_STEP) {
    hipLaunchKernelGGL((k_gen<R, MODE_REFRESH, false, 5>), g, b, C.gen_lds, s, C);
  } else if (sizeof(R) == 4 && C.occ == 4) {
    hipLaunchKernelGGL((k_gen<R, MODE_STEP, false, 4>), g, b, C.gen_lds, s, C);
  } else {
    hipLaunchKernelGGL((k_gen<R, MODE_STEP, false, 5>), g, b, C.gen_lds, s, C);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_tail(const Ctx<R>& C, int mode, hipStream_t s) {
  if (mode == MODE_STEP)
    hipLaunchKernelGGL((k_tail<R, MODE_STEP>), dim3(C.n_inst), dim3(TBLOCK), C.tail_lds, s, C);
  else
    hipLaunchKernelGGL((k_tail<R, MODE_REFRESH>), dim3(C.n_inst), dim3(TBLOCK), C.tail_lds, s, C);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_sort(const Ctx<R>& C, hipStream_t s) {
  hipLaunchKernelGGL((k_sort_count<R>), dim3(C.grid), dim3(BLOCK), C.sort_lds1, s, C);
  hipLaunchKernelGGL((k_sort_scan<R>), dim3(2 * C.n_inst), dim3(BLOCK), 0, s, C);
  hipLaunchKernelGGL((k_sort_scatter<R>), dim3(C.grid), dim3(BLOCK), C.sort_lds2, s, C);
  hipLaunchKernelGGL((k_sort_commit<R>), dim3((2 * C.n_inst + BLOCK - 1) / BLOCK), dim3(BLOCK), 0,
                     s, C);
  hipLaunchKernelGGL((k_sort_switch<R>), dim3(1), dim3(1), 0, s, C);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_seed(const Ctx<R>& C, int inst, int mode, int64_t n, double sigma_v,
                       uint32_t bsel, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL((k_seed<R>), dim3((unsigned)blocks), dim3(BLOCK), 0, s, C, inst, mode, n,
                     sigma_v, bsel);
  return hipGetLastError();
}

// resident particle-kernel workgroups per compute unit for the kernel that
// launch_particles picks for (split, occ)
template <typename R>
hipError_t occupancy_gen(int* blocks_per_cu, size_t dyn_lds, bool split, int occ) {
  if (split)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_gen<R, MODE_STEP, true, 5>,
                                                        BLOCK, dyn_lds);
  if (sizeof(R) == 4 && occ == 4)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_gen<R, MODE_STEP, false, 4>,
                                                        BLOCK, dyn_lds);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_gen<R, MODE_STEP, false, 5>,
                                                      BLOCK, dyn_lds);
}

template hipError_t launch_particles<float>(const Ctx<float>&, int, hipStream_t);
template hipError_t launch_particles<double>(const Ctx<double>&, int, hipStream_t);
template hipError_t launch_tail<float>(const Ctx<float>&, int, hipStream_t);
template hipError_t launch_sort<float>(const Ctx<float>&, hipStream_t);
template hipError_t launch_sort<double>(const Ctx<double>&, hipStream_t);
template hipError_t launch_tail<double>(const Ctx<double>&, int, hipStream_t);
template hipError_t launch_seed<float>(const Ctx<float>&, int, int, int64_t, double, uint32_t,
                                       hipStream_t);
template hipError_t launch_seed<double>(const Ctx<double>&, int, int, int64_t, double, uint32_t,
                                        hipStream_t);
template hipError_t occupancy_gen<float>(int*, size_t, bool, int);
template hipError_t occupancy_gen<double>(int*, size_t, bool, int);

hipError_t launch_philox_test(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n,
                              uint32_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL(k_philox_test, dim3((unsigned)blocks), dim3(BLOCK), 0, s, ctr, k0, k1, n,
                     out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- static workspace
// Workspace of the handles made by slpic_create_static, for callers that
// cannot allocate device memory: a file-scope device array, which the code
// object holds on every device it is loaded on until the process ends.  Host
// code never passes the array's name to a launch or a copy (on the host it
// is only a stand-in for the symbol): each device's address of it comes from
// hipGetSymbolAddress, looked up once per device with that device current and
// kept here.
static __device__ __align__(256) char scratch[STATIC_WS_BYTES];

hipError_t static_workspace(int dev, char** ptr) {
  static std::mutex mu;
  static char* addr[MAX_DEVICES] = {};
  if (dev < 0 || dev >= MAX_DEVICES || !ptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev) return hipErrorInvalidDevice;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || ((uintptr_t)p & 255)) return hipErrorInvalidSymbol;
    addr[dev] = static_cast<char*>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace slpic
