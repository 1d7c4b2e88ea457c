// af_device.h -- device-side building blocks of the Active Flux MHD stage
// (gfx950).  Physics of Section 1 and eq. (cf), the LLF flux of eq.
// (2d_llf_flux) with the Lemma's viscosity (Section 3.1), the limiters of
// Sections 3.2-3.3, boundary index maps.  Included by the kernels only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace afm {

constexpr int NV = 8;
constexpr double EPS_FLOOR = 1e-13;   // lower bounds for rho and p (Sections 3.2, 3.3)
constexpr double LAMBDA_REG = 1e-12;  // regulariser of the density box (Section 3.2)
constexpr double SHRINK = 1e-8;       // round-off fallback step 2^m 1e-8, m = 0..9

// Problem geometry, passed by value to every kernel.
struct Geo {
  int nx, ny, nxp, nyp, bcx, bcy;  // bc: 0 periodic, 1 outflow
  double dx, dy, rdx, rdy, gamma, gm1, kappa, cfl;
  long sc, sx, sy, sv;             // elements per component plane of each DoF set
};

struct CState {
  const double* __restrict__ a;
  const double* __restrict__ x;
  const double* __restrict__ y;
  const double* __restrict__ v;
};
struct MState {
  double* __restrict__ a;
  double* __restrict__ x;
  double* __restrict__ y;
  double* __restrict__ v;
};

// Device counters (integer atomics only; min_theta as the bit pattern of a
// non-negative double, whose integer order is the numeric order).
struct Counters {
  unsigned long long n_llf_not_admissible, n_newton, newton_iters_max, n_fallback, n_not_admissible,
      n_theta_active, n_point_limited, n_centre_limited, n_source_limited, min_theta_bits;
};

// --------------------------------------------------------------- boundaries
// Periodic wrap, or outflow as an even mirror: cells mirror about the
// boundary face, nodes about the boundary node.  |overshoot| <= n.
__device__ __forceinline__ int map_cell(int i, int n, int bc) {
  if (i < 0) return bc ? -1 - i : i + n;
  if (i >= n) return bc ? 2 * n - 1 - i : i - n;
  return i;
}
__device__ __forceinline__ int map_node(int k, int n, int bc) {
  if (k < 0) return bc ? -k : k + n;
  if (bc) return k > n ? 2 * n - k : k;
  return k >= n ? k - n : k;
}

__device__ __forceinline__ void load8(const double* __restrict__ base, long plane, long off, double u[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) u[c] = base[c * plane + off];
}
__device__ __forceinline__ void ldA(const Geo& g, const double* a, int i, int j, double u[NV]) {
  load8(a, g.sc, (long)map_cell(j, g.ny, g.bcy) * g.nx + map_cell(i, g.nx, g.bcx), u);
}
__device__ __forceinline__ void ldX(const Geo& g, const double* x, int k, int j, double u[NV]) {
  load8(x, g.sx, (long)map_cell(j, g.ny, g.bcy) * g.nxp + map_node(k, g.nx, g.bcx), u);
}
__device__ __forceinline__ void ldY(const Geo& g, const double* y, int i, int l, double u[NV]) {
  load8(y, g.sy, (long)map_node(l, g.ny, g.bcy) * g.nx + map_cell(i, g.nx, g.bcx), u);
}
__device__ __forceinline__ void ldV(const Geo& g, const double* v, int k, int l, double u[NV]) {
  load8(v, g.sv, (long)map_node(l, g.ny, g.bcy) * g.nxp + map_node(k, g.nx, g.bcx), u);
}

// ------------------------------------------------------------------ physics
// p = (gamma-1)(E - |m|^2/(2 rho) - |B|^2/2), summed left to right without
// fused multiply-adds and with an IEEE division.  Every positivity limiter
// takes its coefficients and its decisions (in G or not) from this form, so
// that on identical inputs they are the reference's bit for bit: where the
// variables' scales differ a lot these decisions are made by round-off.
__device__ __forceinline__ double pressure(const double U[NV], double gm1) {
#pragma clang fp contract(off)
  const double m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
  const double b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  return gm1 * (U[7] - 0.5 * m2 / U[0] - 0.5 * b2);
}
// U in G: rho > 0 and p > 0 (Section 3), in the form above.
__device__ __forceinline__ bool in_G(const double U[NV], double gm1) {
  return U[0] > 0.0 && pressure(U, gm1) > 0.0;
}
// rho p / (gamma-1) = rho E - |m|^2/2 - rho |B|^2/2: for rho > 0 it has the
// sign of p and p >= eps  <=>  (gamma-1) * this >= rho * eps.  The fast
// tests that no limiter needs to act, and the counters, use this
// division-free form; a limiter that may act recomputes with pressure().
__device__ __forceinline__ double rho_p(const double U[NV]) {
  const double m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
  const double b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  return U[0] * (U[7] - 0.5 * b2) - 0.5 * m2;
}
__device__ __forceinline__ bool in_G_fast(const double U[NV]) {
  return U[0] > 0.0 && rho_p(U) > 0.0;
}
// p(U) >= eps for rho > 0
__device__ __forceinline__ bool p_at_least(const double U[NV], double eps, double gm1) {
  return gm1 * rho_p(U) >= U[0] * eps;
}

// ------------------------------------------------------ compute precision
// The bulk arithmetic (fluxes, wave speeds, FVS and LLF sums, the shock
// sensor, the source sums) runs in R: double for the FP64 stage, float for
// the FP32-bulk stage.  Storage, pressure recovery, the centre value, every
// stage accumulation U + dt RHS and every limiter decision stay FP64.
template <class R> struct IsF32 { static constexpr bool value = false; };
template <> struct IsF32<float> { static constexpr bool value = true; };

// Reciprocal and square root of the flux evaluations and the LLF viscosity.
// FP64: the hardware approximations (relative error up to 2^-23) refined by
// Newton steps -- two for the reciprocal; one for the reciprocal square
// root, then one correction of sqrt(x) = x / sqrt(x) itself, which squares
// the remaining ~2e-14 (about one ulp instead of correctly rounded, with
// much shorter dependency chains than the library sequences); arguments are
// positive or zero (sqrt(0) = 0), never denormal in practice.
// FP32: the hardware's one-ulp instructions.  Pressures, the sensor, the
// limiters and their roots use exact division and sqrt.
template <class R> __device__ __forceinline__ R rcp_r(R x);
template <> __device__ __forceinline__ double rcp_r<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
template <> __device__ __forceinline__ float rcp_r<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <class R> __device__ __forceinline__ R sqrt_r(R x);
template <> __device__ __forceinline__ double sqrt_r<double>(double x) {
  double r = __builtin_amdgcn_rsq(x);  // 1/sqrt(x)
  const double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  double q = x * r;                    // sqrt(x), then one correction
  q = fma(fma(-q, q, x), 0.5 * r, q);
  return x > 0.0 ? q : 0.0;
}
template <> __device__ __forceinline__ float sqrt_r<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <class R> __device__ __forceinline__ R exp_r(R x) { return exp(x); }
template <> __device__ __forceinline__ float exp_r<float>(float x) { return __expf(x); }

// What the directional stencils need from one state: the flux in the
// direction, its spectral radius |v_n| + c_f, c_f, v_n and sqrt(rho).
template <class R>
struct DirEvalT {
  R F[NV];
  R sr, cf, vn, sq;
};
using DirEval = DirEvalT<double>;

// Velocity, |B|^2 and pressure of a state.  FP64 as written; for the
// FP32-bulk stage the cancellation-prone part rho p/(gamma-1) = rho E -
// |m|^2/2 - rho |B|^2/2 is formed in FP64 and only the final scaling by
// 1/rho is FP32.
template <class R>
__device__ __forceinline__ void prim_r(const double U[NV], double gm1, R& ri, R& v1, R& v2, R& v3, R& b2, R& p) {
  if constexpr (IsF32<R>::value) {
    const double b2d = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
    const double rp = U[0] * (U[7] - 0.5 * b2d) - 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]);
    ri = rcp_r((float)U[0]);
    v1 = (float)U[1] * ri;
    v2 = (float)U[2] * ri;
    v3 = (float)U[3] * ri;
    b2 = (float)b2d;
    p = (float)(gm1 * rp) * ri;
  } else {
    ri = rcp_r(U[0]);
    v1 = U[1] * ri;
    v2 = U[2] * ri;
    v3 = U[3] * ri;
    b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
    p = gm1 * (U[7] - 0.5 * (U[1] * v1 + U[2] * v2 + U[3] * v3) - 0.5 * b2);
  }
}

// Flux F_n = v_n U + p_t (e_{m_n} + v_n e_E) - B_n (0, B, v, v.B): the
// physical flux of Section 1 regrouped (transport, total pressure, tension).
template <class R>
__device__ __forceinline__ void flux_from(const double U[NV], int dir, R v1, R v2, R v3, R pt, R F[NV]) {
  const R B1 = (R)U[4], B2 = (R)U[5], B3 = (R)U[6];
  const R vB = v1 * B1 + v2 * B2 + v3 * B3;
  const R vn = dir ? v2 : v1;
  const R Bn = dir ? B2 : B1;
  F[0] = (R)U[0] * vn;
  F[1] = vn * (R)U[1] - Bn * B1 + (dir ? R(0) : pt);
  F[2] = vn * (R)U[2] - Bn * B2 + (dir ? pt : R(0));
  F[3] = vn * (R)U[3] - Bn * B3;
  F[4] = dir ? (vn * B1 - Bn * v1) : R(0);
  F[5] = dir ? R(0) : (vn * B2 - Bn * v2);
  F[6] = vn * B3 - Bn * v3;
  F[7] = ((R)U[7] + pt) * vn - Bn * vB;
}

template <class R>
__device__ __forceinline__ void eval_dir(const double U[NV], const Geo& g, int dir, DirEvalT<R>& e) {
  R ri, v1, v2, v3, b2, p;
  prim_r<R>(U, g.gm1, ri, v1, v2, v3, b2, p);
  const R pt = p + R(0.5) * b2;
  flux_from<R>(U, dir, v1, v2, v3, pt, e.F);
  const R vn = dir ? v2 : v1;
  const R Bn = dir ? (R)U[5] : (R)U[4];
  // fast magnetosonic speed, eq. (cf)
  const R c2 = (R)g.gamma * p * ri;
  const R s = c2 + b2 * ri;
  R disc = s * s - R(4) * c2 * Bn * Bn * ri;
  disc = disc > R(0) ? disc : R(0);
  e.cf = sqrt_r(R(0.5) * (s + sqrt_r(disc)));
  e.vn = vn;
  e.sr = fabs(vn) + e.cf;
  e.sq = sqrt_r((R)U[0]);
}

// Flux only (central differences and Simpson fluxes need no wave speed).
template <class R>
__device__ __forceinline__ void flux_dir(const double U[NV], double gm1, int dir, R F[NV]) {
  R ri, v1, v2, v3, b2, p;
  prim_r<R>(U, gm1, ri, v1, v2, v3, b2, p);
  flux_from<R>(U, dir, v1, v2, v3, p + R(0.5) * b2, F);
}

// Godunov-Powell vector Psi = (0, B, v, v.B), eq. (gp_src).
template <class R, class S>
__device__ __forceinline__ void psi(const S U[NV], R P[NV]) {
  const R ri = rcp_r((R)U[0]);
  const R v1 = (R)U[1] * ri, v2 = (R)U[2] * ri, v3 = (R)U[3] * ri;
  P[0] = R(0);
  P[1] = (R)U[4];
  P[2] = (R)U[5];
  P[3] = (R)U[6];
  P[4] = v1;
  P[5] = v2;
  P[6] = v3;
  P[7] = v1 * (R)U[4] + v2 * (R)U[5] + v3 * (R)U[6];
}

// LLF viscosity of the Lemma, taken with equality: max of the two spectral
// radii and of alpha_*(U,Ut), alpha_*(Ut,U); the latter two share all terms
// but |v_n|, so their maximum uses max(|v_a|, |v_b|, |Roe-type average|).
template <class R, class S>
__device__ __forceinline__ R alpha_llf(const DirEvalT<R>& a, const DirEvalT<R>& b, const S Ua[NV], const S Ub[NV]) {
  const R inv = rcp_r(a.sq + b.sq);
  const R roe = fabs(a.sq * a.vn + b.sq * b.vn) * inv;
  const R d1 = (R)(Ua[4] - Ub[4]), d2 = (R)(Ua[5] - Ub[5]), d3 = (R)(Ua[6] - Ub[6]);
  const R jump = sqrt_r(d1 * d1 + d2 * d2 + d3 * d3) * inv;
  const R al = (fmax(fmax(fabs(a.vn), fabs(b.vn)), roe) + fmax(a.cf, b.cf)) + jump;
  return fmax(al, fmax(a.sr, b.sr));
}

// -------------------------------------------------------------- counters
__device__ __forceinline__ void count(unsigned long long* c) { atomicAdd(c, 1ull); }
__device__ __forceinline__ void count_max(unsigned long long* c, unsigned long long v) { atomicMax(c, v); }
__device__ __forceinline__ void count_min_theta(Counters* cn, double t) {
  atomicMin(&cn->min_theta_bits, (unsigned long long)__double_as_longlong(t));
}

// ------------------------------------------------------------- limiters
// Round-off fallback (closing remark of Section 4): when round-off leaves a
// blended state outside G (rho > 0, p > 0), shrink its coefficient by
// 2^m 1e-8 (m = 0..9, each from the original value); 0 if none passes.
template <class Make>
__device__ double shrink_into_G(double theta, double gm1, Make make) {
#pragma clang fp contract(off)
  double W[NV];
  for (int m = 0; m < 10; ++m) {
    const double t = fmax(theta - ldexp(SHRINK, m), 0.0);
    make(t, W);
    if (in_G(W, gm1)) return t;
  }
  return 0.0;
}

// Scaling limiter of a point value (Section 3.3): density-only step, then a
// whole-state blend towards the LLF state; eps from the LLF state.
__device__ void limit_point(const double UH[NV], const double UL[NV], double gm1, double W[NV], Counters* cn,
                            bool counted) {
#pragma clang fp contract(off)
  const double rhoL = UL[0];
  const double er = fmin(EPS_FLOOR, rhoL);
  // common case: the LLF state has p >= 1e-13 (so eps_p = 1e-13) and the
  // high-order state satisfies both bounds: no limiting, no division (the
  // four tests are combined without short circuits: one branch, not four)
  if ((rhoL > 0.0) & p_at_least(UL, EPS_FLOOR, gm1) & (UH[0] >= er) & p_at_least(UH, EPS_FLOOR, gm1)) {
#pragma unroll
    for (int c = 0; c < NV; ++c) W[c] = UH[c];
    return;
  }
  const double pL = pressure(UL, gm1);
  const double ep = fmin(EPS_FLOOR, pL);
  double th1 = 1.0;
  if (UH[0] < er) th1 = (rhoL - er) / (rhoL - UH[0]);
  double Us[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) Us[c] = UH[c];
  if (th1 < 1.0) Us[0] = th1 * UH[0] + (1.0 - th1) * rhoL;
  const double ps = pressure(Us, gm1);
  double th2 = 1.0;
  if (ps < ep) th2 = (pL - ep) / (pL - ps);
  if (counted && (th1 < 1.0 || th2 < 1.0)) count(&cn->n_point_limited);
  auto make = [&](double t, double* Wt) {
#pragma unroll
    for (int c = 0; c < NV; ++c) Wt[c] = t * Us[c] + (1.0 - t) * UL[c];
  };
  if (th2 == 1.0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) W[c] = Us[c];
    // rho >= er and p >= ep already hold; both bounds are positive when the
    // LLF state is in G, so W is in G without another evaluation.
    if (rhoL > 0.0 && pL > 0.0 && Us[0] > 0.0) return;
  } else {
    make(th2, W);
  }
  if (th2 > 0.0 && !in_G(W, gm1)) {
    if (counted) count(&cn->n_fallback);
    th2 = shrink_into_G(th2, gm1, make);
    make(th2, W);
  }
}

// Limiter of the centre value (remark rmk:cell_center), reading: the whole
// state is blended towards the cell average, first for rho >= eps_rho, then
// for p >= eps_p, eps from the cell average.
__device__ void limit_centre(const double Uc[NV], const double A[NV], double gm1, double C[NV], Counters* cn,
                             bool counted) {
#pragma clang fp contract(off)
  const double rhoA = A[0];
  const double er = fmin(EPS_FLOOR, rhoA);
  if ((rhoA > 0.0) & p_at_least(A, EPS_FLOOR, gm1) & (Uc[0] >= er) & p_at_least(Uc, EPS_FLOOR, gm1)) {
#pragma unroll
    for (int c = 0; c < NV; ++c) C[c] = Uc[c];
    return;
  }
  const double pA = pressure(A, gm1);
  const double ep = fmin(EPS_FLOOR, pA);
  double th1 = 1.0;
  if (Uc[0] < er) th1 = (rhoA - er) / (rhoA - Uc[0]);
  double Ur[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) Ur[c] = th1 < 1.0 ? th1 * Uc[c] + (1.0 - th1) * A[c] : Uc[c];
  const double pr = pressure(Ur, gm1);
  double th2 = 1.0;
  if (pr < ep) th2 = (pA - ep) / (pA - pr);
  if (counted && (th1 < 1.0 || th2 < 1.0)) count(&cn->n_centre_limited);
  auto make = [&](double t, double* Wt) {
#pragma unroll
    for (int c = 0; c < NV; ++c) Wt[c] = t * Ur[c] + (1.0 - t) * A[c];
  };
  if (th2 == 1.0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) C[c] = Ur[c];
    if (rhoA > 0.0 && pA > 0.0 && Ur[0] > 0.0) return;
  } else {
    make(th2, C);
  }
  if (th2 > 0.0 && !in_G(C, gm1)) {
    if (counted) count(&cn->n_fallback);
    th2 = shrink_into_G(th2, gm1, make);
    make(th2, C);
  }
}

// Step (1) of the parametrized flux limiter (Section 3.2) for a cell whose
// LLF-flux update is G: A^LLF = G - dt S^LLF, A^src = G - dt S^s (S^s the
// sensor-blended high-order source); theta_src = 1 if p(A^src) >= eps_p,
// otherwise the scaling fraction towards A^LLF; eps from A^LLF (R20).
// A^{Lim,1} = theta A^src + (1 - theta) A^LLF, then the round-off fallback.
// Returns theta_src; er, ep are the flux limiter's bounds.
template <class R>
__device__ double source_step(const double G[NV], const R S[NV], const R Sl[NV], double dt, double gm1,
                              double A1[NV], double& er, double& ep, Counters* cn, bool counted) {
#pragma clang fp contract(off)
  double Allf[NV], Asrc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    Allf[c] = G[c] - dt * (double)Sl[c];
    Asrc[c] = G[c] - dt * (double)S[c];
  }
  const double rhoL = Allf[0];
  if (counted && !in_G_fast(Allf)) count(&cn->n_llf_not_admissible);
  er = fmin(EPS_FLOOR, rhoL);
  ep = EPS_FLOOR;
  if (rhoL > 0.0 && p_at_least(Allf, EPS_FLOOR, gm1) && p_at_least(Asrc, EPS_FLOOR, gm1)) {
    // both bounds hold with eps_p = 1e-13: theta_src = 1, A^{Lim,1} in G
#pragma unroll
    for (int c = 0; c < NV; ++c) A1[c] = Asrc[c];
    return 1.0;
  }
  // the step may act: the reference form of the pressures
  double th = 1.0;
  {
    const double pL = pressure(Allf, gm1);
    ep = fmin(EPS_FLOOR, pL);
    const double psrc = pressure(Asrc, gm1);
    if (psrc < ep) {
      th = (pL - ep) / (pL - psrc);
      if (counted) count(&cn->n_source_limited);
    }
  }
  auto make = [&](double tt, double* Wt) {
#pragma unroll
    for (int c = 0; c < NV; ++c) Wt[c] = tt * Asrc[c] + (1.0 - tt) * Allf[c];
  };
  if (th == 1.0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) A1[c] = Asrc[c];
  } else {
    make(th, A1);
  }
  if (th > 0.0 && !in_G(A1, gm1)) {
    if (counted) count(&cn->n_fallback);
    th = shrink_into_G(th, gm1, make);
    make(th, A1);
  }
  return th;
}

// The pressure condition along A1 + r D as the cubic of Section 3.2,
// q(r) = rho (E - |B|^2/2 - eps_p/(gamma-1)) - |m|^2/2, and dq/dr.
__device__ __forceinline__ void pressure_cubic(const double A1[NV], const double D[NV], double r, double gm1,
                                               double ep, double& q, double& dq) {
#pragma clang fp contract(off)
  double W[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) W[c] = A1[c] + r * D[c];
  const double b2 = W[4] * W[4] + W[5] * W[5] + W[6] * W[6];
  const double m2 = W[1] * W[1] + W[2] * W[2] + W[3] * W[3];
  const double e = W[7] - 0.5 * b2 - ep / gm1;
  q = W[0] * e - 0.5 * m2;
  const double de = D[7] - (W[4] * D[4] + W[5] * D[5] + W[6] * D[6]);
  dq = D[0] * e + W[0] * de - (W[1] * D[1] + W[2] * D[2] + W[3] * D[3]);
}

// Root in (0,1) of the cubic by Newton from r = 1 inside a sign bracket.
__device__ double vertex_root(const double A1[NV], const double D[NV], double gm1, double ep, int& iters) {
#pragma clang fp contract(off)
  double lo = 0.0, hi = 1.0, r = 1.0;
  iters = 0;
  for (int it = 0; it < 50; ++it) {
    double q, dq;
    pressure_cubic(A1, D, r, gm1, ep, q, dq);
    ++iters;
    if (q >= 0.0) lo = r; else hi = r;
    double rn = r - q / dq;
    if (!(rn >= lo && rn <= hi)) rn = 0.5 * (lo + hi);
    const double step = fabs(rn - r);
    r = rn;
    if (step <= 1e-13) break;
  }
  return r;
}

// Step (2) of the parametrized flux limiter (Section 3.2): density box,
// pressure shrink over the 15 non-trivial vertices, Lambda_{L,R,D,U}, and
// the round-off fallback on the final box.  H(I, c) returns component c of
// the anti-diffusive update H_I (I = L, R, D, U).
template <class HF, bool SHORTCUT = true>
__device__ void limiter_box(const double A1[NV], HF H, double gm1, double er, double ep, double Lam[4], Counters* cn,
                            bool counted) {
#pragma clang fp contract(off)
  double h0[4];
#pragma unroll
  for (int I = 0; I < 4; ++I) h0[I] = H(I, 0);
  double neg = 0.0;
#pragma unroll
  for (int I = 0; I < 4; ++I) neg += h0[I] < 0.0 ? h0[I] : 0.0;
  double Lr[4];
#pragma unroll
  for (int I = 0; I < 4; ++I) Lr[I] = h0[I] < 0.0 ? fmin(1.0, (A1[0] - er) / (LAMBDA_REG - neg)) : 1.0;
  // Sufficient test: every vertex A1 + sum_{I in K} Lr_I H_I is a convex
  // combination of A1 and the four points A1 + 4 Lr_I H_I (weights 1/4 and
  // 1 - |K|/4), and {rho >= er, p >= ep} is convex; when A1 and those four
  // points are admissible no vertex needs the pressure shrink.  A1 itself
  // can miss ep: after the source step's round-off fallback it is only
  // known to lie in G.  (Round-off aside the vertices then pass their own
  // tests; where a vertex's pressure is within round-off of ep the per-vertex
  // test may still ask for a root of size 1 - O(round-off).)
  if constexpr (SHORTCUT) {
    bool all_ok = A1[0] >= er && A1[0] > 0.0 && p_at_least(A1, ep, gm1);
#pragma unroll
    for (int I = 0; I < 4; ++I) {
      double W[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) W[c] = A1[c] + 4.0 * (Lr[I] * H(I, c));
      all_ok = all_ok && W[0] >= er && W[0] > 0.0 && p_at_least(W, ep, gm1);
    }
    if (all_ok) {
#pragma unroll
      for (int I = 0; I < 4; ++I) Lam[I] = Lr[I];
      return;
    }
  }
  double rmin[4] = {1.0, 1.0, 1.0, 1.0};
  bool any_root = false;
  // the vertex loops stay rolled: they run only where the shortcut fails,
  // and unrolled they cost the fast path its registers (spills)
#pragma unroll 1
  for (int k = 1; k < 16; ++k) {
    double D[NV], W[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double d = 0.0;
#pragma unroll
      for (int I = 0; I < 4; ++I)
        if (k & (1 << I)) d += Lr[I] * H(I, c);
      D[c] = d;
      W[c] = A1[c] + d;
    }
    if (pressure(W, gm1) < ep) {
      int it;
      const double r = vertex_root(A1, D, gm1, ep, it);
      any_root = true;
      if (counted) {
        count(&cn->n_newton);
        count_max(&cn->newton_iters_max, (unsigned long long)it);
      }
#pragma unroll
      for (int I = 0; I < 4; ++I)
        if (k & (1 << I)) rmin[I] = fmin(rmin[I], r);
    }
  }
#pragma unroll
  for (int I = 0; I < 4; ++I) Lam[I] = Lr[I] * rmin[I];
  if (!any_root) return;
  auto box_ok = [&](const double L[4]) {
#pragma unroll 1
    for (int k = 1; k < 16; ++k) {
      double W[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double d = 0.0;
#pragma unroll
        for (int I = 0; I < 4; ++I)
          if (k & (1 << I)) d += L[I] * H(I, c);
        W[c] = A1[c] + d;
      }
      if (!in_G(W, gm1)) return false;
    }
    return true;
  };
  if (box_ok(Lam)) return;
  if (counted) count(&cn->n_fallback);
  for (int m = 0; m < 10; ++m) {
    double L[4];
#pragma unroll
    for (int I = 0; I < 4; ++I) L[I] = fmax(Lam[I] - ldexp(SHRINK, m), 0.0);
    if (box_ok(L)) {
#pragma unroll
      for (int I = 0; I < 4; ++I) Lam[I] = L[I];
      return;
    }
  }
#pragma unroll
  for (int I = 0; I < 4; ++I) Lam[I] = 0.0;
}

}  // namespace afm
