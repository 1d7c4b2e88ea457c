// af_adjoint.h -- the discrete adjoint of one forward-Euler stage of the
// positivity-preserving Active Flux scheme (arXiv 2506.04857), as plain FP64
// per-entity functions: a recording forward that stores the limiter and
// sensor decisions of the stage, and the reverse sweep that applies the
// transposed Jacobian of the stage with those decisions frozen.
//
// Entities and their index ranges (owner convention: X(k,j) is the left face
// of cell k, Y(i,l) the bottom face of cell i, V(k,l) the lower-left vertex;
// an outflow direction mirrors evenly, a periodic one wraps):
//   centre      real cells            the limited centre value (Section 2.1
//                                     and the remark on the centre limiter)
//   point       real X, Y, V points   high-order point update (Section 2.3),
//                                     first-order LLF point update and the
//                                     scaling limiter (Section 3.3)
//   sensor      cells [-2,n+2)^2      phi1, phi2, phi3 (Section 3.4)
//   x-interface k in [-1,nx+2), j in [-1,ny+1): Simpson flux, LLF flux and
//               the sensor coefficient (Sections 2.2, 3.1, 3.4)
//   y-interface i in [-1,nx+1), l in [-1,ny+2)
//   limiter     cells [-1,n+1)^2      sources, first-order update, source
//                                     coefficient and the box Lambda of the
//                                     parametrized flux limiter (Section 3.2)
//   update      real cells            interface coefficients and the
//                                     flux-form update of the cell average
// Ghost entities of an outflow boundary are computations of their own (their
// mirrored stencils differ from the owner's), so they are kept as separate
// entities; for a periodic direction they duplicate their owners.
//
// Every max / min breaks ties to its first argument, |x| has derivative +1 at
// x = 0 and sqrt derivative 0 at 0.  The forward here evaluates the scheme
// in the paper's order with IEEE division and square roots; its outputs equal
// those of the fused stage kernels to rounding.
//
// Each function is a host-and-device inline function (AF_HD) so that the
// reverse sweep can be unit-checked on the host.  Scatters go through a
// policy type Add with a static add(double*, double).
#pragma once

#include <stddef.h>
#include <stdint.h>

// Everything is inlined into the kernels: the reverse kernels make no
// device-function calls.  (An out-of-line callee was miscompiled: its
// long-branch expansion used the return-address registers s[30:31] as
// scratch without saving them, so a wave that took that branch returned
// into the middle of the callee.)
#ifndef AF_HD
#define AF_HD __host__ __device__ __forceinline__
#endif

namespace afadj {

constexpr int NV = 8;
constexpr double EPS_FLOOR = 1e-13;   // rho and p bounds of the admissible set
constexpr double LAMBDA_REG = 1e-12;  // regulariser of the density box
constexpr double SHRINK = 1e-8;       // round-off fallback step 2^m * 1e-8
constexpr double SENSOR_TINY = 1e-40;

struct AGeo {
  int nx, ny, nxp, nyp, bcx, bcy;
  double dx, dy, gamma, kappa;
};

AF_HD int mcell(int i, int n, int bc) {
  if (bc == 0) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  if (i < 0) return -1 - i;
  if (i >= n) return 2 * n - 1 - i;
  return i;
}
AF_HD int mnode(int k, int n, int bc) {
  if (bc == 0) {
    k %= n;
    return k < 0 ? k + n : k;
  }
  if (k < 0) return -k;
  if (k > n) return 2 * n - k;
  return k;
}

// A location of one DoF: flat index of component 0 and the plane stride.
struct Loc {
  size_t i, s;
};
AF_HD Loc locA(const AGeo& g, int i, int j) {
  return {(size_t)mcell(j, g.ny, g.bcy) * g.nx + mcell(i, g.nx, g.bcx), (size_t)g.nx * g.ny};
}
AF_HD Loc locX(const AGeo& g, int k, int j) {
  return {(size_t)mcell(j, g.ny, g.bcy) * g.nxp + mnode(k, g.nx, g.bcx), (size_t)g.nxp * g.ny};
}
AF_HD Loc locY(const AGeo& g, int i, int l) {
  return {(size_t)mnode(l, g.ny, g.bcy) * g.nx + mcell(i, g.nx, g.bcx), (size_t)g.nx * g.nyp};
}
AF_HD Loc locV(const AGeo& g, int k, int l) {
  return {(size_t)mnode(l, g.ny, g.bcy) * g.nxp + mnode(k, g.nx, g.bcx), (size_t)g.nxp * g.nyp};
}
AF_HD void ld(const double* p, Loc L, double* u) {
  for (int c = 0; c < NV; ++c) u[c] = p[L.i + c * L.s];
}
template <class Add>
AF_HD void put(double* p, Loc L, const double* l) {
  for (int c = 0; c < NV; ++c)
    if (l[c] != 0.0) Add::add(p + L.i + c * L.s, l[c]);
}
AF_HD void zero8(double* a) {
  for (int c = 0; c < NV; ++c) a[c] = 0.0;
}
AF_HD double sgn(double x) { return x < 0.0 ? -1.0 : 1.0; }
AF_HD double dmax(double a, double b) { return a < b ? b : a; }  // ties: first
AF_HD double dmin(double a, double b) { return b < a ? b : a; }  // ties: first

// ------------------------------------------------------------ physics
// p = (gamma-1)(E - |m|^2/(2 rho) - |B|^2/2), Section 1.
AF_HD double pres(const double* U, double g) {
  const double m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
  const double b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  return (g - 1.0) * (U[7] - m2 / (2.0 * U[0]) - b2 / 2.0);
}
AF_HD bool admissible(const double* U, double g) { return U[0] > 0.0 && pres(U, g) > 0.0; }
// lU += lp dp/dU
AF_HD void pres_vjp(const double* U, double g, double lp, double* lU) {
  const double r = U[0];
  const double v1 = U[1] / r, v2 = U[2] / r, v3 = U[3] / r;
  const double gm = (g - 1.0) * lp;
  lU[0] += gm * 0.5 * (v1 * v1 + v2 * v2 + v3 * v3);
  lU[1] -= gm * v1;
  lU[2] -= gm * v2;
  lU[3] -= gm * v3;
  lU[4] -= gm * U[4];
  lU[5] -= gm * U[5];
  lU[6] -= gm * U[6];
  lU[7] += gm;
}

// Physical flux F_n (n = 0: x, 1: y), Section 1.
AF_HD void flux(const double* U, double g, int n, double* F) {
  const double rho = U[0];
  const double v[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
  const double B[3] = {U[4], U[5], U[6]};
  const double p = pres(U, g);
  const double pt = p + (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]) / 2.0;
  const double vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
  F[0] = rho * v[n];
  for (int i = 0; i < 3; ++i) F[1 + i] = rho * v[n] * v[i] - B[n] * B[i] + (i == n ? pt : 0.0);
  for (int i = 0; i < 3; ++i) F[4 + i] = i == n ? 0.0 : v[n] * B[i] - B[n] * v[i];
  F[7] = (U[7] + pt) * v[n] - B[n] * vB;
}
// lU += (dF_n/dU)^T lF
AF_HD void flux_vjp(const double* U, double g, int n, const double* lF, double* lU) {
  const double rho = U[0];
  const double v[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
  const double B[3] = {U[4], U[5], U[6]};
  const double E = U[7];
  const double p = pres(U, g);
  const double pt = p + (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]) / 2.0;
  const double vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
  double lr = 0.0, lE = 0.0, lpt = 0.0;
  double lv[3] = {0.0, 0.0, 0.0}, lB[3] = {0.0, 0.0, 0.0};
  lr += lF[0] * v[n];
  lv[n] += lF[0] * rho;
  for (int i = 0; i < 3; ++i) {
    const double l = lF[1 + i];
    lr += l * v[n] * v[i];
    lv[n] += l * rho * v[i];
    lv[i] += l * rho * v[n];
    lB[n] -= l * B[i];
    lB[i] -= l * B[n];
    if (i == n) lpt += l;
  }
  for (int i = 0; i < 3; ++i) {
    if (i == n) continue;
    const double l = lF[4 + i];
    lv[n] += l * B[i];
    lB[i] += l * v[n];
    lB[n] -= l * v[i];
    lv[i] -= l * B[n];
  }
  {
    const double l = lF[7];
    lE += l * v[n];
    lpt += l * v[n];
    lv[n] += l * (E + pt);
    lB[n] -= l * vB;
    for (int i = 0; i < 3; ++i) {
      lv[i] -= l * B[n] * B[i];
      lB[i] -= l * B[n] * v[i];
    }
  }
  // pt = p + |B|^2/2, p = (gamma-1)(E - rho |v|^2/2 - |B|^2/2)
  for (int i = 0; i < 3; ++i) lB[i] += lpt * B[i];
  const double gm = (g - 1.0) * lpt;
  lE += gm;
  lr -= gm * 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int i = 0; i < 3; ++i) {
    lv[i] -= gm * rho * v[i];
    lB[i] -= gm * B[i];
  }
  // v = m / rho
  for (int i = 0; i < 3; ++i) {
    lU[1 + i] += lv[i] / rho;
    lr -= lv[i] * v[i] / rho;
    lU[4 + i] += lB[i];
  }
  lU[0] += lr;
  lU[7] += lE;
}

// Fast magnetosonic speed c_{f,n}, with the inner discriminant clamped at 0.
AF_HD double cfast(const double* U, double g, int n) {
  const double rho = U[0];
  const double c2 = g * pres(U, g) / rho;
  const double b2 = (U[4] * U[4] + U[5] * U[5] + U[6] * U[6]) / rho;
  const double Bl = U[4 + n];
  const double s = c2 + b2;
  double disc = s * s - 4.0 * c2 * Bl * Bl / rho;
  if (disc < 0.0) disc = 0.0;
  return sqrt(0.5 * (s + sqrt(disc)));
}
AF_HD void cfast_vjp(const double* U, double g, int n, double lc, double* lU) {
  const double rho = U[0];
  const double p = pres(U, g);
  const double c2 = g * p / rho;
  const double bb = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  const double b2 = bb / rho;
  const double Bl = U[4 + n];
  const double s = c2 + b2;
  double disc = s * s - 4.0 * c2 * Bl * Bl / rho;
  const bool clamped = disc < 0.0;
  if (clamped) disc = 0.0;
  const double rd = sqrt(disc);
  const double cf = sqrt(0.5 * (s + rd));
  if (!(cf > 0.0)) return;
  const double lcf2 = lc / (2.0 * cf);
  double ls = 0.5 * lcf2;
  const double lrd = 0.5 * lcf2;
  const double ldisc = (!clamped && rd > 0.0) ? lrd / (2.0 * rd) : 0.0;
  ls += ldisc * 2.0 * s;
  double lc2 = -ldisc * 4.0 * Bl * Bl / rho;
  const double lBl = -ldisc * 8.0 * c2 * Bl / rho;
  double lr = ldisc * 4.0 * c2 * Bl * Bl / (rho * rho);
  lc2 += ls;
  const double lb2 = ls;
  for (int i = 0; i < 3; ++i) lU[4 + i] += lb2 * 2.0 * U[4 + i] / rho;
  lr -= lb2 * bb / (rho * rho);
  const double lp = lc2 * g / rho;
  lr -= lc2 * g * p / (rho * rho);
  lU[4 + n] += lBl;
  lU[0] += lr;
  pres_vjp(U, g, lp, lU);
}

// Spectral radius |v_n| + c_{f,n} (Section 2.3).
AF_HD double srad(const double* U, double g, int n) { return fabs(U[1 + n] / U[0]) + cfast(U, g, n); }
AF_HD void srad_vjp(const double* U, double g, int n, double l, double* lU) {
  const double v = U[1 + n] / U[0];
  const double lv = l * sgn(v);
  lU[1 + n] += lv / U[0];
  lU[0] -= lv * v / U[0];
  cfast_vjp(U, g, n, l, lU);
}

// Godunov-Powell source vector Psi = (0, B, v, v.B).
AF_HD void psi(const double* U, double* P) {
  const double v1 = U[1] / U[0], v2 = U[2] / U[0], v3 = U[3] / U[0];
  P[0] = 0.0;
  P[1] = U[4];
  P[2] = U[5];
  P[3] = U[6];
  P[4] = v1;
  P[5] = v2;
  P[6] = v3;
  P[7] = v1 * U[4] + v2 * U[5] + v3 * U[6];
}
AF_HD void psi_vjp(const double* U, const double* lP, double* lU) {
  const double rho = U[0];
  for (int i = 0; i < 3; ++i) {
    const double v = U[1 + i] / rho;
    const double lv = lP[4 + i] + lP[7] * U[4 + i];
    lU[4 + i] += lP[1 + i] + lP[7] * v;
    lU[1 + i] += lv / rho;
    lU[0] -= lv * v / rho;
  }
}

// alpha_{n,*}(a, b) of the Lemma of Section 3.1.
AF_HD double astar(const double* a, const double* b, double g, int n) {
  const double sa = sqrt(a[0]), sb = sqrt(b[0]);
  const double va = a[1 + n] / a[0], vb = b[1 + n] / b[0];
  const double t1 = dmax(fabs(va), fabs(sa * va + sb * vb) / (sa + sb));
  const double t2 = dmax(cfast(a, g, n), cfast(b, g, n));
  const double d1 = a[4] - b[4], d2 = a[5] - b[5], d3 = a[6] - b[6];
  const double t3 = sqrt(d1 * d1 + d2 * d2 + d3 * d3) / (sa + sb);
  return t1 + t2 + t3;
}
AF_HD void astar_vjp(const double* a, const double* b, double g, int n, double l, double* la, double* lb) {
  const double sa = sqrt(a[0]), sb = sqrt(b[0]);
  const double va = a[1 + n] / a[0], vb = b[1 + n] / b[0];
  const double den = sa + sb, num = sa * va + sb * vb;
  double lsa = 0.0, lsb = 0.0, lva = 0.0, lvb = 0.0;
  if (fabs(va) < fabs(num) / den) {
    const double lnum = l * sgn(num) / den, lden = -l * fabs(num) / (den * den);
    lsa += lnum * va + lden;
    lsb += lnum * vb + lden;
    lva += lnum * sa;
    lvb += lnum * sb;
  } else {
    lva += l * sgn(va);
  }
  if (cfast(a, g, n) < cfast(b, g, n))
    cfast_vjp(b, g, n, l, lb);
  else
    cfast_vjp(a, g, n, l, la);
  const double d[3] = {a[4] - b[4], a[5] - b[5], a[6] - b[6]};
  const double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double lden3 = -l * nrm / (den * den);
  lsa += lden3;
  lsb += lden3;
  if (nrm > 0.0)
    for (int i = 0; i < 3; ++i) {
      const double t = l / den * d[i] / nrm;
      la[4 + i] += t;
      lb[4 + i] -= t;
    }
  la[0] += lsa / (2.0 * sa);
  lb[0] += lsb / (2.0 * sb);
  la[1 + n] += lva / a[0];
  la[0] -= lva * va / a[0];
  lb[1 + n] += lvb / b[0];
  lb[0] -= lvb * vb / b[0];
}

// LLF viscosity: the Lemma's bound with equality,
// max{max(rho(a), rho(b)), max(alpha*(a,b), alpha*(b,a))}.
AF_HD double alpha_llf(const double* a, const double* b, double g, int n) {
  const double m1 = dmax(srad(a, g, n), srad(b, g, n));
  const double m2 = dmax(astar(a, b, g, n), astar(b, a, g, n));
  return dmax(m1, m2);
}
// The four speeds of the LLF viscosity and which of them is the maximum
// (0: rho(a), 1: rho(b), 2: alpha*(a,b), 3: alpha*(b,a); ties to the first).
AF_HD double alpha_llf_arg(const double* a, const double* b, double g, int n, int& arg) {
  const double r1 = srad(a, g, n), r2 = srad(b, g, n);
  const double s1 = astar(a, b, g, n), s2 = astar(b, a, g, n);
  const double m1 = dmax(r1, r2), m2 = dmax(s1, s2);
  arg = m1 < m2 ? (s1 < s2 ? 3 : 2) : (r1 < r2 ? 1 : 0);
  return dmax(m1, m2);
}
AF_HD void alpha_llf_vjp_at(const double* a, const double* b, double g, int n, int arg, double l, double* la,
                            double* lb) {
  if (arg == 3)
    astar_vjp(b, a, g, n, l, lb, la);
  else if (arg == 2)
    astar_vjp(a, b, g, n, l, la, lb);
  else if (arg == 1)
    srad_vjp(b, g, n, l, lb);
  else
    srad_vjp(a, g, n, l, la);
}
// LLF flux 1/2 [F(a) + F(b) - alpha (b - a)], Section 3.1.
AF_HD void llf(const double* a, const double* b, double g, int n, double* F) {
  const double al = alpha_llf(a, b, g, n);
  double Fa[NV], Fb[NV];
  flux(a, g, n, Fa);
  flux(b, g, n, Fb);
  for (int c = 0; c < NV; ++c) F[c] = 0.5 * (Fa[c] + Fb[c] - al * (b[c] - a[c]));
}
AF_HD void llf_vjp(const double* a, const double* b, double g, int n, const double* lF, double* la, double* lb) {
  int arg;
  const double al = alpha_llf_arg(a, b, g, n, arg);
  double h[NV], lal = 0.0;
  for (int c = 0; c < NV; ++c) {
    h[c] = 0.5 * lF[c];
    la[c] += 0.5 * al * lF[c];
    lb[c] -= 0.5 * al * lF[c];
    lal -= 0.5 * lF[c] * (b[c] - a[c]);
  }
  flux_vjp(a, g, n, h, la);
  flux_vjp(b, g, n, h, lb);
  alpha_llf_vjp_at(a, b, g, n, arg, lal, la, lb);
}

// ------------------------------------------ point values (Section 2.3)
// Flux-vector-split derivative D+F+ + D-F- on the five states at offsets
// -h, -h/2, 0, h/2, h, F+- = 1/2 (F +- alpha w), alpha the largest spectral
// radius on the stencil; dB = 1/2 (D+ B_n + D- B_n).
AF_HD void fvs_line(const double* const w[5], double g, int n, double h, double* R, double& dB) {
  double F[5][NV];
  double alpha = 0.0;
  for (int m = 0; m < 5; ++m) {
    flux(w[m], g, n, F[m]);
    alpha = dmax(alpha, srad(w[m], g, n));
  }
  for (int c = 0; c < NV; ++c) {
    double Fp[5], Fm[5];
    for (int m = 0; m < 5; ++m) {
      Fp[m] = 0.5 * (F[m][c] + alpha * w[m][c]);
      Fm[m] = 0.5 * (F[m][c] - alpha * w[m][c]);
    }
    const double Dp = (Fp[0] - 4.0 * Fp[1] + 3.0 * Fp[2]) / h;
    const double Dm = (-3.0 * Fm[2] + 4.0 * Fm[3] - Fm[4]) / h;
    R[c] = Dp + Dm;
  }
  const int b = 4 + n;
  const double Bp = (w[0][b] - 4.0 * w[1][b] + 3.0 * w[2][b]) / h;
  const double Bm = (-3.0 * w[2][b] + 4.0 * w[3][b] - w[4][b]) / h;
  dB = 0.5 * (Bp + Bm);
}
AF_HD void fvs_line_vjp(const double* const w[5], double g, int n, double h, const double* lR, double ldB,
                        double* const lw[5]) {
  const double cp[5] = {1.0, -4.0, 3.0, 0.0, 0.0};
  const double cm[5] = {0.0, 0.0, -3.0, 4.0, -1.0};
  double alpha = 0.0;
  int am = -1;
  for (int m = 0; m < 5; ++m) {
    const double r = srad(w[m], g, n);
    if (alpha < r) {
      alpha = r;
      am = m;
    }
  }
  double lal = 0.0;
  for (int m = 0; m < 5; ++m) {
    const double sp = 0.5 * (cp[m] + cm[m]) / h, sd = 0.5 * (cp[m] - cm[m]) / h;
    double lF[NV];
    for (int c = 0; c < NV; ++c) {
      lF[c] = sp * lR[c];
      lw[m][c] += sd * alpha * lR[c];
      lal += sd * lR[c] * w[m][c];
    }
    flux_vjp(w[m], g, n, lF, lw[m]);
    lw[m][4 + n] += sp * ldB;
  }
  if (am >= 0) srad_vjp(w[am], g, n, lal, lw[am]);
}

// First-order LLF update of a point value from its four neighbours, with
// the central divergence over 2 dx, 2 dy (Section 3.3, as printed).
AF_HD void point_llf(const double* U, const double* L, const double* R, const double* D, const double* Up, double dt,
                     const AGeo& g, double* W) {
  double FR[NV], FL[NV], FU[NV], FD[NV], P[NV];
  llf(U, R, g.gamma, 0, FR);
  llf(L, U, g.gamma, 0, FL);
  llf(U, Up, g.gamma, 1, FU);
  llf(D, U, g.gamma, 1, FD);
  const double divB = (R[4] - L[4]) / (2.0 * g.dx) + (Up[5] - D[5]) / (2.0 * g.dy);
  psi(U, P);
  for (int c = 0; c < NV; ++c)
    W[c] = U[c] - dt / g.dx * (FR[c] - FL[c]) - dt / g.dy * (FU[c] - FD[c]) - dt * divB * P[c];
}
AF_HD void point_llf_vjp(const double* U, const double* L, const double* R, const double* D, const double* Up,
                         double dt, const AGeo& g, const double* lW, double* lU, double* lL, double* lR, double* lD,
                         double* lUp) {
  double P[NV], lx[NV], ly[NV], lP[NV];
  psi(U, P);
  const double divB = (R[4] - L[4]) / (2.0 * g.dx) + (Up[5] - D[5]) / (2.0 * g.dy);
  double ldiv = 0.0;
  for (int c = 0; c < NV; ++c) {
    lU[c] += lW[c];
    lx[c] = -dt / g.dx * lW[c];
    ly[c] = -dt / g.dy * lW[c];
    ldiv -= dt * lW[c] * P[c];
    lP[c] = -dt * divB * lW[c];
  }
  llf_vjp(U, R, g.gamma, 0, lx, lU, lR);  // + F^(U,R)
  for (int c = 0; c < NV; ++c) lx[c] = -lx[c];
  llf_vjp(L, U, g.gamma, 0, lx, lL, lU);  // - F^(L,U)
  llf_vjp(U, Up, g.gamma, 1, ly, lU, lUp);
  for (int c = 0; c < NV; ++c) ly[c] = -ly[c];
  llf_vjp(D, U, g.gamma, 1, ly, lD, lU);
  psi_vjp(U, lP, lU);
  lR[4] += ldiv / (2.0 * g.dx);
  lL[4] -= ldiv / (2.0 * g.dx);
  lUp[5] += ldiv / (2.0 * g.dy);
  lD[5] -= ldiv / (2.0 * g.dy);
}

// ------------------------------------------------- scaling limiters
// Decision bits of a two-step scaling limiter (points: Section 3.3; centre:
// the remark on the centre value) and of the round-off fallback.
enum : uint32_t {
  BL_T1 = 1u,      // step (1) fraction active
  BL_T2 = 2u,      // step (2) fraction active
  BL_SHIFT = 4u,   // fallback: coefficient shifted by 2^m 1e-8, m in bits 8..11
  BL_ZERO = 8u,    // fallback: coefficient 0
  BL_ER = 16u,     // eps_rho = rho of the safe state (< 1e-13)
  BL_EP = 32u,     // eps_p = p of the safe state (< 1e-13)
};
AF_HD double shrink_step(int m) { return SHRINK * (double)(1 << m); }

// Round-off fallback: keep t if t W1 + (1-t) W0 is in G (or t <= 0), else
// the first t - 2^m 1e-8 (floored at 0), m = 0..9, whose state is in G, else 0.
AF_HD double fallback(double t, const double* W1, const double* W0, double g, uint32_t& fl) {
  double W[NV];
  for (int c = 0; c < NV; ++c) W[c] = t * W1[c] + (1.0 - t) * W0[c];
  if (admissible(W, g) || t <= 0.0) return t;
  for (int m = 0; m < 10; ++m) {
    const double x = t - shrink_step(m);
    const double s = x < 0.0 ? 0.0 : x;
    for (int c = 0; c < NV; ++c) W[c] = s * W1[c] + (1.0 - s) * W0[c];
    if (admissible(W, g)) {
      fl |= x < 0.0 ? (uint32_t)BL_ZERO : (uint32_t)(BL_SHIFT | ((uint32_t)m << 8));
      return s;
    }
  }
  fl |= BL_ZERO;
  return 0.0;
}
AF_HD double fallback_apply(double t, uint32_t fl) {
  if (fl & BL_ZERO) return 0.0;
  if (fl & BL_SHIFT) return t - shrink_step((int)((fl >> 8) & 15u));
  return t;
}

// Point scaling limiter: UH high order, UL the first-order safe state.
AF_HD void point_limit(const double* UH, const double* UL, double g, double* out, uint32_t& fl) {
  const double rhoL = UL[0], pL = pres(UL, g);
  double er = EPS_FLOOR, ep = EPS_FLOOR;
  if (rhoL < EPS_FLOOR) {
    er = rhoL;
    fl |= BL_ER;
  }
  if (pL < EPS_FLOOR) {
    ep = pL;
    fl |= BL_EP;
  }
  double th1 = 1.0;
  if (UH[0] < er) {
    th1 = (rhoL - er) / (rhoL - UH[0]);
    fl |= BL_T1;
  }
  double Us[NV];
  for (int c = 0; c < NV; ++c) Us[c] = UH[c];
  Us[0] = th1 * UH[0] + (1.0 - th1) * rhoL;
  const double ps = pres(Us, g);
  double th2 = 1.0;
  if (ps < ep) {
    th2 = (pL - ep) / (pL - ps);
    fl |= BL_T2;
  }
  th2 = fallback(th2, Us, UL, g, fl);
  for (int c = 0; c < NV; ++c) out[c] = th2 * Us[c] + (1.0 - th2) * UL[c];
}
AF_HD void point_limit_vjp(const double* UH, const double* UL, double g, uint32_t fl, const double* lout,
                           double* lUH, double* lUL) {
  const double rhoL = UL[0], pL = pres(UL, g);
  const double er = (fl & BL_ER) ? rhoL : EPS_FLOOR, ep = (fl & BL_EP) ? pL : EPS_FLOOR;
  const double th1 = (fl & BL_T1) ? (rhoL - er) / (rhoL - UH[0]) : 1.0;
  double Us[NV];
  for (int c = 0; c < NV; ++c) Us[c] = UH[c];
  Us[0] = th1 * UH[0] + (1.0 - th1) * rhoL;
  const double ps = pres(Us, g);
  const double th2r = (fl & BL_T2) ? (pL - ep) / (pL - ps) : 1.0;
  const double th2 = fallback_apply(th2r, fl);
  double lUs[NV], lth2 = 0.0;
  for (int c = 0; c < NV; ++c) {
    lth2 += lout[c] * (Us[c] - UL[c]);
    lUs[c] = th2 * lout[c];
    lUL[c] += (1.0 - th2) * lout[c];
  }
  if (fl & BL_ZERO) lth2 = 0.0;
  double lpL = 0.0, lep = 0.0, lrhoL = 0.0, ler = 0.0;
  if (fl & BL_T2) {
    const double den = pL - ps;
    const double ln = lth2 / den, ldn = -lth2 * th2r / den;
    lpL += ln + ldn;
    lep -= ln;
    pres_vjp(Us, g, -ldn, lUs);
  }
  for (int c = 1; c < NV; ++c) lUH[c] += lUs[c];
  lUH[0] += th1 * lUs[0];
  lrhoL += (1.0 - th1) * lUs[0];
  const double lth1 = lUs[0] * (UH[0] - rhoL);
  if (fl & BL_T1) {
    const double den = rhoL - UH[0];
    const double ln = lth1 / den, ldn = -lth1 * th1 / den;
    lrhoL += ln + ldn;
    ler -= ln;
    lUH[0] -= ldn;
  }
  if (fl & BL_ER) lrhoL += ler;
  if (fl & BL_EP) lpL += lep;
  lUL[0] += lrhoL;
  pres_vjp(UL, g, lpL, lUL);
}

// Centre value C~ = (36 A - 4 (faces) - (corners)) / 16 and its limiter:
// the whole state is blended towards A, first for rho, then for p.
// S9 order of the inputs: A, Xl, Xr, Yd, Yu, Vdl, Vdr, Vul, Vur.
AF_HD void centre_raw(const double* const in[9], double* Uc) {
  for (int c = 0; c < NV; ++c) {
    const double faces = (in[1][c] + in[2][c]) + (in[3][c] + in[4][c]);
    const double corners = (in[5][c] + in[6][c]) + (in[7][c] + in[8][c]);
    Uc[c] = (36.0 * in[0][c] - 4.0 * faces - corners) / 16.0;
  }
}
AF_HD void centre_limit(const double* A, const double* Uc, double g, double* C, uint32_t& fl) {
  const double rhoA = A[0], pA = pres(A, g);
  double er = EPS_FLOOR, ep = EPS_FLOOR;
  if (rhoA < EPS_FLOOR) {
    er = rhoA;
    fl |= BL_ER;
  }
  if (pA < EPS_FLOOR) {
    ep = pA;
    fl |= BL_EP;
  }
  double th1 = 1.0;
  if (Uc[0] < er) {
    th1 = (rhoA - er) / (rhoA - Uc[0]);
    fl |= BL_T1;
  }
  double Ur[NV];
  for (int c = 0; c < NV; ++c) Ur[c] = th1 * Uc[c] + (1.0 - th1) * A[c];
  const double pr = pres(Ur, g);
  double th2 = 1.0;
  if (pr < ep) {
    th2 = (pA - ep) / (pA - pr);
    fl |= BL_T2;
  }
  th2 = fallback(th2, Ur, A, g, fl);
  for (int c = 0; c < NV; ++c) C[c] = th2 * Ur[c] + (1.0 - th2) * A[c];
}
// lA, lUc accumulate.
AF_HD void centre_limit_vjp(const double* A, const double* Uc, double g, uint32_t fl, const double* lC, double* lA,
                            double* lUc) {
  const double rhoA = A[0], pA = pres(A, g);
  const double er = (fl & BL_ER) ? rhoA : EPS_FLOOR, ep = (fl & BL_EP) ? pA : EPS_FLOOR;
  const double th1 = (fl & BL_T1) ? (rhoA - er) / (rhoA - Uc[0]) : 1.0;
  double Ur[NV];
  for (int c = 0; c < NV; ++c) Ur[c] = th1 * Uc[c] + (1.0 - th1) * A[c];
  const double pr = pres(Ur, g);
  const double th2r = (fl & BL_T2) ? (pA - ep) / (pA - pr) : 1.0;
  const double th2 = fallback_apply(th2r, fl);
  double lUr[NV], lth2 = 0.0;
  for (int c = 0; c < NV; ++c) {
    lth2 += lC[c] * (Ur[c] - A[c]);
    lUr[c] = th2 * lC[c];
    lA[c] += (1.0 - th2) * lC[c];
  }
  if (fl & BL_ZERO) lth2 = 0.0;
  double lpA = 0.0, lep = 0.0, lrhoA = 0.0, ler = 0.0;
  if (fl & BL_T2) {
    const double den = pA - pr;
    const double ln = lth2 / den, ldn = -lth2 * th2r / den;
    lpA += ln + ldn;
    lep -= ln;
    pres_vjp(Ur, g, -ldn, lUr);
  }
  double lth1 = 0.0;
  for (int c = 0; c < NV; ++c) {
    lUc[c] += th1 * lUr[c];
    lA[c] += (1.0 - th1) * lUr[c];
    lth1 += lUr[c] * (Uc[c] - A[c]);
  }
  if (fl & BL_T1) {
    const double den = rhoA - Uc[0];
    const double ln = lth1 / den, ldn = -lth1 * th1 / den;
    lrhoA += ln + ldn;
    ler -= ln;
    lUc[0] -= ldn;
  }
  if (fl & BL_ER) lrhoA += ler;
  if (fl & BL_EP) lpA += lep;
  lA[0] += lrhoA;
  pres_vjp(A, g, lpA, lA);
}

// ------------------------------------------- cell average (Section 2.2)
AF_HD double d3(int at, double u0, double u1, double u2) {
  if (at == 0) return -3.0 * u0 + 4.0 * u1 - u2;
  if (at == 1) return u2 - u0;
  return u0 - 4.0 * u1 + 3.0 * u2;
}
AF_HD double d3c(int at, int q) {
  const double c[3][3] = {{-3.0, 4.0, -1.0}, {-1.0, 0.0, 1.0}, {1.0, -4.0, 3.0}};
  return c[at][q];
}
// Powell source of the cell average: 3x3 Simpson quadrature of (div B) Psi on
// the cell's nine points P[a][b] (a along x, b along y).
AF_HD void cell_source(const double* const P[3][3], const AGeo& g, double* S) {
  const double w[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  zero8(S);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double dB1 = d3(a, P[0][b][4], P[1][b][4], P[2][b][4]) / g.dx;
      const double dB2 = d3(b, P[a][0][5], P[a][1][5], P[a][2][5]) / g.dy;
      const double divB = dB1 + dB2;
      double Q[NV];
      psi(P[a][b], Q);
      for (int c = 0; c < NV; ++c) S[c] += w[a] * w[b] * divB * Q[c];
    }
}
AF_HD void cell_source_vjp(const double* const P[3][3], const AGeo& g, const double* lS, double* const lP[3][3]) {
  const double w[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double dB1 = d3(a, P[0][b][4], P[1][b][4], P[2][b][4]) / g.dx;
      const double dB2 = d3(b, P[a][0][5], P[a][1][5], P[a][2][5]) / g.dy;
      const double divB = dB1 + dB2;
      double Q[NV], lQ[NV], ldiv = 0.0;
      psi(P[a][b], Q);
      for (int c = 0; c < NV; ++c) {
        ldiv += w[a] * w[b] * lS[c] * Q[c];
        lQ[c] = w[a] * w[b] * divB * lS[c];
      }
      psi_vjp(P[a][b], lQ, lP[a][b]);
      for (int q = 0; q < 3; ++q) {
        lP[q][b][4] += d3c(a, q) * ldiv / g.dx;
        lP[a][q][5] += d3c(b, q) * ldiv / g.dy;
      }
    }
}

// ------------------------------------------------ shock sensor (Section 3.4)
enum : uint32_t {
  SN_PHI2 = 1u,    // phi2 takes -div/|.| (else 0)
  SN_N1X = 2u,     // numerator of phi1^x negative
  SN_D1X = 4u,     // denominator of phi1^x negative
  SN_N1Y = 8u,
  SN_D1Y = 16u,
  SN_N3 = 32u,     // numerator of phi3 negative
  SN_D3 = 64u,     // B1 + B2 of the cell negative
};
AF_HD double ptot(const double* U, double g) {
  return pres(U, g) + (U[4] * U[4] + U[5] * U[5] + U[6] * U[6]) / 2.0;
}
AF_HD void ptot_vjp(const double* U, double g, double l, double* lU) {
  pres_vjp(U, g, l, lU);
  for (int i = 4; i < 7; ++i) lU[i] += l * U[i];
}
// c centre; l, r, d, u its neighbours.  phi[0..3] = phi1x, phi1y, phi2, phi3.
AF_HD void sensor(const double* c, const double* l, const double* r, const double* d, const double* u,
                  const AGeo& g, double* phi, uint32_t& fl) {
  const double ptc = ptot(c, g.gamma), ptl = ptot(l, g.gamma), ptr = ptot(r, g.gamma), ptd = ptot(d, g.gamma),
               ptu = ptot(u, g.gamma);
  const double n1x = ptr - 2.0 * ptc + ptl, d1x = ptr + 2.0 * ptc + ptl;
  const double n1y = ptu - 2.0 * ptc + ptd, d1y = ptu + 2.0 * ptc + ptd;
  phi[0] = fabs(n1x) / fabs(d1x);
  phi[1] = fabs(n1y) / fabs(d1y);
  const double divv = (r[1] / r[0] - l[1] / l[0]) / (2.0 * g.dx) + (u[2] / u[0] - d[2] / d[0]) / (2.0 * g.dy);
  const double curlv = (r[2] / r[0] - l[2] / l[0]) / (2.0 * g.dx) - (u[1] / u[0] - d[1] / d[0]) / (2.0 * g.dy);
  const double q = -divv / sqrt(divv * divv + curlv * curlv + SENSOR_TINY);
  phi[2] = q < 0.0 ? 0.0 : q;
  const double n3 = r[4] - l[4] + u[5] - d[5], s3 = c[4] + c[5];
  phi[3] = fabs(n3) / (fabs(s3) + SENSOR_TINY);
  fl = (q < 0.0 ? 0u : (uint32_t)SN_PHI2) | (n1x < 0.0 ? (uint32_t)SN_N1X : 0u) | (d1x < 0.0 ? (uint32_t)SN_D1X : 0u) |
       (n1y < 0.0 ? (uint32_t)SN_N1Y : 0u) | (d1y < 0.0 ? (uint32_t)SN_D1Y : 0u) | (n3 < 0.0 ? (uint32_t)SN_N3 : 0u) |
       (s3 < 0.0 ? (uint32_t)SN_D3 : 0u);
}
AF_HD void sensor_vjp(const double* c, const double* l, const double* r, const double* d, const double* u,
                      const AGeo& g, uint32_t fl, const double* lphi, double* lc, double* ll, double* lr, double* ld,
                      double* lu) {
  const double gm = g.gamma;
  const double ptc = ptot(c, gm), ptl = ptot(l, gm), ptr = ptot(r, gm), ptd = ptot(d, gm), ptu = ptot(u, gm);
  double lptc = 0.0, lptl = 0.0, lptr = 0.0, lptd = 0.0, lptu = 0.0;
  {  // phi1x = |N| / |D|
    const double N = ptr - 2.0 * ptc + ptl, D = ptr + 2.0 * ptc + ptl;
    const double sN = (fl & SN_N1X) ? -1.0 : 1.0, sD = (fl & SN_D1X) ? -1.0 : 1.0;
    const double lN = lphi[0] * sN / fabs(D), lD = -lphi[0] * fabs(N) * sD / (D * D);
    lptr += lN + lD;
    lptl += lN + lD;
    lptc += -2.0 * lN + 2.0 * lD;
  }
  {
    const double N = ptu - 2.0 * ptc + ptd, D = ptu + 2.0 * ptc + ptd;
    const double sN = (fl & SN_N1Y) ? -1.0 : 1.0, sD = (fl & SN_D1Y) ? -1.0 : 1.0;
    const double lN = lphi[1] * sN / fabs(D), lD = -lphi[1] * fabs(N) * sD / (D * D);
    lptu += lN + lD;
    lptd += lN + lD;
    lptc += -2.0 * lN + 2.0 * lD;
  }
  ptot_vjp(c, gm, lptc, lc);
  ptot_vjp(l, gm, lptl, ll);
  ptot_vjp(r, gm, lptr, lr);
  ptot_vjp(d, gm, lptd, ld);
  ptot_vjp(u, gm, lptu, lu);
  if (fl & SN_PHI2) {
    const double divv = (r[1] / r[0] - l[1] / l[0]) / (2.0 * g.dx) + (u[2] / u[0] - d[2] / d[0]) / (2.0 * g.dy);
    const double curlv = (r[2] / r[0] - l[2] / l[0]) / (2.0 * g.dx) - (u[1] / u[0] - d[1] / d[0]) / (2.0 * g.dy);
    const double s = sqrt(divv * divv + curlv * curlv + SENSOR_TINY);
    const double lq = lphi[2];
    const double ls = lq * divv / (s * s);
    const double ldiv = -lq / s + ls * divv / s;
    const double lcurl = ls * curlv / s;
    // velocity components v = m / rho of the neighbours
    auto addv = [](const double* U, int i, double lv, double* lU) {
      lU[1 + i] += lv / U[0];
      lU[0] -= lv * U[1 + i] / (U[0] * U[0]);
    };
    addv(r, 0, ldiv / (2.0 * g.dx), lr);
    addv(l, 0, -ldiv / (2.0 * g.dx), ll);
    addv(u, 1, ldiv / (2.0 * g.dy), lu);
    addv(d, 1, -ldiv / (2.0 * g.dy), ld);
    addv(r, 1, lcurl / (2.0 * g.dx), lr);
    addv(l, 1, -lcurl / (2.0 * g.dx), ll);
    addv(u, 0, -lcurl / (2.0 * g.dy), lu);
    addv(d, 0, lcurl / (2.0 * g.dy), ld);
  }
  {  // phi3 = |N| / (|c4 + c5| + tiny)
    const double N = r[4] - l[4] + u[5] - d[5], s3 = c[4] + c[5];
    const double den = fabs(s3) + SENSOR_TINY;
    const double sN = (fl & SN_N3) ? -1.0 : 1.0, sS = (fl & SN_D3) ? -1.0 : 1.0;
    const double lN = lphi[3] * sN / den, lden = -lphi[3] * fabs(N) / (den * den);
    lr[4] += lN;
    ll[4] -= lN;
    lu[5] += lN;
    ld[5] -= lN;
    lc[4] += lden * sS;
    lc[5] += lden * sS;
  }
}
// Interface coefficient exp(-kappa [max(phi1) max(phi2) + max(phi3)]) between
// the sensors of the two adjacent cells; dir selects phi1^x or phi1^y.
// bits: 1, 2, 4 = the max of phi1, phi2, phi3 is taken from the second cell.
AF_HD double sensor_theta(const double* pL, const double* pR, int dir, double kappa, uint32_t& fl) {
  const double a1 = pL[dir], b1 = pR[dir];
  const double p1 = dmax(a1, b1), p2 = dmax(pL[2], pR[2]), p3 = dmax(pL[3], pR[3]);
  fl = (a1 < b1 ? 1u : 0u) | (pL[2] < pR[2] ? 2u : 0u) | (pL[3] < pR[3] ? 4u : 0u);
  return exp(-kappa * (p1 * p2 + p3));
}
AF_HD void sensor_theta_vjp(const double* pL, const double* pR, int dir, double kappa, uint32_t fl, double ts,
                            double l, double* lpL, double* lpR) {
  const double p1 = (fl & 1u) ? pR[dir] : pL[dir];
  const double p2 = (fl & 2u) ? pR[2] : pL[2];
  const double lz = -kappa * ts * l;
  ((fl & 1u) ? lpR : lpL)[dir] += lz * p2;
  ((fl & 2u) ? lpR : lpL)[2] += lz * p1;
  ((fl & 4u) ? lpR : lpL)[3] += lz;
}

// --------------------------------------- parametrized flux limiter (3.2)
// Decision bits of one limiter cell.
enum : uint64_t {
  LM_TSRC = 1ull,          // source coefficient fraction active
  LM_TS_SHIFT = 2ull,      // its fallback shifted, m in bits 4..7
  LM_TS_ZERO = 4ull,       // its fallback gave 0
  LM_ER = 1ull << 8,       // eps_rho = rho(A^LLF)
  LM_EP = 1ull << 9,       // eps_p = p(A^LLF)
  // bits 10..13: Lambda^rho_I is the fraction; bits 14..17: rho(H_I) < 0
  // bits 18..32: a root was solved for vertex k = 1..15 (bit 17 + k)
  // bits 33..48: argmin vertex of Lambda_I (4 bits per I, 0 = none)
  LM_BOX_SHIFT = 1ull << 49,  // box fallback shifted, m in bits 50..53
  LM_BOX_ZERO = 1ull << 54,   // box fallback gave 0
  // bits 55..58: Lambda_I floored at 0 by the shifted fallback
  // bits 59..60: interface of the smallest sensor coefficient (L, R, D, U)
};
// Bits under which some coefficient of steps (1)-(2) depends on the state
// (source fraction or its fallback, a density-box fraction, a vertex root,
// the box fallback); without them theta_src = Lambda_I = 1 are constants.
constexpr uint64_t LM_ACTIVE = LM_TSRC | LM_TS_SHIFT | LM_TS_ZERO | (15ull << 10) | (0x7fffull << 18) |
                               LM_BOX_SHIFT | LM_BOX_ZERO;
AF_HD uint64_t lm_lrf(int I) { return 1ull << (10 + I); }
AF_HD uint64_t lm_neg(int I) { return 1ull << (14 + I); }
AF_HD uint64_t lm_root(int k) { return 1ull << (17 + k); }
AF_HD int lm_arg(uint64_t f, int I) { return (int)((f >> (33 + 4 * I)) & 15ull); }
AF_HD uint64_t lm_floor(int I) { return 1ull << (55 + I); }
AF_HD int lm_tsmin(uint64_t f) { return (int)((f >> 59) & 3ull); }

// q(r) = rho(r) [E(r) - |B(r)|^2/2 - eps_p/(gamma-1)] - |m(r)|^2/2 along
// W(r) = A1 + r D: rho (p - eps_p)/(gamma-1), the pressure condition as a
// cubic in r without the pole at rho = 0.
AF_HD void qcubic(const double* A1, const double* D, double r, double g, double ep, double& q, double& dq) {
  double W[NV];
  for (int c = 0; c < NV; ++c) W[c] = A1[c] + r * D[c];
  const double b2 = W[4] * W[4] + W[5] * W[5] + W[6] * W[6];
  const double m2 = W[1] * W[1] + W[2] * W[2] + W[3] * W[3];
  const double e = W[7] - b2 / 2.0 - ep / (g - 1.0);
  q = W[0] * e - m2 / 2.0;
  const double de = D[7] - (W[4] * D[4] + W[5] * D[5] + W[6] * D[6]);
  dq = D[0] * e + W[0] * de - (W[1] * D[1] + W[2] * D[2] + W[3] * D[3]);
}
// Root in (0,1) of q: Newton from r = 1 kept inside the bracket [lo, hi]
// (a step leaving it is replaced by the midpoint), stopping at a step
// <= 1e-13 or after 50 steps.
AF_HD double vroot(const double* A1, const double* D, double g, double ep) {
  double lo = 0.0, hi = 1.0, r = 1.0;
  for (int it = 0; it < 50; ++it) {
    double q, dq;
    qcubic(A1, D, r, g, ep, q, dq);
    if (q >= 0.0)
      lo = r;
    else
      hi = r;
    double rn = r - q / dq;
    if (!(rn >= lo && rn <= hi)) rn = 0.5 * (lo + hi);
    const double step = fabs(rn - r);
    r = rn;
    if (step <= 1e-13) break;
  }
  return r;
}
AF_HD void box_vertex(const double* A1, const double H[4][NV], const double* L, int k, double* D, double* W) {
  zero8(D);
  for (int I = 0; I < 4; ++I)
    if (k & (1 << I))
      for (int c = 0; c < NV; ++c) D[c] += L[I] * H[I][c];
  for (int c = 0; c < NV; ++c) W[c] = A1[c] + D[c];
}
AF_HD bool box_ok(const double* A1, const double H[4][NV], const double* L, double g) {
  for (int k = 1; k < 16; ++k) {
    double D[NV], W[NV];
    box_vertex(A1, H, L, k, D, W);
    if (!admissible(W, g)) return false;
  }
  return true;
}
// Step (2): density box Lambda^rho, the pressure shrink over the 15 vertices,
// and the round-off fallback on the final box.  H: H_L, H_R, H_D, H_U.
AF_HD void limiter_box(const double* A1, const double H[4][NV], double g, double er, double ep, double* Lam,
                       double* rk, uint64_t& fl) {
  double neg = 0.0;
  for (int I = 0; I < 4; ++I)
    if (H[I][0] < 0.0) {
      neg += H[I][0];
      fl |= lm_neg(I);
    }
  double Lr[4];
  for (int I = 0; I < 4; ++I) {
    Lr[I] = 1.0;
    if (H[I][0] < 0.0) {
      const double f = (A1[0] - er) / (LAMBDA_REG - neg);
      if (f < 1.0) {
        Lr[I] = f;
        fl |= lm_lrf(I);
      }
    }
  }
  double rmin[4] = {1.0, 1.0, 1.0, 1.0};
  int arg[4] = {0, 0, 0, 0};
  bool any_root = false;
  for (int k = 1; k < 16; ++k) {
    double D[NV], W[NV];
    box_vertex(A1, H, Lr, k, D, W);
    double r = 1.0;
    if (pres(W, g) < ep) {
      r = vroot(A1, D, g, ep);
      fl |= lm_root(k);
      any_root = true;
    }
    rk[k - 1] = r;
    for (int I = 0; I < 4; ++I)
      if ((k & (1 << I)) && r < rmin[I]) {
        rmin[I] = r;
        arg[I] = k;
      }
  }
  for (int I = 0; I < 4; ++I) {
    Lam[I] = Lr[I] * rmin[I];
    fl |= (uint64_t)arg[I] << (33 + 4 * I);
  }
  if (!any_root || box_ok(A1, H, Lam, g)) return;
  for (int m = 0; m < 10; ++m) {
    double L[4];
    uint64_t fb = 0;
    for (int I = 0; I < 4; ++I) {
      const double x = Lam[I] - shrink_step(m);
      L[I] = x < 0.0 ? 0.0 : x;
      if (x < 0.0) fb |= lm_floor(I);
    }
    if (box_ok(A1, H, L, g)) {
      for (int I = 0; I < 4; ++I) Lam[I] = L[I];
      fl |= LM_BOX_SHIFT | ((uint64_t)m << 50) | fb;
      return;
    }
  }
  for (int I = 0; I < 4; ++I) Lam[I] = 0.0;
  fl |= LM_BOX_ZERO;
}
// lA1, lH (4 x 8), ler, lep accumulate.
AF_HD void limiter_box_vjp(const double* A1, const double H[4][NV], double g, double er, double ep, const double* rk,
                           uint64_t fl, const double* lLam_in, double* lA1, double lH[4][NV], double& ler,
                           double& lep) {
  if (fl & LM_BOX_ZERO) return;
  double lLam[4];
  for (int I = 0; I < 4; ++I) lLam[I] = ((fl & LM_BOX_SHIFT) && (fl & lm_floor(I))) ? 0.0 : lLam_in[I];
  double neg = 0.0;
  for (int I = 0; I < 4; ++I)
    if (fl & lm_neg(I)) neg += H[I][0];
  const double den = LAMBDA_REG - neg;
  const double frac = (A1[0] - er) / den;
  double Lr[4], lLr[4];
  for (int I = 0; I < 4; ++I) {
    Lr[I] = (fl & lm_lrf(I)) ? frac : 1.0;
    lLr[I] = 0.0;
  }
  double lr[15];
  for (int k = 0; k < 15; ++k) lr[k] = 0.0;
  for (int I = 0; I < 4; ++I) {
    const int a = lm_arg(fl, I);
    const double rmin = a ? rk[a - 1] : 1.0;
    lLr[I] += lLam[I] * rmin;
    if (a) lr[a - 1] += lLam[I] * Lr[I];
  }
  for (int k = 1; k < 16; ++k) {
    if (lr[k - 1] == 0.0 || !(fl & lm_root(k))) continue;
    const double r = rk[k - 1];
    double D[NV], W0[NV];
    box_vertex(A1, H, Lr, k, D, W0);
    double W[NV];
    for (int c = 0; c < NV; ++c) W[c] = A1[c] + r * D[c];
    const double e = W[7] - (W[4] * W[4] + W[5] * W[5] + W[6] * W[6]) / 2.0 - ep / (g - 1.0);
    const double qW[NV] = {e, -W[1], -W[2], -W[3], -W[0] * W[4], -W[0] * W[5], -W[0] * W[6], W[0]};
    double qr = 0.0;
    for (int c = 0; c < NV; ++c) qr += qW[c] * D[c];
    const double s = -lr[k - 1] / qr;
    double lD[NV];
    for (int c = 0; c < NV; ++c) {
      lA1[c] += s * qW[c];
      lD[c] = s * r * qW[c];
    }
    lep += s * (-W[0] / (g - 1.0));
    for (int I = 0; I < 4; ++I)
      if (k & (1 << I))
        for (int c = 0; c < NV; ++c) {
          lLr[I] += lD[c] * H[I][c];
          lH[I][c] += Lr[I] * lD[c];
        }
  }
  double lneg = 0.0;
  for (int I = 0; I < 4; ++I)
    if (fl & lm_lrf(I)) {
      lA1[0] += lLr[I] / den;
      ler -= lLr[I] / den;
      lneg += lLr[I] * frac / den;
    }
  for (int I = 0; I < 4; ++I)
    if (fl & lm_neg(I)) lH[I][0] += lneg;
}

// The limiter cell: inputs A, the sensor-blended and LLF fluxes at the four
// interfaces (L, R, D, U), S^s and S^LLF.  Step (1) (source coefficient) and
// step (2) (box); returns theta_src and Lambda[4], records the decisions.
struct CellIn {
  double A[NV];
  double Fs[4][NV], Fl[4][NV];
  double Ss[NV], Sllf[NV];
};
AF_HD void cell_states(const CellIn& w, double dt, const AGeo& g, double* Allf, double* Asrc) {
  const double ldx = dt / g.dx, ldy = dt / g.dy;
  for (int c = 0; c < NV; ++c) {
    const double G = w.A[c] - ldx * (w.Fl[1][c] - w.Fl[0][c]) - ldy * (w.Fl[3][c] - w.Fl[2][c]);
    Allf[c] = G - dt * w.Sllf[c];
    Asrc[c] = G - dt * w.Ss[c];
  }
}
AF_HD void cell_H(const CellIn& w, double dt, const AGeo& g, double H[4][NV]) {
  const double ldx = dt / g.dx, ldy = dt / g.dy;
  for (int c = 0; c < NV; ++c) {
    H[0][c] = ldx * (w.Fs[0][c] - w.Fl[0][c]);
    H[1][c] = -ldx * (w.Fs[1][c] - w.Fl[1][c]);
    H[2][c] = ldy * (w.Fs[2][c] - w.Fl[2][c]);
    H[3][c] = -ldy * (w.Fs[3][c] - w.Fl[3][c]);
  }
}
AF_HD void cell_limiter(const CellIn& w, double dt, const AGeo& g, double& thsrc, double* Lam, double* rk,
                        uint64_t& fl) {
  const double gm = g.gamma;
  double Allf[NV], Asrc[NV];
  cell_states(w, dt, g, Allf, Asrc);
  const double rhoL = Allf[0], pL = pres(Allf, gm);
  double er = EPS_FLOOR, ep = EPS_FLOOR;
  if (rhoL < EPS_FLOOR) {
    er = rhoL;
    fl |= LM_ER;
  }
  if (pL < EPS_FLOOR) {
    ep = pL;
    fl |= LM_EP;
  }
  double th = 1.0;
  const double psrc = pres(Asrc, gm);
  if (psrc < ep) {
    th = (pL - ep) / (pL - psrc);
    fl |= LM_TSRC;
  }
  uint32_t bf = 0;
  th = fallback(th, Asrc, Allf, gm, bf);
  if (bf & BL_ZERO) fl |= LM_TS_ZERO;
  if (bf & BL_SHIFT) fl |= LM_TS_SHIFT | ((uint64_t)((bf >> 8) & 15u) << 4);
  thsrc = th;
  double A1[NV];
  for (int c = 0; c < NV; ++c) A1[c] = th * Asrc[c] + (1.0 - th) * Allf[c];
  double H[4][NV];
  cell_H(w, dt, g, H);
  limiter_box(A1, H, gm, er, ep, Lam, rk, fl);
}
// Reverse of cell_limiter: given the adjoints of theta_src and Lambda[4],
// accumulate those of A, Fs[4], Fl[4], Ss, Sllf.
struct CellAdj {
  double A[NV];
  double Fs[4][NV], Fl[4][NV];
  double Ss[NV], Sllf[NV];
};
AF_HD void cell_limiter_vjp(const CellIn& w, double dt, const AGeo& g, const double* rk, uint64_t fl,
                                  double lthsrc, const double* lLam, CellAdj& o) {
  const double gm = g.gamma;
  const double ldx = dt / g.dx, ldy = dt / g.dy;
  double Allf[NV], Asrc[NV];
  cell_states(w, dt, g, Allf, Asrc);
  const double rhoL = Allf[0], pL = pres(Allf, gm);
  const double er = (fl & LM_ER) ? rhoL : EPS_FLOOR, ep = (fl & LM_EP) ? pL : EPS_FLOOR;
  const double psrc = pres(Asrc, gm);
  const double thr = (fl & LM_TSRC) ? (pL - ep) / (pL - psrc) : 1.0;
  double th = thr;
  if (fl & LM_TS_ZERO)
    th = 0.0;
  else if (fl & LM_TS_SHIFT)
    th = thr - shrink_step((int)((fl >> 4) & 15ull));
  double A1[NV];
  for (int c = 0; c < NV; ++c) A1[c] = th * Asrc[c] + (1.0 - th) * Allf[c];
  double H[4][NV], lH[4][NV], lA1[NV];
  cell_H(w, dt, g, H);
  for (int I = 0; I < 4; ++I) zero8(lH[I]);
  zero8(lA1);
  double ler = 0.0, lep = 0.0;
  limiter_box_vjp(A1, H, gm, er, ep, rk, fl, lLam, lA1, lH, ler, lep);
  // A1 = th Asrc + (1 - th) Allf
  double lAs[NV], lAl[NV], lth = lthsrc;
  for (int c = 0; c < NV; ++c) {
    lAs[c] = th * lA1[c];
    lAl[c] = (1.0 - th) * lA1[c];
    lth += lA1[c] * (Asrc[c] - Allf[c]);
  }
  if (fl & LM_TS_ZERO) lth = 0.0;
  double lpL = 0.0, lrhoL = 0.0;
  if (fl & LM_TSRC) {
    const double den = pL - psrc;
    const double ln = lth / den, ldn = -lth * thr / den;
    lpL += ln + ldn;
    lep -= ln;
    pres_vjp(Asrc, gm, -ldn, lAs);
  }
  if (fl & LM_ER) lrhoL += ler;
  if (fl & LM_EP) lpL += lep;
  lAl[0] += lrhoL;
  pres_vjp(Allf, gm, lpL, lAl);
  // Allf = G - dt Sllf, Asrc = G - dt Ss, G = A - ldx (FlR - FlL) - ldy (FlU - FlD)
  for (int c = 0; c < NV; ++c) {
    const double lG = lAl[c] + lAs[c];
    o.Sllf[c] -= dt * lAl[c];
    o.Ss[c] -= dt * lAs[c];
    o.A[c] += lG;
    o.Fl[1][c] -= ldx * lG;
    o.Fl[0][c] += ldx * lG;
    o.Fl[3][c] -= ldy * lG;
    o.Fl[2][c] += ldy * lG;
    // H
    o.Fs[0][c] += ldx * lH[0][c];
    o.Fl[0][c] -= ldx * lH[0][c];
    o.Fs[1][c] -= ldx * lH[1][c];
    o.Fl[1][c] += ldx * lH[1][c];
    o.Fs[2][c] += ldy * lH[2][c];
    o.Fl[2][c] -= ldy * lH[2][c];
    o.Fs[3][c] -= ldy * lH[3][c];
    o.Fl[3][c] += ldy * lH[3][c];
  }
}

}  // namespace afadj
