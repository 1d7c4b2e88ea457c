// af_stage.hip -- kernels of one SSP-RK3 stage of the PP Active Flux scheme
// for 2D ideal MHD with the Godunov-Powell source (gfx950), and the C ABI
// declared in include/af_mhd.h.
//
// Stage structure (forward Euler on U^(k), then out = a_k U^n + b_k FE):
//   k_centre      limited centre values (Section 2.1, remark rmk:cell_center)
//   k_sensor      shock-sensor indicators per cell (Section 3.4)
//   k_vertex / k_xface / k_yface
//                 point values: LLF flux-vector splitting + central div B
//                 (Section 2.3), first-order LLF safe state and scaling
//                 limiter (Section 3.3), SSP combination
//   k_iface       Simpson flux (Section 2.2), LLF flux (eq. 2d_llf_flux) and
//                 sensor coefficient per interface
//   k_cell_limit  nine-point Powell source (eq. semi_av_src), LLF source,
//                 sensor blend, flux-limiter steps (1)-(2) (Section 3.2)
//   k_cell_final  step (3) and the limited update, eq. (2d_av_limited)
// Intermediates live in the caller's workspace.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "af_device.h"
#include "af_mhd.h"

using namespace afm;

namespace {

constexpr int BLK = 256;

// Extended index ranges.  Cells whose flux-limiter box is needed: interior
// plus one ghost ring across outflow boundaries.  Interfaces: those of these
// cells.  Sensor: one more ring.  Periodic directions use wrapped indices.
struct Ext {
  int cx0, cnx, cy0, cny;   // limiter cells: [cx0, cx0+cnx) x [cy0, cy0+cny)
  int sx0, snx, sy0, sny;   // sensor cells
  int fx0, fnx;             // x-interfaces k in [fx0, fx0+fnx), rows = limiter rows
  int fy0, fny;             // y-interfaces l in [fy0, fy0+fny), cols = limiter cols
};

struct WS {                 // workspace pointers
  double* centre;           // [8][ny][nx]
  double* sensor;           // [4][sny][snx]
  double* fxs;              // [8][cny][fnx]  sensor-blended flux
  double* fxl;              // [8][cny][fnx]  LLF flux
  double* fxt;              // [cny][fnx]     sensor theta
  double* fys;              // [8][fny][cnx]
  double* fyl;
  double* fyt;              // [fny][cnx]
  double* lam;              // [4][cny][cnx]  Lambda_{L,R,D,U}
  double* slim;             // [8][cny][cnx]  limited source
  double* partial;          // reduction partials
  Counters* cnt;
  double* scratch[2][4];    // two RK scratch states
};

__device__ __forceinline__ int ext_x(const Ext& e, const Geo& g, int k) {  // x-interface column
  return g.bcx ? k - e.fx0 : (k >= g.nx ? k - g.nx : (k < 0 ? k + g.nx : k));
}
__device__ __forceinline__ int ext_y(const Ext& e, const Geo& g, int l) {
  return g.bcy ? l - e.fy0 : (l >= g.ny ? l - g.ny : (l < 0 ? l + g.ny : l));
}
__device__ __forceinline__ int ext_ci(const Ext& e, const Geo& g, int i) {  // limiter-cell column
  return g.bcx ? i - e.cx0 : (i >= g.nx ? i - g.nx : (i < 0 ? i + g.nx : i));
}
__device__ __forceinline__ int ext_cj(const Ext& e, const Geo& g, int j) {
  return g.bcy ? j - e.cy0 : (j >= g.ny ? j - g.ny : (j < 0 ? j + g.ny : j));
}
__device__ __forceinline__ int ext_si(const Ext& e, const Geo& g, int i) {  // sensor column
  return g.bcx ? i - e.sx0 : (i >= g.nx ? i - g.nx : (i < 0 ? i + g.nx : i));
}
__device__ __forceinline__ int ext_sj(const Ext& e, const Geo& g, int j) {
  return g.bcy ? j - e.sy0 : (j >= g.ny ? j - g.ny : (j < 0 ? j + g.ny : j));
}

// ------------------------------------------------------------------ centre
// C = limited [36 A - 4 (sum of face values) - (sum of vertex values)] / 16.
__global__ __launch_bounds__(BLK) void k_centre(Geo g, CState u, double* __restrict__ centre, Counters* cn) {
  const int t = blockIdx.x * BLK + threadIdx.x;
  if (t >= g.nx * g.ny) return;
  const int i = t % g.nx, j = t / g.nx;
  double A[NV], a[NV], b[NV], c[NV], d[NV], Uc[NV];
  ldA(g, u.a, i, j, A);
  ldX(g, u.x, i, j, a);
  ldX(g, u.x, i + 1, j, b);
  ldY(g, u.y, i, j, c);
  ldY(g, u.y, i, j + 1, d);
#pragma unroll
  for (int q = 0; q < NV; ++q) Uc[q] = -4.0 * ((a[q] + b[q]) + (c[q] + d[q]));
  ldV(g, u.v, i, j, a);
  ldV(g, u.v, i + 1, j, b);
  ldV(g, u.v, i, j + 1, c);
  ldV(g, u.v, i + 1, j + 1, d);
#pragma unroll
  for (int q = 0; q < NV; ++q) Uc[q] = (36.0 * A[q] + Uc[q] - ((a[q] + b[q]) + (c[q] + d[q]))) * 0.0625;
  double C[NV];
  limit_centre(Uc, A, g.gm1, C, cn, true);
#pragma unroll
  for (int q = 0; q < NV; ++q) centre[q * g.sc + t] = C[q];
}

__device__ __forceinline__ void ldC(const Geo& g, const double* centre, int i, int j, double u[NV]) {
  load8(centre, g.sc, (long)map_cell(j, g.ny, g.bcy) * g.nx + map_cell(i, g.nx, g.bcx), u);
}

// ------------------------------------------------------------------ sensor
// phi1 (Jameson on the total pressure, per direction), phi2 (modified
// Ducros), phi3 (divergence relative to |B1 + B2|), from cell averages.
// phi2 = max(-d / sqrt(d^2 + w^2 + 1e-40), 0) is ill-conditioned where the
// discrete divergence d and curl w of the averaged velocity both vanish (an
// O(1) jump from a rounding-level d).  This kernel is therefore compiled
// without FMA contraction and with true divisions, so that exact
// cancellations (d = 0 for a field whose v1 depends on y only and v2 on x
// only, e.g. Orszag-Tang initial data) stay exact.
__device__ double sensor_pressure(const double U[NV], double gamma) {
#pragma clang fp contract(off)
  const double m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
  const double b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  return (gamma - 1.0) * (U[7] - m2 / (2.0 * U[0]) - b2 / 2.0);
}

__global__ __launch_bounds__(BLK) void k_sensor(Geo g, Ext e, CState u, double* __restrict__ sen) {
#pragma clang fp contract(off)
  const int t = blockIdx.x * BLK + threadIdx.x;
  if (t >= e.snx * e.sny) return;
  const int i = e.sx0 + t % e.snx, j = e.sy0 + t / e.snx;
  double U[NV];
  double pt[5], v1[5], v2[5], b1[5], b2[5];
  const int di[5] = {0, -1, 1, 0, 0}, dj[5] = {0, 0, 0, -1, 1};
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    ldA(g, u.a, i + di[m], j + dj[m], U);
    pt[m] = sensor_pressure(U, g.gamma) + (U[4] * U[4] + U[5] * U[5] + U[6] * U[6]) / 2.0;
    v1[m] = U[1] / U[0];
    v2[m] = U[2] / U[0];
    b1[m] = U[4];
    b2[m] = U[5];
  }
  const long plane = (long)e.snx * e.sny;
  sen[t] = fabs(pt[2] - 2.0 * pt[0] + pt[1]) / fabs(pt[2] + 2.0 * pt[0] + pt[1]);
  sen[plane + t] = fabs(pt[4] - 2.0 * pt[0] + pt[3]) / fabs(pt[4] + 2.0 * pt[0] + pt[3]);
  const double dv = (v1[2] - v1[1]) / (2.0 * g.dx) + (v2[4] - v2[3]) / (2.0 * g.dy);
  const double cv = (v2[2] - v2[1]) / (2.0 * g.dx) - (v1[4] - v1[3]) / (2.0 * g.dy);
  sen[2 * plane + t] = fmax(-dv / sqrt(dv * dv + cv * cv + 1e-40), 0.0);
  sen[3 * plane + t] = fabs(b1[2] - b1[1] + b2[4] - b2[3]) / (fabs(b1[0] + b2[0]) + 1e-40);
}

// ------------------------------------------------------------ point values
// One direction of the point update along a 5-point line w0..w4 at offsets
// -h, -h/2, 0, h/2, h through the point (w2 = U0, evaluation e0):
//   R  = D+F+ + D-F-, F+- = (F +- alpha U)/2, alpha = max spectral radius
//      = [F0 - 4F1 + 4F3 - F4 + alpha (w0 - 4w1 + 6w2 - 4w3 + w4)] / (2h)
//   dB = (D+B_n + D-B_n)/2 = (B0 - 4B1 + 4B3 - B4) / (2h)
//   G  = F^LLF(U0, w4) - F^LLF(w0, U0) (neighbours of the first-order scheme)
//   jl = B_n(w4) - B_n(w0)
template <class Load>
__device__ __forceinline__ void line_fvs(const Geo& g, int dir, double h, const double U0[NV], const DirEval& e0,
                                         Load load, double R[NV], double& dB, double G[NV], double& jl) {
  double SF[NV], SW[NV], w[NV];
  DirEval ew;
  double alpha = e0.sr;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    SF[c] = 0.0;
    SW[c] = 6.0 * U0[c];
  }
  const int bn = 4 + dir;
  dB = 0.0;
  // m = 0 and m = 4 are also the LLF neighbours
  load(0, w);
  eval_dir(w, g, dir, ew);
  alpha = fmax(alpha, ew.sr);
  {
    const double al = alpha_llf(ew, e0, w, U0);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      SF[c] += ew.F[c];
      SW[c] += w[c];
      G[c] = -0.5 * (ew.F[c] + e0.F[c] - al * (U0[c] - w[c]));
    }
    dB += w[bn];
    jl = -w[bn];
  }
  load(4, w);
  eval_dir(w, g, dir, ew);
  alpha = fmax(alpha, ew.sr);
  {
    const double al = alpha_llf(e0, ew, U0, w);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      SF[c] -= ew.F[c];
      SW[c] += w[c];
      G[c] += 0.5 * (e0.F[c] + ew.F[c] - al * (w[c] - U0[c]));
    }
    dB -= w[bn];
    jl += w[bn];
  }
  load(1, w);
  eval_dir(w, g, dir, ew);
  alpha = fmax(alpha, ew.sr);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    SF[c] -= 4.0 * ew.F[c];
    SW[c] -= 4.0 * w[c];
  }
  dB -= 4.0 * w[bn];
  load(3, w);
  eval_dir(w, g, dir, ew);
  alpha = fmax(alpha, ew.sr);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    SF[c] += 4.0 * ew.F[c];
    SW[c] -= 4.0 * w[c];
  }
  dB += 4.0 * w[bn];
  const double s = 0.5 / h;
#pragma unroll
  for (int c = 0; c < NV; ++c) R[c] = (SF[c] + alpha * SW[c]) * s;
  dB *= s;
}

// Central direction (the face points across their face): R = (F(up) - F(dn))/h,
// dB = (B_n(up) - B_n(dn))/h, LLF neighbours dn and up.
__device__ __forceinline__ void line_central(const Geo& g, int dir, double h, const double U0[NV], const DirEval& e0,
                                             const double dn[NV], const double up[NV], double R[NV], double& dB,
                                             double G[NV], double& jl) {
  DirEval ed, eu;
  eval_dir(dn, g, dir, ed);
  eval_dir(up, g, dir, eu);
  const double ad = alpha_llf(ed, e0, dn, U0), au = alpha_llf(e0, eu, U0, up);
  const double rh = 1.0 / h;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    R[c] = (eu.F[c] - ed.F[c]) * rh;
    G[c] = 0.5 * (e0.F[c] + eu.F[c] - au * (up[c] - U0[c])) - 0.5 * (ed.F[c] + e0.F[c] - ad * (U0[c] - dn[c]));
  }
  const int bn = 4 + dir;
  dB = (up[bn] - dn[bn]) * rh;
  jl = up[bn] - dn[bn];
}

// Assemble the high-order and LLF states, limit, combine, store.
__device__ __forceinline__ void finish_point(const Geo& g, const double U0[NV], const double R1[NV], double dB1,
                                             const double G1[NV], double jl1, const double R2[NV], double dB2,
                                             const double G2[NV], double jl2, double dt, double ca, double cb,
                                             const double* un, double* out, long plane, long off, Counters* cn) {
  double P[NV];
  psi(U0, P);
  const double divH = dB1 + dB2;
  const double divL = 0.5 * (jl1 * g.rdx + jl2 * g.rdy);
  const double lx = dt * g.rdx, ly = dt * g.rdy;
  double UH[NV], UL[NV], W[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    UH[c] = U0[c] + dt * (-R1[c] - R2[c] - divH * P[c]);
    UL[c] = U0[c] - lx * G1[c] - ly * G2[c] - dt * divL * P[c];
  }
  if (!in_G(UL, g.gm1)) count(&cn->n_llf_not_admissible);
  limit_point(UH, UL, g.gm1, W, cn);
  if (!in_G(W, g.gm1)) count(&cn->n_not_admissible);
  if (ca == 0.0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c * plane + off] = W[c];
  } else {
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c * plane + off] = ca * un[c * plane + off] + cb * W[c];
  }
}

// Vertex V(k,l): FVS in x (V, Y, V, Y, V) and in y (V, X, V, X, V).
__global__ __launch_bounds__(BLK) void k_vertex(Geo g, CState u, const double* __restrict__ un, double* out,
                                                const double* dtp, double ca, double cb, Counters* cn) {
  const int t = blockIdx.x * BLK + threadIdx.x;
  if (t >= g.nxp * g.nyp) return;
  const int k = t % g.nxp, l = t / g.nxp;
  const double dt = *dtp;
  double U0[NV], R1[NV], G1[NV], R2[NV], G2[NV], dB1, dB2, jl1, jl2;
  ldV(g, u.v, k, l, U0);
  DirEval e0;
  eval_dir(U0, g, 0, e0);
  line_fvs(g, 0, g.dx, U0, e0, [&](int m, double* w) {
    if (m == 0) ldV(g, u.v, k - 1, l, w);
    else if (m == 1) ldY(g, u.y, k - 1, l, w);
    else if (m == 3) ldY(g, u.y, k, l, w);
    else ldV(g, u.v, k + 1, l, w);
  }, R1, dB1, G1, jl1);
  eval_dir(U0, g, 1, e0);
  line_fvs(g, 1, g.dy, U0, e0, [&](int m, double* w) {
    if (m == 0) ldV(g, u.v, k, l - 1, w);
    else if (m == 1) ldX(g, u.x, k, l - 1, w);
    else if (m == 3) ldX(g, u.x, k, l, w);
    else ldV(g, u.v, k, l + 1, w);
  }, R2, dB2, G2, jl2);
  finish_point(g, U0, R1, dB1, G1, jl1, R2, dB2, G2, jl2, dt, ca, cb, un, out, g.sv, t, cn);
}

// Vertical face X(k,j): FVS in x (X, C, X, C, X), central in y (V(k,j), V(k,j+1)).
__global__ __launch_bounds__(BLK) void k_xface(Geo g, CState u, const double* __restrict__ centre,
                                               const double* __restrict__ un, double* out, const double* dtp,
                                               double ca, double cb, Counters* cn) {
  const int t = blockIdx.x * BLK + threadIdx.x;
  if (t >= g.nxp * g.ny) return;
  const int k = t % g.nxp, j = t / g.nxp;
  const double dt = *dtp;
  double U0[NV], R1[NV], G1[NV], R2[NV], G2[NV], dB1, dB2, jl1, jl2;
  ldX(g, u.x, k, j, U0);
  DirEval e0;
  eval_dir(U0, g, 0, e0);
  line_fvs(g, 0, g.dx, U0, e0, [&](int m, double* w) {
    if (m == 0) ldX(g, u.x, k - 1, j, w);
    else if (m == 1) ldC(g, centre, k - 1, j, w);
    else if (m == 3) ldC(g, centre, k, j, w);
    else ldX(g, u.x, k + 1, j, w);
  }, R1, dB1, G1, jl1);
  eval_dir(U0, g, 1, e0);
  double dn[NV], up[NV];
  ldV(g, u.v, k, j, dn);
  ldV(g, u.v, k, j + 1, up);
  line_central(g, 1, g.dy, U0, e0, dn, up, R2, dB2, G2, jl2);
  finish_point(g, U0, R1, dB1, G1, jl1, R2, dB2, G2, jl2, dt, ca, cb, un, out, g.sx, t, cn);
}

// Horizontal face Y(i,l): central in x (V(i,l), V(i+1,l)), FVS in y (Y, C, Y, C, Y).
__global__ __launch_bounds__(BLK) void k_yface(Geo g, CState u, const double* __restrict__ centre,
                                               const double* __restrict__ un, double* out, const double* dtp,
                                               double ca, double cb, Counters* cn) {
  const int t = blockIdx.x * BLK + threadIdx.x;
  if (t >= g.nx * g.nyp) return;
  const int i = t % g.nx, l = t / g.nx;
  const double dt = *dtp;
  double U0[NV], R1[NV], G1[NV], R2[NV], G2[NV], dB1, dB2, jl1, jl2;
  ldY(g, u.y, i, l, U0);
  DirEval e0;
  eval_dir(U0, g, 0, e0);
  double dn[NV], up[NV];
  ldV(g, u.v, i, l, dn);
  ldV(g, u.v, i + 1, l, up);
  line_central(g, 0, g.dx, U0, e0, dn, up, R1, dB1, G1, jl1);
  eval_dir(U0, g, 1, e0);
  line_fvs(g, 1, g.dy, U0, e0, [&](int m, double* w) {
    if (m == 0) ldY(g, u.y, i, l - 1, w);
    else if (m == 1) ldC(g, centre, i, l - 1, w);
    else if (m == 3) ldC(g, centre, i, l, w);
    else ldY(g, u.y, i, l + 1, w);
  }, R2, dB2, G2, jl2);
  finish_point(g, U0, R1, dB1, G1, jl1, R2, dB2, G2, jl2, dt, ca, cb, un, out, g.sy, t, cn);
}

// ---------------------------------------------------------------- interfaces
__device__ __forceinline__ double sensor_theta(const Geo& g, const Ext& e, const double* sen, int iL, int jL,
                                               int iR, int jR, int dir) {
  const long plane = (long)e.snx * e.sny;
  const long a = (long)ext_sj(e, g, jL) * e.snx + ext_si(e, g, iL);
  const long b = (long)ext_sj(e, g, jR) * e.snx + ext_si(e, g, iR);
  const double p1 = fmax(sen[dir * plane + a], sen[dir * plane + b]);
  const double p2 = fmax(sen[2 * plane + a], sen[2 * plane + b]);
  const double p3 = fmax(sen[3 * plane + a], sen[3 * plane + b]);
  return exp(-g.kappa * (p1 * p2 + p3));
}

// x-interface k of row j (dir 0) or y-interface l of column i (dir 1):
// Simpson flux over the edge's three point values, LLF flux of the two
// adjacent cell averages, sensor coefficient, sensor-blended flux.
__global__ __launch_bounds__(BLK) void k_iface(Geo g, Ext e, CState u, const double* __restrict__ sen, int dir,
                                               double* __restrict__ fs, double* __restrict__ fl,
                                               double* __restrict__ ft) {
  const int t = blockIdx.x * BLK + threadIdx.x;
  const int W = dir ? e.cnx : e.fnx, H = dir ? e.fny : e.cny;
  if (t >= W * H) return;
  const int a = t % W, b = t / W;
  double w0[NV], w1[NV], w2[NV], Fh[NV], F[NV];
  int iL, jL, iR, jR;
  if (dir == 0) {
    const int k = e.fx0 + a, j = e.cy0 + b;
    ldV(g, u.v, k, j, w0);
    ldX(g, u.x, k, j, w1);
    ldV(g, u.v, k, j + 1, w2);
    iL = k - 1; jL = j; iR = k; jR = j;
  } else {
    const int i = e.cx0 + a, l = e.fy0 + b;
    ldV(g, u.v, i, l, w0);
    ldY(g, u.y, i, l, w1);
    ldV(g, u.v, i + 1, l, w2);
    iL = i; jL = l - 1; iR = i; jR = l;
  }
  flux_dir(w0, g.gm1, dir, Fh);
  flux_dir(w1, g.gm1, dir, F);
#pragma unroll
  for (int c = 0; c < NV; ++c) Fh[c] += 4.0 * F[c];
  flux_dir(w2, g.gm1, dir, F);
  constexpr double sixth = 1.0 / 6.0;
#pragma unroll
  for (int c = 0; c < NV; ++c) Fh[c] = (Fh[c] + F[c]) * sixth;
  DirEval eL, eR;
  ldA(g, u.a, iL, jL, w0);
  ldA(g, u.a, iR, jR, w1);
  eval_dir(w0, g, dir, eL);
  eval_dir(w1, g, dir, eR);
  const double al = alpha_llf(eL, eR, w0, w1);
  const double ts = sensor_theta(g, e, sen, iL, jL, iR, jR, dir);
  const long plane = (long)W * H;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const double llf = 0.5 * (eL.F[c] + eR.F[c] - al * (w1[c] - w0[c]));
    fl[c * plane + t] = llf;
    fs[c * plane + t] = ts * Fh[c] + (1.0 - ts) * llf;
  }
  ft[t] = ts;
}

// ----------------------------------------------------------- cell limiter
__device__ __forceinline__ void ld_iface(const double* base, long plane, long off, double f[NV]) {
  load8(base, plane, off, f);
}

// Nine-point Powell source of the cell (eq. semi_av_src): Simpson weights
// (1/6, 2/3, 1/6) per direction, divergence from the one-sided / central
// differences of eq. (2d_fd) along the cell's rows and columns.
__device__ void cell_source(const Geo& g, CState u, const double* centre, int i, int j, double S[NV]) {
  double B1[3][3], B2[3][3];  // [a][b]: a along x, b along y
  double Pv[3][3][NV];        // Psi at the nine points
  double U[NV];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (b == 1 && a == 1) ldC(g, centre, i, j, U);
      else if (b == 1) ldX(g, u.x, i + a / 2, j, U);
      else if (a == 1) ldY(g, u.y, i, j + b / 2, U);
      else ldV(g, u.v, i + a / 2, j + b / 2, U);
      B1[a][b] = U[4];
      B2[a][b] = U[5];
      psi(U, Pv[a][b]);
    }
  const double w[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
#pragma unroll
  for (int c = 0; c < NV; ++c) S[c] = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double dx1 = a == 0 ? (-3.0 * B1[0][b] + 4.0 * B1[1][b] - B1[2][b])
                       : a == 1 ? (B1[2][b] - B1[0][b])
                                : (B1[0][b] - 4.0 * B1[1][b] + 3.0 * B1[2][b]);
      const double dy2 = b == 0 ? (-3.0 * B2[a][0] + 4.0 * B2[a][1] - B2[a][2])
                       : b == 1 ? (B2[a][2] - B2[a][0])
                                : (B2[a][0] - 4.0 * B2[a][1] + 3.0 * B2[a][2]);
      const double f = w[a] * w[b] * (dx1 * g.rdx + dy2 * g.rdy);
#pragma unroll
      for (int c = 1; c < NV; ++c) S[c] += f * Pv[a][b][c];
    }
}

__global__ __launch_bounds__(BLK) void k_cell_limit(Geo g, Ext e, CState u, const double* __restrict__ centre,
                                                    WS ws, const double* dtp, Counters* cn) {
  const int t = blockIdx.x * BLK + threadIdx.x;
  if (t >= e.cnx * e.cny) return;
  const int i = e.cx0 + t % e.cnx, j = e.cy0 + t / e.cnx;
  const bool interior = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
  const double dt = *dtp;
  const double lx = dt * g.rdx, ly = dt * g.rdy;
  // interface data
  const long pfx = (long)e.fnx * e.cny, pfy = (long)e.cnx * e.fny;
  const int cj = ext_cj(e, g, j), ci = ext_ci(e, g, i);
  const long oL = (long)cj * e.fnx + ext_x(e, g, i), oR = (long)cj * e.fnx + ext_x(e, g, i + 1);
  const long oD = (long)ext_y(e, g, j) * e.cnx + ci, oU = (long)ext_y(e, g, j + 1) * e.cnx + ci;
  const double tsij = fmin(fmin(ws.fxt[oL], ws.fxt[oR]), fmin(ws.fyt[oD], ws.fyt[oU]));
  double A[NV], S[NV], Sl[NV], P[NV], Allf[NV], Asrc[NV];
  ldA(g, u.a, i, j, A);
  cell_source(g, u, centre, i, j, S);
  double Al[NV], Ar[NV];
  ldA(g, u.a, i - 1, j, Al);
  ldA(g, u.a, i + 1, j, Ar);
  double divb = (Ar[4] - Al[4]) * (0.5 * g.rdx);
  ldA(g, u.a, i, j - 1, Al);
  ldA(g, u.a, i, j + 1, Ar);
  divb += (Ar[5] - Al[5]) * (0.5 * g.rdy);
  psi(A, P);
  double H[4][NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const double fLs = ws.fxs[c * pfx + oL], fLl = ws.fxl[c * pfx + oL];
    const double fRs = ws.fxs[c * pfx + oR], fRl = ws.fxl[c * pfx + oR];
    const double fDs = ws.fys[c * pfy + oD], fDl = ws.fyl[c * pfy + oD];
    const double fUs = ws.fys[c * pfy + oU], fUl = ws.fyl[c * pfy + oU];
    Sl[c] = divb * P[c];
    S[c] = tsij * S[c] + (1.0 - tsij) * Sl[c];
    const double G = A[c] - lx * (fRl - fLl) - ly * (fUl - fDl);
    Allf[c] = G - dt * Sl[c];
    Asrc[c] = G - dt * S[c];
    H[0][c] = lx * (fLs - fLl);
    H[1][c] = -lx * (fRs - fRl);
    H[2][c] = ly * (fDs - fDl);
    H[3][c] = -ly * (fUs - fUl);
  }
  const double rhoL = Allf[0], pL = pressure(Allf, g.gm1);
  if (interior && !(rhoL > 0.0 && pL > 0.0)) count(&cn->n_llf_not_admissible);
  const double er = fmin(EPS_FLOOR, rhoL), ep = fmin(EPS_FLOOR, pL);
  // step (1): limit the source
  double th = 1.0;
  const double psrc = pressure(Asrc, g.gm1);
  if (psrc < ep) {
    th = (pL - ep) / (pL - psrc);
    if (interior) count(&cn->n_source_limited);
  }
  double A1[NV];
  auto make = [&](double tt, double* Wt) {
#pragma unroll
    for (int c = 0; c < NV; ++c) Wt[c] = tt * Asrc[c] + (1.0 - tt) * Allf[c];
  };
  make(th, A1);
  if (th > 0.0 && !in_G(A1, g.gm1)) {
    if (interior) count(&cn->n_fallback);
    th = shrink_into_G(th, g.gm1, make, cn, interior);
    make(th, A1);
  }
  // step (2): the box of admissible coefficients
  double Lam[4];
  limiter_box(A1, H, g.gm1, er, ep, Lam, cn, interior);
  const long pc = (long)e.cnx * e.cny;
#pragma unroll
  for (int I = 0; I < 4; ++I) ws.lam[I * pc + t] = Lam[I];
#pragma unroll
  for (int c = 0; c < NV; ++c) ws.slim[c * pc + t] = th * S[c] + (1.0 - th) * Sl[c];
}

// Step (3): unique interface coefficients theta = min of the two cells'
// Lambda, then the limited update in flux form and the SSP combination.
__global__ __launch_bounds__(BLK) void k_cell_final(Geo g, Ext e, CState u, WS ws, const double* __restrict__ un,
                                                    double* out, const double* dtp, double ca, double cb,
                                                    Counters* cn) {
  const int t = blockIdx.x * BLK + threadIdx.x;
  if (t >= g.nx * g.ny) return;
  const int i = t % g.nx, j = t / g.nx;
  const double dt = *dtp;
  const double lx = dt * g.rdx, ly = dt * g.rdy;
  const long pc = (long)e.cnx * e.cny;
  auto lam = [&](int ii, int jj, int I) {
    return ws.lam[I * pc + (long)ext_cj(e, g, jj) * e.cnx + ext_ci(e, g, ii)];
  };
  const double thL = fmin(lam(i - 1, j, 1), lam(i, j, 0));
  const double thR = fmin(lam(i, j, 1), lam(i + 1, j, 0));
  const double thD = fmin(lam(i, j - 1, 3), lam(i, j, 2));
  const double thU = fmin(lam(i, j, 3), lam(i, j + 1, 2));
  if (thL < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thL); }
  if (thD < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thD); }
  if (g.bcx && i == g.nx - 1 && thR < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thR); }
  if (g.bcy && j == g.ny - 1 && thU < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thU); }
  const long pfx = (long)e.fnx * e.cny, pfy = (long)e.cnx * e.fny;
  const int cj = ext_cj(e, g, j), ci = ext_ci(e, g, i);
  const long oL = (long)cj * e.fnx + ext_x(e, g, i), oR = (long)cj * e.fnx + ext_x(e, g, i + 1);
  const long oD = (long)ext_y(e, g, j) * e.cnx + ci, oU = (long)ext_y(e, g, j + 1) * e.cnx + ci;
  const long oc = (long)cj * e.cnx + ci;
  double An[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const double FL = thL * ws.fxs[c * pfx + oL] + (1.0 - thL) * ws.fxl[c * pfx + oL];
    const double FR = thR * ws.fxs[c * pfx + oR] + (1.0 - thR) * ws.fxl[c * pfx + oR];
    const double FD = thD * ws.fys[c * pfy + oD] + (1.0 - thD) * ws.fyl[c * pfy + oD];
    const double FU = thU * ws.fys[c * pfy + oU] + (1.0 - thU) * ws.fyl[c * pfy + oU];
    An[c] = u.a[c * g.sc + t] - lx * (FR - FL) - ly * (FU - FD) - dt * ws.slim[c * pc + oc];
  }
  if (!in_G(An, g.gm1)) count(&cn->n_not_admissible);
  if (ca == 0.0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c * g.sc + t] = An[c];
  } else {
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c * g.sc + t] = ca * un[c * g.sc + t] + cb * An[c];
  }
}

// ------------------------------------------------------------- reductions
// Max over all DoFs of rho_1/dx + rho_2/dy, two passes (deterministic).
constexpr int RED_BLOCKS = 1024;

__device__ __forceinline__ double block_max(double v) {
  __shared__ double sh[BLK / 64];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BLK / 64; ++w) v = fmax(v, sh[w]);
    sh[0] = v;
  }
  __syncthreads();
  v = sh[0];
  __syncthreads();
  return v;
}

__device__ __forceinline__ void dof_ptr(const Geo& g, CState u, long t, const double*& base, long& plane, long& off) {
  if (t < g.sc) { base = u.a; plane = g.sc; off = t; return; }
  t -= g.sc;
  if (t < g.sx) { base = u.x; plane = g.sx; off = t; return; }
  t -= g.sx;
  if (t < g.sy) { base = u.y; plane = g.sy; off = t; return; }
  t -= g.sy;
  base = u.v; plane = g.sv; off = t;
}

__global__ __launch_bounds__(BLK) void k_dt_partial(Geo g, CState u, double* partial) {
  const long n = g.sc + g.sx + g.sy + g.sv;
  double m = 0.0;
  for (long t = (long)blockIdx.x * BLK + threadIdx.x; t < n; t += (long)gridDim.x * BLK) {
    const double* base;
    long plane, off;
    dof_ptr(g, u, t, base, plane, off);
    double U[NV];
    load8(base, plane, off, U);
    DirEval e;
    eval_dir(U, g, 0, e);
    const double s1 = e.sr;
    eval_dir(U, g, 1, e);
    m = fmax(m, s1 * g.rdx + e.sr * g.rdy);
  }
  m = block_max(m);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(BLK) void k_dt_final(const double* partial, int nparts, double cfl, double t_rem,
                                                  double* dt) {
  double m = 0.0;
  for (int t = threadIdx.x; t < nparts; t += BLK) m = fmax(m, partial[t]);
  m = block_max(m);
  if (threadIdx.x == 0) {
    double d = cfl / m;
    *dt = d > t_rem ? t_rem : d;
  }
}

// Statistics: min rho, min p, number of DoFs outside G, sum of cell densities.
__global__ __launch_bounds__(BLK) void k_stats_partial(Geo g, CState u, double* partial) {
  const long n = g.sc + g.sx + g.sy + g.sv;
  double mr = 1e300, mp = 1e300, bad = 0.0, mass = 0.0;
  for (long t = (long)blockIdx.x * BLK + threadIdx.x; t < n; t += (long)gridDim.x * BLK) {
    const double* base;
    long plane, off;
    dof_ptr(g, u, t, base, plane, off);
    double U[NV];
    load8(base, plane, off, U);
    const double p = pressure(U, g.gm1);
    mr = fmin(mr, U[0]);
    mp = fmin(mp, p);
    bad += (U[0] > 0.0 && p > 0.0) ? 0.0 : 1.0;
    if (t < g.sc) mass += U[0];
  }
  __shared__ double sh[4][BLK];
  sh[0][threadIdx.x] = mr;
  sh[1][threadIdx.x] = mp;
  sh[2][threadIdx.x] = bad;
  sh[3][threadIdx.x] = mass;
  __syncthreads();
  for (int s = BLK / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + s]);
      sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + s]);
      sh[2][threadIdx.x] += sh[2][threadIdx.x + s];
      sh[3][threadIdx.x] += sh[3][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[threadIdx.x * gridDim.x + blockIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_zero_counters(Counters* cn) {
  if (threadIdx.x == 0) {
    cn->n_llf_not_admissible = cn->n_newton = cn->newton_iters_max = cn->n_fallback = cn->n_not_admissible = 0;
    cn->n_theta_active = cn->n_point_limited = cn->n_centre_limited = cn->n_source_limited = 0;
    cn->min_theta_bits = (unsigned long long)__double_as_longlong(1.0);
  }
}

inline int nblocks(long n) { return (int)((n + BLK - 1) / BLK); }

}  // namespace

// =================================================================== C ABI
struct af_mhd_ctx {
  Geo g;
  Ext e;
  WS ws;
  hipStream_t stream;
  std::string err;
};

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool valid_params(const af_mhd_params* p) {
  if (!p) return false;
  if (p->nx < 4 || p->ny < 4 || p->nx > (1 << 16) || p->ny > (1 << 16)) return false;
  if (!(p->x1 > p->x0) || !(p->y1 > p->y0) || !(p->gamma > 1.0)) return false;
  if (!(p->cfl > 0.0 && p->cfl <= 1.0) || !(p->kappa >= 0.0)) return false;
  if ((p->bc_x != AF_BC_PERIODIC && p->bc_x != AF_BC_OUTFLOW) ||
      (p->bc_y != AF_BC_PERIODIC && p->bc_y != AF_BC_OUTFLOW))
    return false;
  return p->flags == 0;
}

void make_geo(const af_mhd_params* p, Geo& g, Ext& e) {
  g.nx = p->nx;
  g.ny = p->ny;
  g.bcx = p->bc_x;
  g.bcy = p->bc_y;
  g.nxp = p->nx + (g.bcx ? 1 : 0);
  g.nyp = p->ny + (g.bcy ? 1 : 0);
  g.dx = (p->x1 - p->x0) / p->nx;
  g.dy = (p->y1 - p->y0) / p->ny;
  g.rdx = 1.0 / g.dx;
  g.rdy = 1.0 / g.dy;
  g.gamma = p->gamma;
  g.gm1 = p->gamma - 1.0;
  g.kappa = p->kappa;
  g.cfl = p->cfl;
  g.sc = (long)g.nx * g.ny;
  g.sx = (long)g.nxp * g.ny;
  g.sy = (long)g.nx * g.nyp;
  g.sv = (long)g.nxp * g.nyp;
  e.cx0 = g.bcx ? -1 : 0;
  e.cnx = g.nx + (g.bcx ? 2 : 0);
  e.cy0 = g.bcy ? -1 : 0;
  e.cny = g.ny + (g.bcy ? 2 : 0);
  e.sx0 = g.bcx ? -2 : 0;
  e.snx = g.nx + (g.bcx ? 4 : 0);
  e.sy0 = g.bcy ? -2 : 0;
  e.sny = g.ny + (g.bcy ? 4 : 0);
  e.fx0 = g.bcx ? -1 : 0;
  e.fnx = g.nx + (g.bcx ? 3 : 0);
  e.fy0 = g.bcy ? -1 : 0;
  e.fny = g.ny + (g.bcy ? 3 : 0);
}

// Workspace layout; with base == nullptr only the size is computed.
size_t layout(const Geo& g, const Ext& e, char* base, WS* ws) {
  size_t off = 0;
  auto take = [&](size_t doubles) {
    double* ptr = base ? reinterpret_cast<double*>(base + off) : nullptr;
    off += align256(doubles * sizeof(double));
    return ptr;
  };
  WS w;
  w.centre = take(8 * g.sc);
  w.sensor = take(4 * (size_t)e.snx * e.sny);
  w.fxs = take(8 * (size_t)e.fnx * e.cny);
  w.fxl = take(8 * (size_t)e.fnx * e.cny);
  w.fxt = take((size_t)e.fnx * e.cny);
  w.fys = take(8 * (size_t)e.cnx * e.fny);
  w.fyl = take(8 * (size_t)e.cnx * e.fny);
  w.fyt = take((size_t)e.cnx * e.fny);
  w.lam = take(4 * (size_t)e.cnx * e.cny);
  w.slim = take(8 * (size_t)e.cnx * e.cny);
  w.partial = take(4 * (size_t)RED_BLOCKS);
  w.cnt = reinterpret_cast<Counters*>(take(sizeof(Counters) / sizeof(double) + 1));
  const size_t sizes[4] = {(size_t)g.sc, (size_t)g.sx, (size_t)g.sy, (size_t)g.sv};
  for (int s = 0; s < 2; ++s)
    for (int q = 0; q < 4; ++q) w.scratch[s][q] = take(8 * sizes[q]);
  if (ws) *ws = w;
  return off;
}

int fail(af_mhd_ctx* c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}

int check_hip(af_mhd_ctx* c, const char* where) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return AF_OK;
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return AF_EHIP;
}

bool aligned8(const void* p) { return p && ((uintptr_t)p & 7) == 0; }
bool valid_state(const af_mhd_state* s) {
  return s && aligned8(s->cell) && aligned8(s->xface) && aligned8(s->yface) && aligned8(s->vert);
}
CState cstate(const af_mhd_state* s) { return CState{s->cell, s->xface, s->yface, s->vert}; }

int run_stage(af_mhd_ctx* c, int k, const af_mhd_state* un, const af_mhd_state* uk, af_mhd_state* out,
              const double* dt_dev) {
  static const double A[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double B[3] = {1.0, 0.25, 2.0 / 3.0};
  const Geo& g = c->g;
  const Ext& e = c->e;
  const WS& ws = c->ws;
  hipStream_t s = c->stream;
  const CState u = cstate(uk);
  const double ca = A[k], cb = B[k];
  const af_mhd_state* n = k == 0 ? uk : un;
  k_centre<<<nblocks(g.sc), BLK, 0, s>>>(g, u, ws.centre, ws.cnt);
  k_sensor<<<nblocks((long)e.snx * e.sny), BLK, 0, s>>>(g, e, u, ws.sensor);
  k_vertex<<<nblocks(g.sv), BLK, 0, s>>>(g, u, n->vert, out->vert, dt_dev, ca, cb, ws.cnt);
  k_xface<<<nblocks(g.sx), BLK, 0, s>>>(g, u, ws.centre, n->xface, out->xface, dt_dev, ca, cb, ws.cnt);
  k_yface<<<nblocks(g.sy), BLK, 0, s>>>(g, u, ws.centre, n->yface, out->yface, dt_dev, ca, cb, ws.cnt);
  k_iface<<<nblocks((long)e.fnx * e.cny), BLK, 0, s>>>(g, e, u, ws.sensor, 0, ws.fxs, ws.fxl, ws.fxt);
  k_iface<<<nblocks((long)e.cnx * e.fny), BLK, 0, s>>>(g, e, u, ws.sensor, 1, ws.fys, ws.fyl, ws.fyt);
  k_cell_limit<<<nblocks((long)e.cnx * e.cny), BLK, 0, s>>>(g, e, u, ws.centre, ws, dt_dev, ws.cnt);
  k_cell_final<<<nblocks(g.sc), BLK, 0, s>>>(g, e, u, ws, n->cell, out->cell, dt_dev, ca, cb, ws.cnt);
  return check_hip(c, "stage launch");
}

int run_dt(af_mhd_ctx* c, const af_mhd_state* u, double t_rem, double* dt_dev) {
  const Geo& g = c->g;
  const long n = g.sc + g.sx + g.sy + g.sv;
  const int nb = (int)std::min<long>(RED_BLOCKS, std::max<long>(1, nblocks(n)));
  k_dt_partial<<<nb, BLK, 0, c->stream>>>(g, cstate(u), c->ws.partial);
  k_dt_final<<<1, BLK, 0, c->stream>>>(c->ws.partial, nb, g.cfl, t_rem, dt_dev);
  return check_hip(c, "dt launch");
}

}  // namespace

extern "C" {

size_t af_mhd_workspace_bytes(const af_mhd_params* p) {
  if (!valid_params(p)) return 0;
  Geo g;
  Ext e;
  make_geo(p, g, e);
  return layout(g, e, nullptr, nullptr);
}

int af_mhd_init(const af_mhd_params* p, void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                af_mhd_ctx** out) {
  if (!out) return AF_EINVAL;
  if (!valid_params(p)) return AF_EINVAL;
  if (!workspace_dev || ((uintptr_t)workspace_dev & 255)) return AF_EINVAL;
  af_mhd_ctx* c = new (std::nothrow) af_mhd_ctx();
  if (!c) return AF_EINVAL;
  make_geo(p, c->g, c->e);
  const size_t need = layout(c->g, c->e, nullptr, nullptr);
  if (workspace_bytes < need) {
    delete c;
    return AF_EWORKSPACE;
  }
  layout(c->g, c->e, static_cast<char*>(workspace_dev), &c->ws);
  c->stream = static_cast<hipStream_t>(hip_stream);
  k_zero_counters<<<1, 64, 0, c->stream>>>(c->ws.cnt);
  const int rc = check_hip(c, "init");
  if (rc != AF_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return AF_OK;
}

int af_mhd_dt(af_mhd_ctx* c, const af_mhd_state* u, double t_remaining, double* dt_dev) {
  if (!c) return AF_EINVAL;
  if (!valid_state(u) || !aligned8(dt_dev) || !(t_remaining > 0.0)) return fail(c, AF_EINVAL, "af_mhd_dt: bad argument");
  return run_dt(c, u, t_remaining, dt_dev);
}

int af_mhd_stage(af_mhd_ctx* c, int k, const af_mhd_state* un, const af_mhd_state* uk, af_mhd_state* out,
                 const double* dt_dev) {
  if (!c) return AF_EINVAL;
  if (k < 0 || k > 2 || !valid_state(uk) || !valid_state(out) || !aligned8(dt_dev) || (k > 0 && !valid_state(un)))
    return fail(c, AF_EINVAL, "af_mhd_stage: bad argument");
  if (out->cell == uk->cell || out->xface == uk->xface || out->yface == uk->yface || out->vert == uk->vert)
    return fail(c, AF_EINVAL, "af_mhd_stage: out aliases uk");
  return run_stage(c, k, un, uk, out, dt_dev);
}

int af_mhd_step(af_mhd_ctx* c, af_mhd_state* u, double t_remaining, double* dt_dev) {
  if (!c) return AF_EINVAL;
  if (!valid_state(u) || !aligned8(dt_dev) || !(t_remaining > 0.0)) return fail(c, AF_EINVAL, "af_mhd_step: bad argument");
  af_mhd_state s1{c->ws.scratch[0][0], c->ws.scratch[0][1], c->ws.scratch[0][2], c->ws.scratch[0][3]};
  af_mhd_state s2{c->ws.scratch[1][0], c->ws.scratch[1][1], c->ws.scratch[1][2], c->ws.scratch[1][3]};
  int rc = run_dt(c, u, t_remaining, dt_dev);
  if (rc == AF_OK) rc = run_stage(c, 0, u, u, &s1, dt_dev);
  if (rc == AF_OK) rc = run_stage(c, 1, u, &s1, &s2, dt_dev);
  if (rc == AF_OK) rc = run_stage(c, 2, u, &s2, u, dt_dev);
  return rc;
}

int af_mhd_reset_counters(af_mhd_ctx* c) {
  if (!c) return AF_EINVAL;
  k_zero_counters<<<1, 64, 0, c->stream>>>(c->ws.cnt);
  return check_hip(c, "reset counters");
}

int af_mhd_stats(af_mhd_ctx* c, const af_mhd_state* u, af_mhd_stats_t* out) {
  if (!c) return AF_EINVAL;
  if (!valid_state(u) || !out) return fail(c, AF_EINVAL, "af_mhd_stats: bad argument");
  const Geo& g = c->g;
  const long n = g.sc + g.sx + g.sy + g.sv;
  const int nb = (int)std::min<long>(RED_BLOCKS, std::max<long>(1, nblocks(n)));
  k_stats_partial<<<nb, BLK, 0, c->stream>>>(g, cstate(u), c->ws.partial);
  int rc = check_hip(c, "stats launch");
  if (rc != AF_OK) return rc;
  double* host = new (std::nothrow) double[4 * nb];
  if (!host) return fail(c, AF_EINVAL, "af_mhd_stats: out of host memory");
  Counters cn;
  hipError_t e = hipMemcpyAsync(host, c->ws.partial, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&cn, c->ws.cnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete[] host;
    c->err = std::string("af_mhd_stats: ") + hipGetErrorString(e);
    return AF_EHIP;
  }
  double mr = 1e300, mp = 1e300, bad = 0.0, mass = 0.0;
  for (int b = 0; b < nb; ++b) {
    mr = std::min(mr, host[b]);
    mp = std::min(mp, host[nb + b]);
    bad += host[2 * nb + b];
    mass += host[3 * nb + b];
  }
  delete[] host;
  out->min_rho = mr;
  out->min_p = mp;
  out->mass = mass * g.dx * g.dy;
  double mt;
  std::memcpy(&mt, &cn.min_theta_bits, sizeof(double));
  out->min_theta = mt;
  out->n_llf_not_admissible = (int64_t)cn.n_llf_not_admissible;
  out->n_newton = (int64_t)cn.n_newton;
  out->newton_iters_max = (int64_t)cn.newton_iters_max;
  out->n_fallback = (int64_t)cn.n_fallback;
  out->n_not_admissible = (int64_t)cn.n_not_admissible;
  out->n_theta_active = (int64_t)cn.n_theta_active;
  out->n_point_limited = (int64_t)cn.n_point_limited;
  out->n_centre_limited = (int64_t)cn.n_centre_limited;
  out->n_source_limited = (int64_t)cn.n_source_limited;
  out->n_dof_not_admissible = (int64_t)bad;
  c->err.clear();
  return bad > 0.0 ? AF_ENOTADMISSIBLE : AF_OK;
}

void af_mhd_destroy(af_mhd_ctx* c) { delete c; }

const char* af_mhd_last_error(const af_mhd_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
