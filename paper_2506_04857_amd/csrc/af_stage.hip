// af_stage.hip -- kernels of one SSP-RK3 stage of the PP Active Flux scheme
// for 2D ideal MHD with the Godunov-Powell source (gfx950), and the C ABI
// declared in include/af_mhd.h.
//
// A stage (forward Euler on U^(k), then out = a_k U^n + b_k FE) is two
// launches that read only U^(k) (and U^n for the combination):
//   k_points  point values (Section 2.3): centre values (Section 2.1,
//             remark rmk:cell_center), LLF flux-vector splitting with the
//             central div B source, first-order LLF safe state and scaling
//             limiter (Section 3.3), SSP combination
//   k_cells   cell averages (Sections 2.2, 3.1-3.4): Simpson and LLF fluxes,
//             shock sensor, nine-point and LLF Powell sources, parametrized
//             flux limiter, limited update in flux form, SSP combination
// Both are LDS-tiled: every derived quantity a tile needs is computed once
// per tile and shared through LDS; there are no HBM intermediates.
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

struct WS {                 // workspace pointers
  double* partial;          // reduction partials
  Counters* cnt;
  double* scratch[2][4];    // two RK scratch states
};

// Centre value of cell (i,j) from the bi-parabolic reconstruction
// (Section 2.1): C = [36 A - 4 (face values) - (vertex values)] / 16, then
// limited towards A (remark rmk:cell_center).  Also returns the nine sample
// points of the cell through the callback keep(a, b, U) (a along x, b along y).
template <class Keep>
__device__ __forceinline__ void centre_and_points(const Geo& g, CState u, int i, int j, const double A[NV],
                                                  double C[NV], Counters* cn, bool counted, Keep keep) {
  double w[NV], Uc[NV], f[NV];
  ldX(g, u.x, i, j, w);
  keep(0, 1, w);
#pragma unroll
  for (int q = 0; q < NV; ++q) f[q] = w[q];
  ldX(g, u.x, i + 1, j, w);
  keep(2, 1, w);
#pragma unroll
  for (int q = 0; q < NV; ++q) f[q] += w[q];
  ldY(g, u.y, i, j, w);
  keep(1, 0, w);
#pragma unroll
  for (int q = 0; q < NV; ++q) Uc[q] = w[q];
  ldY(g, u.y, i, j + 1, w);
  keep(1, 2, w);
#pragma unroll
  for (int q = 0; q < NV; ++q) f[q] = -4.0 * (f[q] + (Uc[q] + w[q]));
  ldV(g, u.v, i, j, w);
  keep(0, 0, w);
#pragma unroll
  for (int q = 0; q < NV; ++q) Uc[q] = w[q];
  ldV(g, u.v, i + 1, j, w);
  keep(2, 0, w);
#pragma unroll
  for (int q = 0; q < NV; ++q) Uc[q] += w[q];
  double v2[NV];
  ldV(g, u.v, i, j + 1, v2);
  keep(0, 2, v2);
  ldV(g, u.v, i + 1, j + 1, w);
  keep(2, 2, w);
#pragma unroll
  for (int q = 0; q < NV; ++q) Uc[q] = (36.0 * A[q] + f[q] - (Uc[q] + (v2[q] + w[q]))) * 0.0625;
  limit_centre(Uc, A, g.gm1, C, cn, counted);
}

__device__ double sensor_pressure(const double U[NV], double gamma) {
#pragma clang fp contract(off)
  const double m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
  const double b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  return (gamma - 1.0) * (U[7] - m2 / (2.0 * U[0]) - b2 / 2.0);
}

// ------------------------------------------------------- fused point update
// One launch updates the point values V, X, Y owned by a tile of
// (PB-2) x (PB-2) cells (cell (i,j) owns V(i,j), X(i,j), Y(i,j)); the
// PB x PB threads cover the tile plus a one-cell ring.  The point-value
// stencils of Section 2.3 run along four families of lines of the
// half-spaced lattice:
//   a  horizontal lines through V and Y  (V: FVS in x; Y: central in x)
//   b  vertical lines through V and X    (V: FVS in y; X: central in y)
//   c  horizontal lines through X and C  (X: FVS in x)
//   d  vertical lines through Y and C    (Y: FVS in y)
// For each family every point is evaluated once (flux, spectral radius,
// c_f, v_n, sqrt(rho)) and shared through LDS.  FVS in direction n at a
// point with line neighbours w0..w4 (offsets -h, -h/2, 0, h/2, h):
//   R = D+F+ + D-F- = [F0 - 4F1 + 4F3 - F4 + alpha (w0 - 4w1 + 6w2 - 4w3 + w4)] / (2h)
//   alpha = max spectral radius over the five, div part (B0 - 4B1 + 4B3 - B4)/(2h).
// Central direction: R = (F(up) - F(dn))/h, div part (B(up) - B(dn))/h.
// The first-order LLF state uses the four neighbours of the point (the
// line neighbours at +-h for FVS directions, at +-h/2 for the central one).
constexpr int PB = 16, PNT = PB * PB;
constexpr int RF = 12;  // record: F[8], sr, cf, vn, sq

__device__ __forceinline__ void put_rec(double (*s)[PB][PB], int base, int ty, int tx, const DirEval& e) {
#pragma unroll
  for (int c = 0; c < NV; ++c) s[base + c][ty][tx] = e.F[c];
  s[base + 8][ty][tx] = e.sr;
  s[base + 9][ty][tx] = e.cf;
  s[base + 10][ty][tx] = e.vn;
  s[base + 11][ty][tx] = e.sq;
}
__device__ __forceinline__ void get_rec(double (*s)[PB][PB], int base, int ty, int tx, DirEval& e) {
#pragma unroll
  for (int c = 0; c < NV; ++c) e.F[c] = s[base + c][ty][tx];
  e.sr = s[base + 8][ty][tx];
  e.cf = s[base + 9][ty][tx];
  e.vn = s[base + 10][ty][tx];
  e.sq = s[base + 11][ty][tx];
}

// Incremental FVS along a line (own point e0/U0 at offset 0).  Outer
// neighbours (offsets -h, +h) are also the LLF neighbours; inner ones
// (-h/2, +h/2) enter the FVS sums only.  R = (SF + alpha SW)/(2h).
struct LineAcc {
  double SF[NV], SW[NV], G[NV];
  double alpha, dB, jl;
};

__device__ __forceinline__ void line_begin(LineAcc& L, const DirEval& e0, const double U0[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    L.SF[c] = 0.0;
    L.SW[c] = 6.0 * U0[c];
    L.G[c] = 0.0;
  }
  L.alpha = e0.sr;
  L.dB = 0.0;
  L.jl = 0.0;
}

// side = -1 for the neighbour at -h (left/below), +1 at +h.
__device__ __forceinline__ void line_outer(LineAcc& L, int bn, int side, const DirEval& e, const double U[NV],
                                           const DirEval& e0, const double U0[NV]) {
  L.alpha = fmax(L.alpha, e.sr);
  const double al = side < 0 ? alpha_llf(e, e0, U, U0) : alpha_llf(e0, e, U0, U);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    L.SF[c] -= side * e.F[c];
    L.SW[c] += U[c];
    // F^LLF(U0, U) for side +1, -F^LLF(U, U0) for side -1
    L.G[c] += side < 0 ? -0.5 * (e.F[c] + e0.F[c] - al * (U0[c] - U[c]))
                       : 0.5 * (e0.F[c] + e.F[c] - al * (U[c] - U0[c]));
  }
  L.dB -= side * U[bn];
  L.jl += side * U[bn];
}

__device__ __forceinline__ void line_inner(LineAcc& L, int bn, int side, const DirEval& e, const double U[NV]) {
  L.alpha = fmax(L.alpha, e.sr);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    L.SF[c] += side * 4.0 * e.F[c];
    L.SW[c] -= 4.0 * U[c];
  }
  L.dB += side * 4.0 * U[bn];
}

// Point accumulators: high-order RHS h = -R_x - R_y with the div part, and
// the LLF update l = -dt/dx G_x - dt/dy G_y with its div part.
struct PointAcc {
  double h[NV], l[NV];
  double divh, divl;
};

__device__ __forceinline__ void acc_fvs(PointAcc& P, const LineAcc& L, double rh, double lam) {
  const double s = 0.5 * rh;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    P.h[c] -= (L.SF[c] + L.alpha * L.SW[c]) * s;
    P.l[c] -= lam * L.G[c];
  }
  P.divh += L.dB * s;
  P.divl += L.jl * s;
}

// Central direction across a face point: neighbours dn/up at -h/2, +h/2;
// they are also its LLF neighbours.
__device__ __forceinline__ void acc_central(PointAcc& P, int bn, double rh, double lam, const DirEval& ed,
                                            const double dn[NV], const DirEval& e0, const double U0[NV],
                                            const DirEval& eu, const double up[NV]) {
  const double ad = alpha_llf(ed, e0, dn, U0), au = alpha_llf(e0, eu, U0, up);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    P.h[c] -= (eu.F[c] - ed.F[c]) * rh;
    const double G = 0.5 * (e0.F[c] + eu.F[c] - au * (up[c] - U0[c])) - 0.5 * (ed.F[c] + e0.F[c] - ad * (U0[c] - dn[c]));
    P.l[c] -= lam * G;
  }
  P.divh += (up[bn] - dn[bn]) * rh;
  P.divl += 0.5 * rh * (up[bn] - dn[bn]);
}

__device__ __forceinline__ void acc_zero(PointAcc& P) {
#pragma unroll
  for (int c = 0; c < NV; ++c) P.h[c] = P.l[c] = 0.0;
  P.divh = P.divl = 0.0;
}

// High-order and LLF states from the accumulators, scaling limiter, SSP
// combination, store.
__device__ __forceinline__ void finish(const Geo& g, double dt, const double U0[NV], const PointAcc& P, double ca,
                                      double cb, const double* __restrict__ un, double* __restrict__ out, long plane,
                                      long off, Counters* cn) {
  double Ps[NV], UH[NV], UL[NV], W[NV];
  psi(U0, Ps);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    UH[c] = U0[c] + dt * (P.h[c] - P.divh * Ps[c]);
    UL[c] = U0[c] + P.l[c] - dt * P.divl * Ps[c];
  }
  if (!in_G(UL, g.gm1)) count(&cn->n_llf_not_admissible);
  limit_point(UH, UL, g.gm1, W, cn, true);
  if (!in_G(W, g.gm1)) count(&cn->n_not_admissible);
  if (ca == 0.0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c * plane + off] = W[c];
  } else {
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c * plane + off] = ca * un[c * plane + off] + cb * W[c];
  }
}

__device__ __forceinline__ int clamp_pt(int i, int np) { return i < -1 ? -1 : (i > np ? np : i); }

// LDS layout of k_points (fields of PB x PB doubles): raw states of the
// tile's V, X, Y and centre values, then two directional records.
constexpr int SV_ = 0, SX_ = 8, SY_ = 16, SC_ = 24, SR0 = 32, SR1 = 32 + RF, SFIELDS = 32 + 2 * RF;

__device__ __forceinline__ void lds8(double (*s)[PB][PB], int base, int ty, int tx, double U[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) U[c] = s[base + c][ty][tx];
}

__global__ __launch_bounds__(PNT) void k_points(Geo g, CState u, CState un, MState out, const double* dtp, double ca,
                                                double cb, Counters* cn) {
  __shared__ double s[SFIELDS][PB][PB];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i0 = (int)blockIdx.x * (PB - 2) - 1, j0 = (int)blockIdx.y * (PB - 2) - 1;
  const int i = clamp_pt(i0 + tx, g.nxp), j = clamp_pt(j0 + ty, g.nyp);
  const bool inner = tx >= 1 && tx < PB - 1 && ty >= 1 && ty < PB - 1;
  const bool outV = inner && i0 + tx < g.nxp && j0 + ty < g.nyp;
  const bool outX = inner && i0 + tx < g.nxp && j0 + ty < g.ny;
  const bool outY = inner && i0 + tx < g.nx && j0 + ty < g.nyp;
  const double dt = *dtp;
  const double lx = dt * g.rdx, ly = dt * g.rdy;
  const int txl = tx > 0 ? tx - 1 : tx, txr = tx < PB - 1 ? tx + 1 : tx;
  const int tyd = ty > 0 ? ty - 1 : ty, tyu = ty < PB - 1 ? ty + 1 : ty;

  // 0: the tile's raw point values into LDS
  {
    double w[NV];
    ldV(g, u.v, i, j, w);
#pragma unroll
    for (int c = 0; c < NV; ++c) s[SV_ + c][ty][tx] = w[c];
    ldX(g, u.x, i, j, w);
#pragma unroll
    for (int c = 0; c < NV; ++c) s[SX_ + c][ty][tx] = w[c];
    ldY(g, u.y, i, j, w);
#pragma unroll
    for (int c = 0; c < NV; ++c) s[SY_ + c][ty][tx] = w[c];
  }
  __syncthreads();
  // 1: centre values (the last column/row's are never used)
  {
    double A[NV], Uc[NV], f[NV], w[NV], q[NV], C[NV];
    ldA(g, u.a, i, j, A);
    lds8(s, SX_, ty, tx, f);
    lds8(s, SX_, ty, txr, w);
    lds8(s, SY_, ty, tx, Uc);
    lds8(s, SY_, tyu, tx, q);
#pragma unroll
    for (int c = 0; c < NV; ++c) f[c] = -4.0 * ((f[c] + w[c]) + (Uc[c] + q[c]));
    lds8(s, SV_, ty, tx, Uc);
    lds8(s, SV_, ty, txr, w);
#pragma unroll
    for (int c = 0; c < NV; ++c) Uc[c] += w[c];
    lds8(s, SV_, tyu, tx, q);
    lds8(s, SV_, tyu, txr, w);
#pragma unroll
    for (int c = 0; c < NV; ++c) Uc[c] = (36.0 * A[c] + f[c] - (Uc[c] + (q[c] + w[c]))) * 0.0625;
    limit_centre(Uc, A, g.gm1, C, cn, inner && i0 + tx < g.nx && j0 + ty < g.ny);
#pragma unroll
    for (int c = 0; c < NV; ++c) s[SC_ + c][ty][tx] = C[c];
  }
  PointAcc PA, PB_;
  DirEval e0, e1, en;
  double U0[NV], U1[NV], Un[NV];
  LineAcc L;

  // b: vertical lines through V and X.  V: FVS in y over V(l-1), X(l-1), V,
  // X(l), V(l+1).  X: central in y between V(k,j) and V(k,j+1).
  lds8(s, SV_, ty, tx, U0);
  lds8(s, SX_, ty, tx, U1);
  eval_dir(U0, g, 1, e0);
  eval_dir(U1, g, 1, e1);
  put_rec(s, SR0, ty, tx, e0);
  put_rec(s, SR1, ty, tx, e1);
  __syncthreads();
  acc_zero(PA);  // V
  acc_zero(PB_); // X
  line_begin(L, e0, U0);
  get_rec(s, SR0, tyd, tx, en);
  lds8(s, SV_, tyd, tx, Un);
  line_outer(L, 5, -1, en, Un, e0, U0);
  get_rec(s, SR1, tyd, tx, en);
  lds8(s, SX_, tyd, tx, Un);
  line_inner(L, 5, -1, en, Un);
  line_inner(L, 5, +1, e1, U1);
  get_rec(s, SR0, tyu, tx, en);
  lds8(s, SV_, tyu, tx, Un);
  line_outer(L, 5, +1, en, Un, e0, U0);
  acc_fvs(PA, L, g.rdy, ly);
  acc_central(PB_, 5, g.rdy, ly, e0, U0, e1, U1, en, Un);
  __syncthreads();

  // a: horizontal lines through V and Y.  V: FVS in x over V(k-1), Y(k-1),
  // V, Y(k), V(k+1) -> V complete.  Y: central in x between V(i,l), V(i+1,l).
  lds8(s, SY_, ty, tx, U1);
  eval_dir(U0, g, 0, e0);
  eval_dir(U1, g, 0, e1);
  put_rec(s, SR0, ty, tx, e0);
  put_rec(s, SR1, ty, tx, e1);
  __syncthreads();
  line_begin(L, e0, U0);
  get_rec(s, SR0, ty, txl, en);
  lds8(s, SV_, ty, txl, Un);
  line_outer(L, 4, -1, en, Un, e0, U0);
  get_rec(s, SR1, ty, txl, en);
  lds8(s, SY_, ty, txl, Un);
  line_inner(L, 4, -1, en, Un);
  line_inner(L, 4, +1, e1, U1);
  get_rec(s, SR0, ty, txr, en);
  lds8(s, SV_, ty, txr, Un);
  line_outer(L, 4, +1, en, Un, e0, U0);
  acc_fvs(PA, L, g.rdx, lx);
  if (outV) finish(g, dt, U0, PA, ca, cb, un.v, out.v, g.sv, (long)j * g.nxp + i, cn);
  acc_zero(PA);  // now Y
  acc_central(PA, 4, g.rdx, lx, e0, U0, e1, U1, en, Un);
  __syncthreads();

  // c: horizontal lines through X and C.  X: FVS in x over X(k-1), C(k-1),
  // X, C(k), X(k+1) -> X complete.
  lds8(s, SX_, ty, tx, U0);
  lds8(s, SC_, ty, tx, Un);
  eval_dir(U0, g, 0, e0);
  eval_dir(Un, g, 0, e1);
  put_rec(s, SR0, ty, tx, e0);
  put_rec(s, SR1, ty, tx, e1);
  __syncthreads();
  line_begin(L, e0, U0);
  line_inner(L, 4, +1, e1, Un);
  get_rec(s, SR0, ty, txl, en);
  lds8(s, SX_, ty, txl, Un);
  line_outer(L, 4, -1, en, Un, e0, U0);
  get_rec(s, SR1, ty, txl, en);
  lds8(s, SC_, ty, txl, Un);
  line_inner(L, 4, -1, en, Un);
  get_rec(s, SR0, ty, txr, en);
  lds8(s, SX_, ty, txr, Un);
  line_outer(L, 4, +1, en, Un, e0, U0);
  acc_fvs(PB_, L, g.rdx, lx);
  if (outX) finish(g, dt, U0, PB_, ca, cb, un.x, out.x, g.sx, (long)j * g.nxp + i, cn);
  __syncthreads();

  // d: vertical lines through Y and C.  Y: FVS in y over Y(l-1), C(l-1), Y,
  // C(l), Y(l+1) -> Y complete.
  lds8(s, SC_, ty, tx, Un);
  eval_dir(U1, g, 1, e0);
  eval_dir(Un, g, 1, e1);
  put_rec(s, SR0, ty, tx, e0);
  put_rec(s, SR1, ty, tx, e1);
  __syncthreads();
  line_begin(L, e0, U1);
  line_inner(L, 5, +1, e1, Un);
  get_rec(s, SR0, tyd, tx, en);
  lds8(s, SY_, tyd, tx, Un);
  line_outer(L, 5, -1, en, Un, e0, U1);
  get_rec(s, SR1, tyd, tx, en);
  lds8(s, SC_, tyd, tx, Un);
  line_inner(L, 5, -1, en, Un);
  get_rec(s, SR0, tyu, tx, en);
  lds8(s, SY_, tyu, tx, Un);
  line_outer(L, 5, +1, en, Un, e0, U1);
  acc_fvs(PA, L, g.rdy, ly);
  if (outY) finish(g, dt, U1, PA, ca, cb, un.y, out.y, g.sy, (long)j * g.nx + i, cn);
}

// ------------------------------------------------------ fused cell update
// One launch computes the cell averages of the stage for a tile of
// (CBX-3) x (CBY-3) cells; the block's CBX x CBY threads cover the cells
// whose flux-limiter box is needed plus one trailing row/column whose left
// and bottom interfaces close the region.  Per thread (cell (i,j)):
//   1  shock-sensor indicators of the block's cells and one ring (LDS)
//   2  x-interface at the cell's left: Simpson flux, LLF flux, sensor blend;
//      exchanged through LDS so each cell has both of its x-interfaces
//   3  the same for the bottom y-interface
//   4  nine-point and LLF sources, flux-limiter steps (1)-(2) -> Lambda
//   5  Lambda exchanged through LDS, unique interface coefficients, and the
//      limited update in flux form written as
//        A^new = G - dt S^Lim + sum_I theta_I H_I,
//      G = A - dt/dx (F^LLF_R - F^LLF_L) - dt/dy (F^LLF_U - F^LLF_D),
//      H_L = dt/dx (F^s_L - F^LLF_L), H_R = -dt/dx (F^s_R - F^LLF_R), ...
constexpr int CBX = 32, CBY = 16, CNT = CBX * CBY;
constexpr int XF = 20;  // exchange fields: directional record (12) + state (8)

// Sensor primitives of one cell from its average: total pressure, v1, v2,
// B1, B2 (contraction-free, true divisions, as the indicators need).
__device__ void sensor_prims(const double U[NV], double gamma, double q[5]) {
#pragma clang fp contract(off)
  q[0] = sensor_pressure(U, gamma) + (U[4] * U[4] + U[5] * U[5] + U[6] * U[6]) / 2.0;
  q[1] = U[1] / U[0];
  q[2] = U[2] / U[0];
  q[3] = U[4];
  q[4] = U[5];
}

// Indicators from the primitives of the cell (c) and its neighbours
// l, r (x) and d, u (y): phi1x, phi1y, phi2, phi3.
__device__ void sensor_from_prims(const double c[5], const double l[5], const double r[5], const double d[5],
                                  const double u[5], double dx, double dy, double phi[4]) {
#pragma clang fp contract(off)
  phi[0] = fabs(r[0] - 2.0 * c[0] + l[0]) / fabs(r[0] + 2.0 * c[0] + l[0]);
  phi[1] = fabs(u[0] - 2.0 * c[0] + d[0]) / fabs(u[0] + 2.0 * c[0] + d[0]);
  const double dv = (r[1] - l[1]) / (2.0 * dx) + (u[2] - d[2]) / (2.0 * dy);
  const double cv = (r[2] - l[2]) / (2.0 * dx) - (u[1] - d[1]) / (2.0 * dy);
  phi[2] = fmax(-dv / sqrt(dv * dv + cv * cv + 1e-40), 0.0);
  phi[3] = fabs(r[3] - l[3] + u[4] - d[4]) / (fabs(c[3] + c[4]) + 1e-40);
}

// Nine-point Powell source of cell (i,j), eq. (semi_av_src): weights
// (1/6, 2/3, 1/6) per direction, the divergence at each sample point from
// the one-sided / central differences of eq. (2d_fd) along the cell's rows
// and columns, Psi at each point; the centre value is the limited one.
__device__ void cell_source(const Geo& g, CState u, int i, int j, const double A[NV], double S[NV]) {
  double B1[3][3], B2[3][3], C[NV];  // [a][b]: a along x, b along y
  centre_and_points(g, u, i, j, A, C, nullptr, false, [&](int a, int b, const double* w) {
    B1[a][b] = w[4];
    B2[a][b] = w[5];
  });
  B1[1][1] = C[4];
  B2[1][1] = C[5];
  const double wq[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
#pragma unroll
  for (int c = 0; c < NV; ++c) S[c] = 0.0;
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double dx1 = a == 0 ? (-3.0 * B1[0][b] + 4.0 * B1[1][b] - B1[2][b])
                       : a == 1 ? (B1[2][b] - B1[0][b])
                                : (B1[0][b] - 4.0 * B1[1][b] + 3.0 * B1[2][b]);
      const double dy2 = b == 0 ? (-3.0 * B2[a][0] + 4.0 * B2[a][1] - B2[a][2])
                       : b == 1 ? (B2[a][2] - B2[a][0])
                                : (B2[a][0] - 4.0 * B2[a][1] + 3.0 * B2[a][2]);
      const double f = wq[a] * wq[b] * (dx1 * g.rdx + dy2 * g.rdy);
      double w[NV], P[NV];
      if (a == 1 && b == 1) {
#pragma unroll
        for (int c = 0; c < NV; ++c) w[c] = C[c];
      } else if (b == 1) {
        ldX(g, u.x, i + a / 2, j, w);
      } else if (a == 1) {
        ldY(g, u.y, i, j + b / 2, w);
      } else {
        ldV(g, u.v, i + a / 2, j + b / 2, w);
      }
      psi(w, P);
#pragma unroll
      for (int c = 1; c < NV; ++c) S[c] += f * P[c];
    }
}

__device__ __forceinline__ int clamp_cell(int i, int n) { return i < -2 ? -2 : (i > n + 1 ? n + 1 : i); }
// Sensor primitives are needed on cells [-3, n+2]: the indicators of the
// ghost cells -2 and n+1 enter the sensor of the outermost interfaces whose
// flux-limiter coefficients the boundary cells take.
__device__ __forceinline__ int clamp_prim(int i, int n) { return i < -3 ? -3 : (i > n + 2 ? n + 2 : i); }

__device__ __forceinline__ void put_xrec(double (*s)[CBY][CBX], int ty, int tx, const DirEval& e, const double U[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) s[c][ty][tx] = e.F[c];
  s[8][ty][tx] = e.sr;
  s[9][ty][tx] = e.cf;
  s[10][ty][tx] = e.vn;
  s[11][ty][tx] = e.sq;
#pragma unroll
  for (int c = 0; c < NV; ++c) s[12 + c][ty][tx] = U[c];
}
__device__ __forceinline__ void get_xrec(double (*s)[CBY][CBX], int ty, int tx, DirEval& e, double U[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) e.F[c] = s[c][ty][tx];
  e.sr = s[8][ty][tx];
  e.cf = s[9][ty][tx];
  e.vn = s[10][ty][tx];
  e.sq = s[11][ty][tx];
#pragma unroll
  for (int c = 0; c < NV; ++c) U[c] = s[12 + c][ty][tx];
}

// Simpson flux over the edge points w0, w1, w2 (Section 2.2), LLF flux of
// the adjacent averages (eq. 2d_llf_flux) and the sensor blend: returns
// F^LLF and dF = theta^s (F_simpson - F^LLF).
__device__ __forceinline__ void interface_flux(const Geo& g, int dir, const double w0[NV], const double w1[NV],
                                               const double w2[NV], const DirEval& eL, const double AL[NV],
                                               const DirEval& eR, const double AR[NV], double ts, double Fl[NV],
                                               double dF[NV]) {
  double Fh[NV], F[NV];
  flux_dir(w0, g.gm1, dir, Fh);
  flux_dir(w1, g.gm1, dir, F);
#pragma unroll
  for (int c = 0; c < NV; ++c) Fh[c] += 4.0 * F[c];
  flux_dir(w2, g.gm1, dir, F);
  constexpr double sixth = 1.0 / 6.0;
#pragma unroll
  for (int c = 0; c < NV; ++c) Fh[c] = (Fh[c] + F[c]) * sixth;
  const double al = alpha_llf(eL, eR, AL, AR);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    Fl[c] = 0.5 * (eL.F[c] + eR.F[c] - al * (AR[c] - AL[c]));
    dF[c] = ts * Fh[c] + (1.0 - ts) * Fl[c] - Fl[c];
  }
}

__device__ __forceinline__ double sensor_theta(double kappa, const double* a, const double* b, int dir) {
  const double p1 = fmax(a[dir], b[dir]), p2 = fmax(a[2], b[2]), p3 = fmax(a[3], b[3]);
  return exp(-kappa * (p1 * p2 + p3));
}

__global__ __launch_bounds__(CNT) void k_cells(Geo g, CState u, const double* __restrict__ un,
                                               double* __restrict__ out, const double* dtp, double ca, double cb,
                                               Counters* cn) {
  __shared__ double s_x[XF][CBY][CBX];
  __shared__ double s_phi[CBY + 1][CBX + 1][4];
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * CBX + tx;
  const int i0 = (int)blockIdx.x * (CBX - 3) - 1, j0 = (int)blockIdx.y * (CBY - 3) - 1;
  const int i = clamp_cell(i0 + tx, g.nx), j = clamp_cell(j0 + ty, g.ny);
  const bool output = tx >= 1 && tx < CBX - 2 && ty >= 1 && ty < CBY - 2 && i0 + tx < g.nx && j0 + ty < g.ny;
  const double dt = *dtp;
  const double lx = dt * g.rdx, ly = dt * g.rdy;

  // 1a: sensor primitives on [i0-2, i0+CBX+1) x [j0-2, j0+CBY+1), aliased
  //     onto the exchange buffer
  constexpr int PW = CBX + 3, PH = CBY + 3;
  double* prim = &s_x[0][0][0];
  for (int it = tid; it < PW * PH; it += CNT) {
    const int a = it % PW, b = it / PW;
    double U[NV], q[5];
    ldA(g, u.a, clamp_prim(i0 - 2 + a, g.nx), clamp_prim(j0 - 2 + b, g.ny), U);
    sensor_prims(U, g.gamma, q);
#pragma unroll
    for (int m = 0; m < 5; ++m) prim[m * PW * PH + it] = q[m];
  }
  __syncthreads();
  // 1b: indicators on [i0-1, i0+CBX) x [j0-1, j0+CBY)
  for (int it = tid; it < (CBX + 1) * (CBY + 1); it += CNT) {
    const int a = it % (CBX + 1), b = it / (CBX + 1);
    const int pc = (b + 1) * PW + (a + 1);
    double c[5], l[5], r[5], d[5], up[5], ph[4];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const double* pm = prim + m * PW * PH;
      c[m] = pm[pc];
      l[m] = pm[pc - 1];
      r[m] = pm[pc + 1];
      d[m] = pm[pc - PW];
      up[m] = pm[pc + PW];
    }
    sensor_from_prims(c, l, r, d, up, g.dx, g.dy, ph);
#pragma unroll
    for (int q = 0; q < 4; ++q) s_phi[b][a][q] = ph[q];
  }
  __syncthreads();

  double A[NV], G[NV], H[4][NV], w0[NV], w1[NV], w2[NV], AN[NV], Fl[NV], dF[NV];
  DirEval eA, eN;
  double tsmin;
  ldA(g, u.a, i, j, A);
  // 2: x-interfaces.  The cell's own evaluation is shared with its right
  //    neighbour; the interface at the cell's left is computed here and
  //    shared with the left neighbour.
  eval_dir(A, g, 0, eA);
  put_xrec(s_x, ty, tx, eA, A);
  __syncthreads();
  if (tx > 0) {
    get_xrec(s_x, ty, tx - 1, eN, AN);
  } else {
    ldA(g, u.a, i - 1, j, AN);
    eval_dir(AN, g, 0, eN);
  }
  ldV(g, u.v, i, j, w0);
  ldX(g, u.x, i, j, w1);
  ldV(g, u.v, i, j + 1, w2);
  double ts = sensor_theta(g.kappa, s_phi[ty + 1][tx], s_phi[ty + 1][tx + 1], 0);
  tsmin = ts;
  interface_flux(g, 0, w0, w1, w2, eN, AN, eA, A, ts, Fl, dF);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    s_x[c][ty][tx] = Fl[c];
    s_x[NV + c][ty][tx] = dF[c];
    G[c] = A[c] + lx * Fl[c];
    H[0][c] = lx * dF[c];
  }
  __syncthreads();
  {
    const int tr = tx + 1 < CBX ? tx + 1 : tx;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      G[c] -= lx * s_x[c][ty][tr];
      H[1][c] = -lx * s_x[NV + c][ty][tr];
    }
    tsmin = fmin(tsmin, sensor_theta(g.kappa, s_phi[ty + 1][tx + 1], s_phi[ty + 1][tx + 2 <= CBX ? tx + 2 : CBX], 0));
  }
  __syncthreads();
  // 3: y-interfaces, the same with the neighbour below/above
  eval_dir(A, g, 1, eA);
  put_xrec(s_x, ty, tx, eA, A);
  __syncthreads();
  if (ty > 0) {
    get_xrec(s_x, ty - 1, tx, eN, AN);
  } else {
    ldA(g, u.a, i, j - 1, AN);
    eval_dir(AN, g, 1, eN);
  }
  ldV(g, u.v, i, j, w0);
  ldY(g, u.y, i, j, w1);
  ldV(g, u.v, i + 1, j, w2);
  ts = sensor_theta(g.kappa, s_phi[ty][tx + 1], s_phi[ty + 1][tx + 1], 1);
  tsmin = fmin(tsmin, ts);
  interface_flux(g, 1, w0, w1, w2, eN, AN, eA, A, ts, Fl, dF);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    s_x[c][ty][tx] = Fl[c];
    s_x[NV + c][ty][tx] = dF[c];
    G[c] += ly * Fl[c];
    H[2][c] = ly * dF[c];
  }
  __syncthreads();
  {
    const int tu = ty + 1 < CBY ? ty + 1 : ty;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      G[c] -= ly * s_x[c][tu][tx];
      H[3][c] = -ly * s_x[NV + c][tu][tx];
    }
    tsmin = fmin(tsmin, sensor_theta(g.kappa, s_phi[ty + 1][tx + 1], s_phi[ty + 2 <= CBY ? ty + 2 : CBY][tx + 1], 1));
  }
  // 4: sources and flux-limiter steps (1)-(2)
  double S[NV], Sl[NV], Allf[NV], Asrc[NV];
  cell_source(g, u, i, j, A, S);
  {
    double P[NV], b;
    ldA(g, u.a, i + 1, j, AN);
    b = AN[4];
    ldA(g, u.a, i - 1, j, AN);
    double divb = (b - AN[4]) * (0.5 * g.rdx);
    ldA(g, u.a, i, j + 1, AN);
    b = AN[5];
    ldA(g, u.a, i, j - 1, AN);
    divb += (b - AN[5]) * (0.5 * g.rdy);
    psi(A, P);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      Sl[c] = divb * P[c];
      S[c] = tsmin * S[c] + (1.0 - tsmin) * Sl[c];
      Allf[c] = G[c] - dt * Sl[c];
      Asrc[c] = G[c] - dt * S[c];
    }
  }
  const double rhoL = Allf[0];
  const bool llf_in = in_G(Allf, g.gm1);
  if (output && !llf_in) count(&cn->n_llf_not_admissible);
  const double er = fmin(EPS_FLOOR, rhoL);
  double ep = EPS_FLOOR, th = 1.0;
  double A1[NV];
  if (!(rhoL > 0.0 && p_at_least(Allf, EPS_FLOOR, g.gm1) && p_at_least(Asrc, EPS_FLOOR, g.gm1))) {
    // step (1) of the flux limiter may act: exact pressures
    const double pL = pressure(Allf, g.gm1);
    ep = fmin(EPS_FLOOR, pL);
    const double psrc = pressure(Asrc, g.gm1);
    if (psrc < ep) {
      th = (pL - ep) / (pL - psrc);
      if (output) count(&cn->n_source_limited);
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
  if (th > 0.0 && !in_G(A1, g.gm1)) {
    if (output) count(&cn->n_fallback);
    th = shrink_into_G(th, g.gm1, make);
    make(th, A1);
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) S[c] = th * S[c] + (1.0 - th) * Sl[c];  // S^Lim
  double Lam[4];
  limiter_box(A1, H, g.gm1, er, ep, Lam, cn, output);
  // 5: unique interface coefficients and the limited update
  __syncthreads();
#pragma unroll
  for (int I = 0; I < 4; ++I) s_x[I][ty][tx] = Lam[I];
  __syncthreads();
  if (!output) return;
  const double thL = fmin(s_x[1][ty][tx - 1], Lam[0]);
  const double thR = fmin(Lam[1], s_x[0][ty][tx + 1]);
  const double thD = fmin(s_x[3][ty - 1][tx], Lam[2]);
  const double thU = fmin(Lam[3], s_x[2][ty + 1][tx]);
  if (thL < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thL); }
  if (thD < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thD); }
  if (g.bcx && i == g.nx - 1 && thR < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thR); }
  if (g.bcy && j == g.ny - 1 && thU < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thU); }
  double An[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c)
    An[c] = G[c] - dt * S[c] + thL * H[0][c] + thR * H[1][c] + thD * H[2][c] + thU * H[3][c];
  if (!in_G(An, g.gm1)) count(&cn->n_not_admissible);
  const long off = (long)j * g.nx + i;
  if (ca == 0.0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c * g.sc + off] = An[c];
  } else {
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c * g.sc + off] = ca * un[c * g.sc + off] + cb * An[c];
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

void make_geo(const af_mhd_params* p, Geo& g) {
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
}

// Workspace layout; with base == nullptr only the size is computed.
size_t layout(const Geo& g, char* base, WS* ws) {
  size_t off = 0;
  auto take = [&](size_t doubles) {
    double* ptr = base ? reinterpret_cast<double*>(base + off) : nullptr;
    off += align256(doubles * sizeof(double));
    return ptr;
  };
  WS w;
  w.partial = take(4 * (size_t)RED_BLOCKS);
  w.cnt = reinterpret_cast<Counters*>(take(sizeof(Counters) / sizeof(double) + 1));
  const size_t sizes[4] = {(size_t)g.sc, (size_t)g.sx, (size_t)g.sy, (size_t)g.sv};
  for (int k = 0; k < 2; ++k)
    for (int q = 0; q < 4; ++q) w.scratch[k][q] = take(8 * sizes[q]);
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
  hipStream_t s = c->stream;
  const CState u = cstate(uk);
  const CState n = cstate(k == 0 ? uk : un);  // not read when a_k = 0
  const MState o{out->cell, out->xface, out->yface, out->vert};
  const dim3 pgrid((g.nxp + PB - 3) / (PB - 2), (g.nyp + PB - 3) / (PB - 2));
  k_points<<<pgrid, dim3(PB, PB), 0, s>>>(g, u, n, o, dt_dev, A[k], B[k], c->ws.cnt);
  const dim3 cgrid((g.nx + CBX - 4) / (CBX - 3), (g.ny + CBY - 4) / (CBY - 3));
  k_cells<<<cgrid, dim3(CBX, CBY), 0, s>>>(g, u, n.a, o.a, dt_dev, A[k], B[k], c->ws.cnt);
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
  make_geo(p, g);
  return layout(g, nullptr, nullptr);
}

int af_mhd_init(const af_mhd_params* p, void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                af_mhd_ctx** out) {
  if (!out) return AF_EINVAL;
  if (!valid_params(p)) return AF_EINVAL;
  if (!workspace_dev || ((uintptr_t)workspace_dev & 255)) return AF_EINVAL;
  af_mhd_ctx* c = new (std::nothrow) af_mhd_ctx();
  if (!c) return AF_EINVAL;
  make_geo(p, c->g);
  const size_t need = layout(c->g, nullptr, nullptr);
  if (workspace_bytes < need) {
    delete c;
    return AF_EWORKSPACE;
  }
  layout(c->g, static_cast<char*>(workspace_dev), &c->ws);
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
