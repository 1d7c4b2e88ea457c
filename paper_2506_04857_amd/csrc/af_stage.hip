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
  double* centre;           // limited centre values of the stage input, [8][ny][nx]
};

// XCD-aware tile order: the hardware deals consecutive workgroups round-robin
// to the 8 XCDs, each with its own L2.  Workgroup b takes logical tile
// (b % 8) * per + b / 8, so every XCD walks one contiguous band of tiles in
// row-major order and the halos its tiles share stay in its L2.  Returns
// false for the padding workgroups of the last band.
constexpr int NXCD = 8;
__device__ __forceinline__ bool xcd_tile(int ntx, int nty, int& bx, int& by) {
  const int n = ntx * nty, per = (n + NXCD - 1) / NXCD;
  const int b = (int)blockIdx.x;
  const int t = (b % NXCD) * per + b / NXCD;
  if (t >= n) return false;
  bx = t % ntx;
  by = t / ntx;
  return true;
}
inline int xcd_grid(int ntx, int nty) { return NXCD * ((ntx * nty + NXCD - 1) / NXCD); }

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

template <int W, int H, class R>
__device__ __forceinline__ void put_rec(R (*s)[H][W], int ty, int tx, const DirEvalT<R>& e) {
#pragma unroll
  for (int c = 0; c < NV; ++c) s[c][ty][tx] = e.F[c];
  s[8][ty][tx] = e.sr;
  s[9][ty][tx] = e.cf;
  s[10][ty][tx] = e.vn;
  s[11][ty][tx] = e.sq;
}
template <int W, int H, class R>
__device__ __forceinline__ void get_rec(R (*s)[H][W], int ty, int tx, DirEvalT<R>& e) {
#pragma unroll
  for (int c = 0; c < NV; ++c) e.F[c] = s[c][ty][tx];
  e.sr = s[8][ty][tx];
  e.cf = s[9][ty][tx];
  e.vn = s[10][ty][tx];
  e.sq = s[11][ty][tx];
}

template <class R>
__device__ __forceinline__ void put_rec(R (*s)[PB][PB], int base, int ty, int tx, const DirEvalT<R>& e) {
#pragma unroll
  for (int c = 0; c < NV; ++c) s[base + c][ty][tx] = e.F[c];
  s[base + 8][ty][tx] = e.sr;
  s[base + 9][ty][tx] = e.cf;
  s[base + 10][ty][tx] = e.vn;
  s[base + 11][ty][tx] = e.sq;
}
template <class R>
__device__ __forceinline__ void get_rec(R (*s)[PB][PB], int base, int ty, int tx, DirEvalT<R>& e) {
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
template <class R>
struct LineAcc {
  R SF[NV], SW[NV], G[NV];
  R alpha, dB, jl;
};

template <class R>
__device__ __forceinline__ void line_begin(LineAcc<R>& L, const DirEvalT<R>& e0, const R U0[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    L.SF[c] = R(0);
    L.SW[c] = R(6) * U0[c];
    L.G[c] = R(0);
  }
  L.alpha = e0.sr;
  L.dB = R(0);
  L.jl = R(0);
}

// side = -1 for the neighbour at -h (left/below), +1 at +h.
template <class R>
__device__ __forceinline__ void line_outer(LineAcc<R>& L, int bn, int side, const DirEvalT<R>& e, const R U[NV],
                                           const DirEvalT<R>& e0, const R U0[NV]) {
  L.alpha = fmax(L.alpha, e.sr);
  const R al = side < 0 ? alpha_llf(e, e0, U, U0) : alpha_llf(e0, e, U0, U);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    L.SF[c] -= side * e.F[c];
    L.SW[c] += U[c];
    // F^LLF(U0, U) for side +1, -F^LLF(U, U0) for side -1
    L.G[c] += side < 0 ? R(-0.5) * (e.F[c] + e0.F[c] - al * (U0[c] - U[c]))
                       : R(0.5) * (e0.F[c] + e.F[c] - al * (U[c] - U0[c]));
  }
  L.dB -= side * U[bn];
  L.jl += side * U[bn];
}

template <class R>
__device__ __forceinline__ void line_inner(LineAcc<R>& L, int bn, int side, const DirEvalT<R>& e, const R U[NV]) {
  L.alpha = fmax(L.alpha, e.sr);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    L.SF[c] += side * R(4) * e.F[c];
    L.SW[c] -= R(4) * U[c];
  }
  L.dB += side * R(4) * U[bn];
}

// Point accumulators: high-order RHS h = -R_x - R_y with the div part, and
// the LLF update l = -dt/dx G_x - dt/dy G_y with its div part.
template <class R>
struct PointAcc {
  R h[NV], l[NV];
  R divh, divl;
};

template <class R>
__device__ __forceinline__ void acc_fvs(PointAcc<R>& P, const LineAcc<R>& L, R rh, R lam) {
  const R s = R(0.5) * rh;
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
template <class R>
__device__ __forceinline__ void acc_central(PointAcc<R>& P, int bn, R rh, R lam, const DirEvalT<R>& ed,
                                            const R dn[NV], const DirEvalT<R>& e0, const R U0[NV],
                                            const DirEvalT<R>& eu, const R up[NV]) {
  const R ad = alpha_llf(ed, e0, dn, U0), au = alpha_llf(e0, eu, U0, up);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    P.h[c] -= (eu.F[c] - ed.F[c]) * rh;
    const R G = R(0.5) * (e0.F[c] + eu.F[c] - au * (up[c] - U0[c])) - R(0.5) * (ed.F[c] + e0.F[c] - ad * (U0[c] - dn[c]));
    P.l[c] -= lam * G;
  }
  P.divh += (up[bn] - dn[bn]) * rh;
  P.divl += R(0.5) * rh * (up[bn] - dn[bn]);
}

template <class R>
__device__ __forceinline__ void acc_zero(PointAcc<R>& P) {
#pragma unroll
  for (int c = 0; c < NV; ++c) P.h[c] = P.l[c] = R(0);
  P.divh = P.divl = R(0);
}

// High-order and LLF states from the accumulators (the right-hand sides in
// the compute type, the states in FP64), scaling limiter, SSP combination,
// store.
template <class R>
__device__ __forceinline__ void finish(const Geo& g, double dt, const double U0[NV], const PointAcc<R>& P,
                                      double ca, double cb, const double* __restrict__ un, double* __restrict__ out,
                                      long plane, long off, Counters* cn) {
  double UH[NV], UL[NV], W[NV];
  R Ps[NV];
  psi(U0, Ps);
  if constexpr (IsF32<R>::value) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      UH[c] = U0[c] + dt * (double)(P.h[c] - P.divh * Ps[c]);
      UL[c] = U0[c] + (double)(P.l[c] - (float)dt * P.divl * Ps[c]);
    }
  } else {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      UH[c] = U0[c] + dt * (P.h[c] - P.divh * Ps[c]);
      UL[c] = U0[c] + P.l[c] - dt * P.divl * Ps[c];
    }
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

// LDS layout of k_points (fields of PB x PB values of the compute type):
// states of the tile's V, X, Y and centre values, then two directional
// records.
constexpr int SV_ = 0, SX_ = 8, SY_ = 16, SC_ = 24, SR0 = 32, SR1 = 32 + RF, SFIELDS = 32 + 2 * RF;

template <class R>
__device__ __forceinline__ void lds8(R (*s)[PB][PB], int base, int ty, int tx, R U[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) U[c] = s[base + c][ty][tx];
}
template <class R>
__device__ __forceinline__ void sts8(R (*s)[PB][PB], int base, int ty, int tx, const double U[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) s[base + c][ty][tx] = (R)U[c];
}

// R = double: the FP64 stage; R = float: the FP32-bulk stage (LDS holds the
// compute type; a thread's own states are re-read in FP64 from memory for
// the evaluations and the FP64 accumulation).
template <class R>
__global__ __launch_bounds__(PNT, IsF32<R>::value ? 2 : 1) void k_points(Geo g, CState u, CState un, MState out, double* __restrict__ centre,
                                                const double* dtp, double ca, double cb, Counters* cn, int ntx,
                                                int nty) {
  constexpr bool F32 = IsF32<R>::value;
  __shared__ R s[SFIELDS][PB][PB];
  int bx, by;
  if (!xcd_tile(ntx, nty, bx, by)) return;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i0 = bx * (PB - 2) - 1, j0 = by * (PB - 2) - 1;
  const int i = clamp_pt(i0 + tx, g.nxp), j = clamp_pt(j0 + ty, g.nyp);
  const bool inner = tx >= 1 && tx < PB - 1 && ty >= 1 && ty < PB - 1;
  const bool outV = inner && i0 + tx < g.nxp && j0 + ty < g.nyp;
  const bool outX = inner && i0 + tx < g.nxp && j0 + ty < g.ny;
  const bool outY = inner && i0 + tx < g.nx && j0 + ty < g.nyp;
  const double dt = *dtp;
  const double lx = dt * g.rdx, ly = dt * g.rdy;
  const R rdx = (R)g.rdx, rdy = (R)g.rdy, lxr = (R)lx, lyr = (R)ly;
  const int txl = tx > 0 ? tx - 1 : tx, txr = tx < PB - 1 ? tx + 1 : tx;
  const int tyd = ty > 0 ? ty - 1 : ty, tyu = ty < PB - 1 ? ty + 1 : ty;

  // 0: the tile's raw point values into LDS
  {
    double w[NV];
    ldV(g, u.v, i, j, w);
    sts8(s, SV_, ty, tx, w);
    ldX(g, u.x, i, j, w);
    sts8(s, SX_, ty, tx, w);
    ldY(g, u.y, i, j, w);
    sts8(s, SY_, ty, tx, w);
  }
  __syncthreads();
  // a thread's own FP64 states (V, X, Y; the centre is kept in C64)
  double C64[NV];
  auto own = [&](int which, double U[NV]) {
    if constexpr (F32) {
      if (which == 0) ldV(g, u.v, i, j, U);
      else if (which == 1) ldX(g, u.x, i, j, U);
      else if (which == 2) ldY(g, u.y, i, j, U);
      else {
#pragma unroll
        for (int c = 0; c < NV; ++c) U[c] = C64[c];
      }
    } else {
      lds8(s, which == 0 ? SV_ : which == 1 ? SX_ : which == 2 ? SY_ : SC_, ty, tx, U);
    }
  };
  // 1: centre values in FP64 (the last column/row's are never used); the
  //    owner also stores its value for the cell kernel's source term
  {
    double A[NV], Uc[NV], f[NV], w[NV], q[NV];
    ldA(g, u.a, i, j, A);
    if constexpr (F32) {
      ldX(g, u.x, i, j, f);
      ldX(g, u.x, i + 1, j, w);
      ldY(g, u.y, i, j, Uc);
      ldY(g, u.y, i, j + 1, q);
    } else {
      lds8(s, SX_, ty, tx, f);
      lds8(s, SX_, ty, txr, w);
      lds8(s, SY_, ty, tx, Uc);
      lds8(s, SY_, tyu, tx, q);
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) f[c] = -4.0 * ((f[c] + w[c]) + (Uc[c] + q[c]));
    if constexpr (F32) {
      ldV(g, u.v, i, j, Uc);
      ldV(g, u.v, i + 1, j, w);
    } else {
      lds8(s, SV_, ty, tx, Uc);
      lds8(s, SV_, ty, txr, w);
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) Uc[c] += w[c];
    if constexpr (F32) {
      ldV(g, u.v, i, j + 1, q);
      ldV(g, u.v, i + 1, j + 1, w);
    } else {
      lds8(s, SV_, tyu, tx, q);
      lds8(s, SV_, tyu, txr, w);
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) Uc[c] = (36.0 * A[c] + f[c] - (Uc[c] + (q[c] + w[c]))) * 0.0625;
    const bool owner = inner && i0 + tx < g.nx && j0 + ty < g.ny;
    limit_centre(Uc, A, g.gm1, C64, cn, owner);
    sts8(s, SC_, ty, tx, C64);
    if (owner) {
#pragma unroll
      for (int c = 0; c < NV; ++c) centre[c * g.sc + (long)j * g.nx + i] = C64[c];
    }
  }
  PointAcc<R> PA, PB_;
  DirEvalT<R> e0, e1, en;
  R U0[NV], U1[NV], Un[NV];
  LineAcc<R> L;

  // b: vertical lines through V and X.  V: FVS in y over V(l-1), X(l-1), V,
  // X(l), V(l+1).  X: central in y between V(k,j) and V(k,j+1).
  {
    double w[NV];
    own(0, w);
    eval_dir(w, g, 1, e0);
    own(1, w);
    eval_dir(w, g, 1, e1);
  }
  lds8(s, SV_, ty, tx, U0);
  lds8(s, SX_, ty, tx, U1);
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
  acc_fvs(PA, L, rdy, lyr);
  acc_central(PB_, 5, rdy, lyr, e0, U0, e1, U1, en, Un);
  __syncthreads();

  // a: horizontal lines through V and Y.  V: FVS in x over V(k-1), Y(k-1),
  // V, Y(k), V(k+1) -> V complete.  Y: central in x between V(i,l), V(i+1,l).
  {
    double w[NV];
    own(0, w);
    eval_dir(w, g, 0, e0);
    own(2, w);
    eval_dir(w, g, 0, e1);
  }
  lds8(s, SY_, ty, tx, U1);
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
  acc_fvs(PA, L, rdx, lxr);
  if (outV) {
    double w[NV];
    own(0, w);
    finish(g, dt, w, PA, ca, cb, un.v, out.v, g.sv, (long)j * g.nxp + i, cn);
  }
  acc_zero(PA);  // now Y
  acc_central(PA, 4, rdx, lxr, e0, U0, e1, U1, en, Un);
  __syncthreads();

  // c: horizontal lines through X and C.  X: FVS in x over X(k-1), C(k-1),
  // X, C(k), X(k+1) -> X complete.
  {
    double w[NV];
    own(1, w);
    eval_dir(w, g, 0, e0);
    own(3, w);
    eval_dir(w, g, 0, e1);
  }
  lds8(s, SX_, ty, tx, U0);
  lds8(s, SC_, ty, tx, Un);
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
  acc_fvs(PB_, L, rdx, lxr);
  if (outX) {
    double w[NV];
    own(1, w);
    finish(g, dt, w, PB_, ca, cb, un.x, out.x, g.sx, (long)j * g.nxp + i, cn);
  }
  __syncthreads();

  // d: vertical lines through Y and C.  Y: FVS in y over Y(l-1), C(l-1), Y,
  // C(l), Y(l+1) -> Y complete.
  {
    double w[NV];
    own(2, w);
    eval_dir(w, g, 1, e0);
    own(3, w);
    eval_dir(w, g, 1, e1);
  }
  lds8(s, SC_, ty, tx, Un);
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
  acc_fvs(PA, L, rdy, lyr);
  if (outY) {
    double w[NV];
    own(2, w);
    finish(g, dt, w, PA, ca, cb, un.y, out.y, g.sy, (long)j * g.nx + i, cn);
  }
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
// Formed in FP64 (pressure recovery), stored in the compute type.
template <class R>
__device__ void sensor_prims(const double U[NV], double gamma, R q[5]) {
#pragma clang fp contract(off)
  q[0] = (R)(sensor_pressure(U, gamma) + (U[4] * U[4] + U[5] * U[5] + U[6] * U[6]) / 2.0);
  q[1] = (R)(U[1] / U[0]);
  q[2] = (R)(U[2] / U[0]);
  q[3] = (R)U[4];
  q[4] = (R)U[5];
}

// Indicators from the primitives of the cell (c) and its neighbours
// l, r (x) and d, u (y): phi1x, phi1y, phi2, phi3.
template <class R>
__device__ void sensor_from_prims(const R c[5], const R l[5], const R r[5], const R d[5], const R u[5], R dx, R dy,
                                  R phi[4]) {
#pragma clang fp contract(off)
  // the regulariser 1e-40 underflows to 0 in FP32; 1e-30 keeps it there
  const R tiny = IsF32<R>::value ? R(1e-30) : R(1e-40);
  phi[0] = fabs(r[0] - R(2) * c[0] + l[0]) / fabs(r[0] + R(2) * c[0] + l[0]);
  phi[1] = fabs(u[0] - R(2) * c[0] + d[0]) / fabs(u[0] + R(2) * c[0] + d[0]);
  const R dv = (r[1] - l[1]) / (R(2) * dx) + (u[2] - d[2]) / (R(2) * dy);
  const R cv = (r[2] - l[2]) / (R(2) * dx) - (u[1] - d[1]) / (R(2) * dy);
  phi[2] = fmax(-dv / sqrt(dv * dv + cv * cv + tiny), R(0));
  phi[3] = fabs(r[3] - l[3] + u[4] - d[4]) / (fabs(c[3] + c[4]) + tiny);
}

// Nine-point Powell source of cell (i,j), eq. (semi_av_src): weights
// (1/6, 2/3, 1/6) per direction, the divergence at each sample point from
// the one-sided / central differences of eq. (2d_fd) along the cell's rows
// and columns, Psi at each point.  The centre sample is the limited centre
// value, read from the buffer the point kernel fills.
template <class R>
__device__ void cell_source(const Geo& g, CState u, const double* __restrict__ centre, int i, int j, R S[NV]) {
  double C[NV];
  ldA(g, centre, i, j, C);
  // B1, B2 at the nine samples, [a][b] with a along x, b along y
  R B1[3][3], B2[3][3];
  auto ldB = [&](int a, int b, R& b1, R& b2) {
    long off;
    const double* base;
    long plane;
    if (a == 1 && b == 1) {
      b1 = (R)C[4];
      b2 = (R)C[5];
      return;
    } else if (b == 1) {
      base = u.x, plane = g.sx, off = (long)map_cell(j, g.ny, g.bcy) * g.nxp + map_node(i + a / 2, g.nx, g.bcx);
    } else if (a == 1) {
      base = u.y, plane = g.sy, off = (long)map_node(j + b / 2, g.ny, g.bcy) * g.nx + map_cell(i, g.nx, g.bcx);
    } else {
      base = u.v, plane = g.sv,
      off = (long)map_node(j + b / 2, g.ny, g.bcy) * g.nxp + map_node(i + a / 2, g.nx, g.bcx);
    }
    b1 = (R)base[4 * plane + off];
    b2 = (R)base[5 * plane + off];
  };
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) ldB(a, b, B1[a][b], B2[a][b]);
  const R wq[3] = {R(1.0 / 6.0), R(2.0 / 3.0), R(1.0 / 6.0)};
  const R rdx = (R)g.rdx, rdy = (R)g.rdy;
  R f[9];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R dx1 = a == 0 ? (R(-3) * B1[0][b] + R(4) * B1[1][b] - B1[2][b])
                  : a == 1 ? (B1[2][b] - B1[0][b])
                           : (B1[0][b] - R(4) * B1[1][b] + R(3) * B1[2][b]);
      const R dy2 = b == 0 ? (R(-3) * B2[a][0] + R(4) * B2[a][1] - B2[a][2])
                  : b == 1 ? (B2[a][2] - B2[a][0])
                           : (B2[a][0] - R(4) * B2[a][1] + R(3) * B2[a][2]);
      f[3 * b + a] = wq[a] * wq[b] * (dx1 * rdx + dy2 * rdy);
    }
#pragma unroll
  for (int c = 0; c < NV; ++c) S[c] = R(0);
  // One sample at a time (a rolled loop): the states of all nine are never
  // live together.
#pragma unroll 1
  for (int q = 0; q < 9; ++q) {
    const int a = q % 3, b = q / 3;
    R fq = f[0];
#pragma unroll
    for (int r = 1; r < 9; ++r) fq = q == r ? f[r] : fq;
    double w[NV];
    R P[NV];
    if (q == 4) {
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
    for (int c = 1; c < NV; ++c) S[c] += fq * P[c];
  }
}

__device__ __forceinline__ int clamp_cell(int i, int n) { return i < -2 ? -2 : (i > n + 1 ? n + 1 : i); }
// Sensor primitives are needed on cells [-3, n+2]: the indicators of the
// ghost cells -2 and n+1 enter the sensor of the outermost interfaces whose
// flux-limiter coefficients the boundary cells take.
__device__ __forceinline__ int clamp_prim(int i, int n) { return i < -3 ? -3 : (i > n + 2 ? n + 2 : i); }

// Simpson flux over the edge points w0, w1, w2 (Section 2.2), LLF flux of
// the adjacent averages (eq. 2d_llf_flux) and the sensor blend: returns
// F^LLF and dF = theta^s (F_simpson - F^LLF).
template <class R>
__device__ __forceinline__ void interface_flux(const Geo& g, int dir, const double w0[NV], const double w1[NV],
                                               const double w2[NV], const DirEvalT<R>& eL, const double AL[NV],
                                               const DirEvalT<R>& eR, const double AR[NV], R ts, R Fl[NV],
                                               R dF[NV]) {
  R Fh[NV], F[NV];
  flux_dir(w0, g.gm1, dir, Fh);
  flux_dir(w1, g.gm1, dir, F);
#pragma unroll
  for (int c = 0; c < NV; ++c) Fh[c] += R(4) * F[c];
  flux_dir(w2, g.gm1, dir, F);
  constexpr R sixth = R(1.0 / 6.0);
#pragma unroll
  for (int c = 0; c < NV; ++c) Fh[c] = (Fh[c] + F[c]) * sixth;
  const R al = alpha_llf(eL, eR, AL, AR);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    Fl[c] = R(0.5) * (eL.F[c] + eR.F[c] - al * (R)(AR[c] - AL[c]));
    dF[c] = ts * Fh[c] + (R(1) - ts) * Fl[c] - Fl[c];
  }
}

template <class R>
__device__ __forceinline__ R sensor_theta(R kappa, const R* a, const R* b, int dir) {
  const R p1 = fmax(a[dir], b[dir]), p2 = fmax(a[2], b[2]), p3 = fmax(a[3], b[3]);
  return exp_r(-kappa * (p1 * p2 + p3));
}

template <class R>
__global__ __launch_bounds__(CNT) void k_cells(Geo g, CState u, const double* __restrict__ centre,
                                               const double* __restrict__ un, double* __restrict__ out,
                                               const double* dtp, double ca, double cb, Counters* cn, int ntx,
                                               int nty) {
  // s_dfx / s_dfy: theta^s (F_simpson - F^LLF) at the x-interface left of /
  // the y-interface below each thread's cell; they give H_L, H_R, H_D, H_U.
  __shared__ R s_dfx[NV][CBY][CBX];
  __shared__ R s_dfy[NV][CBY][CBX];
  __shared__ R s_x[RF][CBY][CBX];  // exchange: primitives, records, F^LLF, Lambda
  __shared__ R s_ts[2][CBY][CBX];  // theta^s at the two interfaces
  __shared__ R s_phi[CBY + 1][CBX + 1][4];
  // Lambda exchange (FP64): the exchange buffer itself for the FP64 stage
  double (*s_lam)[CBY][CBX];
  if constexpr (IsF32<R>::value) {
    __shared__ double lam_buf[4][CBY][CBX];
    s_lam = lam_buf;
  } else {
    s_lam = reinterpret_cast<double (*)[CBY][CBX]>(&s_x[0][0][0]);
  }
  int bx, by;
  if (!xcd_tile(ntx, nty, bx, by)) return;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * CBX + tx;
  const int i0 = bx * (CBX - 3) - 1, j0 = by * (CBY - 3) - 1;
  const int i = clamp_cell(i0 + tx, g.nx), j = clamp_cell(j0 + ty, g.ny);
  const bool output = tx >= 1 && tx < CBX - 2 && ty >= 1 && ty < CBY - 2 && i0 + tx < g.nx && j0 + ty < g.ny;
  const int txr = tx + 1 < CBX ? tx + 1 : tx, tyu = ty + 1 < CBY ? ty + 1 : ty;
  const double dt = *dtp;
  const double lx = dt * g.rdx, ly = dt * g.rdy;

  // 1a: sensor primitives on [i0-2, i0+CBX+1) x [j0-2, j0+CBY+1), aliased
  //     onto the exchange buffer
  constexpr int PW = CBX + 3, PH = CBY + 3;
  static_assert(5 * PW * PH <= RF * CBX * CBY, "primitives must fit the exchange buffer");
  R* prim = &s_x[0][0][0];
  for (int it = tid; it < PW * PH; it += CNT) {
    const int a = it % PW, b = it / PW;
    double U[NV];
    R q[5];
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
    R c[5], l[5], r[5], d[5], up[5], ph[4];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const R* pm = prim + m * PW * PH;
      c[m] = pm[pc];
      l[m] = pm[pc - 1];
      r[m] = pm[pc + 1];
      d[m] = pm[pc - PW];
      up[m] = pm[pc + PW];
    }
    sensor_from_prims(c, l, r, d, up, (R)g.dx, (R)g.dy, ph);
#pragma unroll
    for (int q = 0; q < 4; ++q) s_phi[b][a][q] = ph[q];
  }
  __syncthreads();

  double A[NV], G[NV];
  R S[NV];
  ldA(g, u.a, i, j, A);
  // 2: nine-point source (before the interfaces: its temporaries and theirs
  //    are never live together)
  cell_source(g, u, centre, i, j, S);
#pragma unroll
  for (int c = 0; c < NV; ++c) G[c] = A[c];

  // 3: interfaces.  dir 0: the x-interface left of the cell, dir 1: the
  //    y-interface below it.  The cell's own directional evaluation is
  //    shared with the neighbour on the other side through LDS.
  const R kappa = (R)g.kappa;
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    R Fl[NV];
    {
      DirEvalT<R> eA, eN;
      double AN[NV];
      eval_dir(A, g, dir, eA);
      put_rec(s_x, ty, tx, eA);
      __syncthreads();
      const int nx_ = dir == 0 ? tx - 1 : tx, ny_ = dir == 0 ? ty : ty - 1;
      if (dir == 0) ldA(g, u.a, i - 1, j, AN); else ldA(g, u.a, i, j - 1, AN);
      if ((dir == 0 ? tx : ty) > 0) {
        get_rec(s_x, ny_, nx_, eN);
      } else {
        eval_dir(AN, g, dir, eN);
      }
      double w0[NV], w1[NV], w2[NV];
      R dF[NV];
      ldV(g, u.v, i, j, w0);
      if (dir == 0) {
        ldX(g, u.x, i, j, w1);
        ldV(g, u.v, i, j + 1, w2);
      } else {
        ldY(g, u.y, i, j, w1);
        ldV(g, u.v, i + 1, j, w2);
      }
      const R ts = dir == 0 ? sensor_theta(kappa, s_phi[ty + 1][tx], s_phi[ty + 1][tx + 1], 0)
                            : sensor_theta(kappa, s_phi[ty][tx + 1], s_phi[ty + 1][tx + 1], 1);
      interface_flux(g, dir, w0, w1, w2, eN, AN, eA, A, ts, Fl, dF);
      s_ts[dir][ty][tx] = ts;
#pragma unroll
      for (int c = 0; c < NV; ++c) (dir == 0 ? s_dfx : s_dfy)[c][ty][tx] = dF[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NV; ++c) s_x[c][ty][tx] = Fl[c];
    __syncthreads();
    const double lam = dir == 0 ? lx : ly;
#pragma unroll
    for (int c = 0; c < NV; ++c) G[c] += lam * (double)(Fl[c] - (dir == 0 ? s_x[c][ty][txr] : s_x[c][tyu][tx]));
    __syncthreads();
  }
  // H_I(c): anti-diffusive updates of the four interfaces
  auto H = [&](int I, int c) -> double {
    switch (I) {
      case 0: return lx * (double)s_dfx[c][ty][tx];
      case 1: return -lx * (double)s_dfx[c][ty][txr];
      case 2: return ly * (double)s_dfy[c][ty][tx];
      default: return -ly * (double)s_dfy[c][tyu][tx];
    }
  };
  const R tsmin = fmin(fmin(s_ts[0][ty][tx], s_ts[0][ty][txr]), fmin(s_ts[1][ty][tx], s_ts[1][tyu][tx]));

  // 4: LLF source, sensor blend of the source, flux-limiter steps (1)-(2)
  R Sl[NV];
  double Allf[NV], Asrc[NV];
  {
    R P[NV];
    double AN[NV], b;
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
      Sl[c] = (R)divb * P[c];
      S[c] = tsmin * S[c] + (R(1) - tsmin) * Sl[c];
      Allf[c] = G[c] - dt * (double)Sl[c];
      Asrc[c] = G[c] - dt * (double)S[c];
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
  double SL[NV];  // S^Lim
#pragma unroll
  for (int c = 0; c < NV; ++c) SL[c] = th * (double)S[c] + (1.0 - th) * (double)Sl[c];
  double Lam[4];
  limiter_box(A1, H, g.gm1, er, ep, Lam, cn, output);
  // 5: unique interface coefficients and the limited update
#pragma unroll
  for (int I = 0; I < 4; ++I) s_lam[I][ty][tx] = Lam[I];
  __syncthreads();
  if (!output) return;
  const double thL = fmin(s_lam[1][ty][tx - 1], Lam[0]);
  const double thR = fmin(Lam[1], s_lam[0][ty][tx + 1]);
  const double thD = fmin(s_lam[3][ty - 1][tx], Lam[2]);
  const double thU = fmin(Lam[3], s_lam[2][ty + 1][tx]);
  if (thL < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thL); }
  if (thD < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thD); }
  if (g.bcx && i == g.nx - 1 && thR < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thR); }
  if (g.bcy && j == g.ny - 1 && thU < 1.0) { count(&cn->n_theta_active); count_min_theta(cn, thU); }
  double An[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c)
    An[c] = G[c] - dt * SL[c] + thL * H(0, c) + thR * H(1, c) + thD * H(2, c) + thU * H(3, c);
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
// Optional per-kernel timing (AF_FLAG_KERNEL_TIMING): a pair of events
// recorded on the context's stream around each launch; pairs are folded
// into totals when the pool is full and on af_mhd_kernel_times.
struct KernelTimer {
  enum { POINTS = 0, CELLS = 1, DT = 2, NKIND = 3, POOL = 1024 };
  hipEvent_t ev[2 * POOL];
  int kind[POOL];
  int created = 0, used = 0;
  double ms[NKIND] = {0.0, 0.0, 0.0};
  long long n[NKIND] = {0, 0, 0};
};

struct af_mhd_ctx {
  Geo g;
  WS ws;
  hipStream_t stream;
  std::string err;
  KernelTimer* timer = nullptr;
  bool f32 = false;  // AF_FLAG_FP32_BULK
  ~af_mhd_ctx() {
    if (timer) {
      for (int q = 0; q < timer->created; ++q) (void)hipEventDestroy(timer->ev[q]);
      delete timer;
    }
  }
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
  return (p->flags & ~(uint32_t)(AF_FLAG_KERNEL_TIMING | AF_FLAG_FP32_BULK)) == 0;
}

// Fold every recorded pair into the totals (synchronises on the last event).
hipError_t timer_fold(KernelTimer* t) {
  if (!t || t->used == 0) return hipSuccess;
  hipError_t e = hipEventSynchronize(t->ev[2 * t->used - 1]);
  for (int q = 0; q < t->used && e == hipSuccess; ++q) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, t->ev[2 * q], t->ev[2 * q + 1]);
    t->ms[t->kind[q]] += ms;
    t->n[t->kind[q]] += 1;
  }
  t->used = 0;
  return e;
}

// Start event of a timed launch of the given kind (nullptr when timing is
// off); the matching end event is returned through *end.
hipError_t timer_begin(af_mhd_ctx* c, int kind, hipEvent_t* end) {
  *end = nullptr;
  KernelTimer* t = c->timer;
  if (!t) return hipSuccess;
  hipError_t e = hipSuccess;
  if (t->used == KernelTimer::POOL) e = timer_fold(t);
  const int q = t->used;
  while (e == hipSuccess && t->created < 2 * (q + 1)) e = hipEventCreate(&t->ev[t->created++]);
  if (e == hipSuccess) e = hipEventRecord(t->ev[2 * q], c->stream);
  if (e != hipSuccess) return e;
  t->kind[q] = kind;
  t->used = q + 1;
  *end = t->ev[2 * q + 1];
  return hipSuccess;
}
hipError_t timer_end(af_mhd_ctx* c, hipEvent_t end) { return end ? hipEventRecord(end, c->stream) : hipSuccess; }

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
  w.centre = take(8 * sizes[0]);
  if (ws) *ws = w;
  return off;
}

// Message of the last failed af_mhd_init on this thread (no context exists).
thread_local std::string init_err;

int fail(af_mhd_ctx* c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}

int init_fail(int code, const std::string& msg) {
  init_err = msg;
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
  const int ptx = (g.nxp + PB - 3) / (PB - 2), pty = (g.nyp + PB - 3) / (PB - 2);
  hipEvent_t end;
  hipError_t e = timer_begin(c, KernelTimer::POINTS, &end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  if (c->f32)
    k_points<float><<<xcd_grid(ptx, pty), dim3(PB, PB), 0, s>>>(g, u, n, o, c->ws.centre, dt_dev, A[k], B[k],
                                                                c->ws.cnt, ptx, pty);
  else
    k_points<double><<<xcd_grid(ptx, pty), dim3(PB, PB), 0, s>>>(g, u, n, o, c->ws.centre, dt_dev, A[k], B[k],
                                                                 c->ws.cnt, ptx, pty);
  e = timer_end(c, end);
  if (e == hipSuccess) e = timer_begin(c, KernelTimer::CELLS, &end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  const int ctx_ = (g.nx + CBX - 4) / (CBX - 3), cty = (g.ny + CBY - 4) / (CBY - 3);
  if (c->f32)
    k_cells<float><<<xcd_grid(ctx_, cty), dim3(CBX, CBY), 0, s>>>(g, u, c->ws.centre, n.a, o.a, dt_dev, A[k], B[k],
                                                                  c->ws.cnt, ctx_, cty);
  else
    k_cells<double><<<xcd_grid(ctx_, cty), dim3(CBX, CBY), 0, s>>>(g, u, c->ws.centre, n.a, o.a, dt_dev, A[k],
                                                                   B[k], c->ws.cnt, ctx_, cty);
  e = timer_end(c, end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  return check_hip(c, "stage launch");
}

int run_dt(af_mhd_ctx* c, const af_mhd_state* u, double t_rem, double* dt_dev) {
  const Geo& g = c->g;
  const long n = g.sc + g.sx + g.sy + g.sv;
  const int nb = (int)std::min<long>(RED_BLOCKS, std::max<long>(1, nblocks(n)));
  hipEvent_t end;
  hipError_t e = timer_begin(c, KernelTimer::DT, &end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  k_dt_partial<<<nb, BLK, 0, c->stream>>>(g, cstate(u), c->ws.partial);
  k_dt_final<<<1, BLK, 0, c->stream>>>(c->ws.partial, nb, g.cfl, t_rem, dt_dev);
  e = timer_end(c, end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
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
  init_err.clear();
  if (!out) return init_fail(AF_EINVAL, "af_mhd_init: null output");
  if (!valid_params(p)) return init_fail(AF_EINVAL, "af_mhd_init: invalid parameters");
  if (!workspace_dev || ((uintptr_t)workspace_dev & 255))
    return init_fail(AF_EINVAL, "af_mhd_init: workspace null or not 256-byte aligned");
  af_mhd_ctx* c = new (std::nothrow) af_mhd_ctx();
  if (!c) return init_fail(AF_EINVAL, "af_mhd_init: out of host memory");
  make_geo(p, c->g);
  const size_t need = layout(c->g, nullptr, nullptr);
  if (workspace_bytes < need) {
    delete c;
    return init_fail(AF_EWORKSPACE, "af_mhd_init: workspace too small");
  }
  layout(c->g, static_cast<char*>(workspace_dev), &c->ws);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->f32 = (p->flags & AF_FLAG_FP32_BULK) != 0;
  if (p->flags & AF_FLAG_KERNEL_TIMING) {
    c->timer = new (std::nothrow) KernelTimer();
    if (!c->timer) {
      delete c;
      return init_fail(AF_EINVAL, "af_mhd_init: out of host memory");
    }
  }
  (void)hipGetLastError();  // report only what this launch raises
  k_zero_counters<<<1, 64, 0, c->stream>>>(c->ws.cnt);
  const int rc = check_hip(c, "af_mhd_init");
  if (rc != AF_OK) {
    init_fail(rc, c->err);
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

int af_mhd_kernel_times(af_mhd_ctx* c, af_mhd_kernel_times_t* out, int reset) {
  if (!c) return AF_EINVAL;
  if (!out || !c->timer) return fail(c, AF_EINVAL, "af_mhd_kernel_times: timing not enabled or null output");
  const hipError_t e = timer_fold(c->timer);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  KernelTimer* t = c->timer;
  out->ms_points = t->ms[KernelTimer::POINTS];
  out->ms_cells = t->ms[KernelTimer::CELLS];
  out->ms_dt = t->ms[KernelTimer::DT];
  out->n_points = t->n[KernelTimer::POINTS];
  out->n_cells = t->n[KernelTimer::CELLS];
  out->n_dt = t->n[KernelTimer::DT];
  if (reset) {
    for (int q = 0; q < KernelTimer::NKIND; ++q) {
      t->ms[q] = 0.0;
      t->n[q] = 0;
    }
  }
  c->err.clear();
  return AF_OK;
}

void af_mhd_destroy(af_mhd_ctx* c) { delete c; }

const char* af_mhd_last_error(const af_mhd_ctx* c) { return c ? c->err.c_str() : init_err.c_str(); }

}  // extern "C"
