// af_tiles.h -- the tile bodies of one SSP-RK3 stage of the PP Active Flux
// scheme for 2D ideal MHD with the Godunov-Powell source (gfx950): the point
// update (points_tile) and the cell update (cells_tile), the XCD-aware tile
// order and the reduction helpers.  Shared by the single-grid kernels
// (af_stage.hip) and the persistent batched kernels (af_batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "af_device.h"

namespace afm {

constexpr int BLK = 256;

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

__device__ inline double sensor_pressure(const double U[NV], double gamma) {
#pragma clang fp contract(off)
  const double m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
  const double b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  return (gamma - 1.0) * (U[7] - m2 / (2.0 * U[0]) - b2 / 2.0);
}

// rho_1/dx + rho_2/dy of a state (rho_l = |v_l| + c_f,l, eq. (cf)): dt is
// cfl over its maximum over all DoFs.  Contraction-free, so that every
// kernel that takes this maximum (the reduction over a state, the epilogue
// of a step's last stage, the batched reduction) gets the same bits.
__device__ __forceinline__ double dt_speed(const double U[NV], const Geo& g) {
#pragma clang fp contract(off)
  const double ri = rcp_r(U[0]);
  const double v1 = U[1] * ri, v2 = U[2] * ri, v3 = U[3] * ri;
  const double b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  const double p = g.gm1 * (U[7] - 0.5 * (U[1] * v1 + U[2] * v2 + U[3] * v3) - 0.5 * b2);
  const double c2 = g.gamma * p * ri;
  const double s = c2 + b2 * ri;
  double d1 = s * s - 4.0 * c2 * U[4] * U[4] * ri;
  double d2 = s * s - 4.0 * c2 * U[5] * U[5] * ri;
  d1 = d1 > 0.0 ? d1 : 0.0;
  d2 = d2 > 0.0 ? d2 : 0.0;
  const double c1 = sqrt_r(0.5 * (s + sqrt_r(d1))), cy = sqrt_r(0.5 * (s + sqrt_r(d2)));
  return (fabs(v1) + c1) * g.rdx + (fabs(v2) + cy) * g.rdy;
}

// Maximum of v over the workgroup (nthreads a multiple of 64, every thread
// calling), written by thread 0 to *slot.  scratch: nthreads/64 doubles of
// LDS no other thread reads or writes meanwhile.
__device__ __forceinline__ void block_max_store(double v, int tid, int nthreads, double* scratch, double* slot) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((tid & 63) == 0) scratch[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < nthreads / 64; ++w) v = fmax(v, scratch[w]);
    *slot = v;
  }
}

// Nine-point Powell source of a cell, eq. (semi_av_src): weights
// (1/6, 2/3, 1/6) per direction, the divergence at each sample point from
// the one-sided / central differences of eq. (2d_fd) along the cell's rows
// and columns, Psi at each point.  Bat(a, b, B1, B2) and Psiat(a, b, P) give
// the field and Psi at sample (a, b) (a along x, b along y; (1, 1) is the
// limited centre value): one body of arithmetic whichever memory the
// samples come from.
template <class R, class BF, class PF>
__device__ __forceinline__ void source_nine(BF Bat, PF Psiat, R rdx, R rdy, R S[NV]) {
  R B1[3][3], B2[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) Bat(a, b, B1[a][b], B2[a][b]);
  const R wq[3] = {R(1.0 / 6.0), R(2.0 / 3.0), R(1.0 / 6.0)};
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
  // Three samples per trip: their loads are in flight together, while the
  // states of all nine are never live together.
#pragma unroll 3
  for (int q = 0; q < 9; ++q) {
    const int a = q % 3, b = q / 3;
    R fq = f[0];
#pragma unroll
    for (int r = 1; r < 9; ++r) fq = q == r ? f[r] : fq;
    R P[NV];
    Psiat(a, b, P);
#pragma unroll
    for (int c = 1; c < NV; ++c) S[c] += fq * P[c];
  }
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
// FVS in direction n at a point with line neighbours w0..w4 (offsets -h,
// -h/2, 0, h/2, h):
//   R = D+F+ + D-F- = [F0 - 4F1 + 4F3 - F4 + alpha (w0 - 4w1 + 6w2 - 4w3 + w4)] / (2h)
//   alpha = max spectral radius over the five, div part (B0 - 4B1 + 4B3 - B4)/(2h).
// Central direction: R = (F(up) - F(dn))/h, div part (B(up) - B(dn))/h.
// The first-order LLF state uses the four neighbours of the point (the
// line neighbours at +-h for FVS directions, at +-h/2 for the central one).
constexpr int PB = 16, PNT = PB * PB;
constexpr int RF = 12;  // exchange fields of the cell tile: record (4) + LLF flux (8)

// Point accumulators: high-order RHS h = -R_x - R_y with the div part, and
// the LLF update l = -dt/dx G_x - dt/dy G_y with its div part.
template <class R>
struct PointAcc {
  R h[NV], l[NV];
  R divh, divl;
};

template <class R>
__device__ __forceinline__ void acc_zero(PointAcc<R>& P) {
#pragma unroll
  for (int c = 0; c < NV; ++c) P.h[c] = P.l[c] = R(0);
  P.divh = P.divl = R(0);
}

// High-order and LLF states from the accumulators (the right-hand sides in
// the compute type, the states in FP64), scaling limiter, SSP combination,
// store.
// Un: the point's U^n (used only when ca != 0), loaded by the caller one
// phase ahead so that its latency overlaps other work.
template <class R>
__device__ __forceinline__ void finish(const Geo& g, double dt, const double U0[NV], const PointAcc<R>& P,
                                      double ca, double cb, const double Un[NV], double* __restrict__ out,
                                      long plane, long off, Counters* cn, double* wmax) {
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
  if (!in_G_fast(UL)) count(&cn->n_llf_not_admissible);
  limit_point(UH, UL, g.gm1, W, cn, true);
  if (!in_G_fast(W)) count(&cn->n_not_admissible);
  if (ca != 0.0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) W[c] = ca * Un[c] + cb * W[c];
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) out[c * plane + off] = W[c];
  // a step's last stage: the next step's wave-speed maximum over its outputs
  if (wmax) *wmax = fmax(*wmax, dt_speed(W, g));
}

__device__ __forceinline__ int clamp_pt(int i, int np) { return i < -1 ? -1 : (i > np ? np : i); }

// LDS layout (fields of PB x PB values of the compute type): states of the
// tile's V, X, Y and centre values, then the records of the line family in
// flight (see points_tile_lean).
constexpr int SV_ = 0, SX_ = 8, SY_ = 16, SC_ = 24;
template <class R>
constexpr int point_fields() { return 40; }

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

// ---------------------------------- point tile with rebuilt evaluations
// LDS holds the tile's V, X, Y and centre states (32 fields of the compute
// type R) and, for the one line family in flight, the record
// (1/rho, p, c_f, sqrt(rho)) of its two point types (8 fields): 40 x PB x PB
// values, 80 KB for the FP64 stage (two workgroups per CU), 40 KB for the
// FP32-bulk one.  A point's flux, v_n and spectral radius in the family's
// direction are rebuilt from its state and record with the operations of
// eval_dir (for FP64 bit for bit).  The families run in the order b, c, a,
// d, which keeps at most two point accumulators live: b's records are
// formed from the values the tile load brings and its line sums share the
// centre-value phase (they read no centre value); c, a and d each take a
// barrier pair (records, then line sums).  A point is finished (limiter,
// SSP combination, store) after the next family's records, its U^n loaded
// just before them.
// FP32-bulk: states and records in FP32; a thread's own FP64 states (for the
// records, whose pressure recovery is FP64, and for the finish) and its FP64
// centre value stay in registers from the tile load.
constexpr int LQ0 = 32, LQ1 = 36;

// Flux of a state held in any type S (the FP64 stage: S = R = double, the
// operations of flux_from).
template <class R, class S>
__device__ __forceinline__ void flux_of(const S U[NV], int dir, R v1, R v2, R v3, R pt, R F[NV]) {
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

// (1/rho, p, c_f in direction dir, sqrt(rho)) of an FP64 state, as in
// eval_dir.
template <class R>
__device__ __forceinline__ void rec_eval(const double U[NV], const Geo& g, int dir, R q[4]) {
  R ri, v1, v2, v3, b2, p;
  prim_r<R>(U, g.gm1, ri, v1, v2, v3, b2, p);
  const R Bn = dir ? (R)U[5] : (R)U[4];
  const R c2 = (R)g.gamma * p * ri;
  const R s = c2 + b2 * ri;
  R disc = s * s - R(4) * c2 * Bn * Bn * ri;
  disc = disc > R(0) ? disc : R(0);
  q[0] = ri;
  q[1] = p;
  q[2] = sqrt_r(R(0.5) * (s + sqrt_r(disc)));
  q[3] = sqrt_r((R)U[0]);
}

// The directional evaluation of a state from its record.
template <class R>
__device__ __forceinline__ void rec_rebuild(const R U[NV], int dir, const R q[4], DirEvalT<R>& e) {
  const R ri = q[0];
  const R v1 = U[1] * ri, v2 = U[2] * ri, v3 = U[3] * ri;
  const R b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  flux_of<R, R>(U, dir, v1, v2, v3, q[1] + R(0.5) * b2, e.F);
  const R vn = dir ? v2 : v1;
  e.cf = q[2];
  e.vn = vn;
  e.sr = fabs(vn) + q[2];
  e.sq = q[3];
}

// The directional evaluation of an FP64 state from its record, with the
// operations of eval_dir for either compute type (|B|^2 summed in FP64).
template <class R>
__device__ __forceinline__ void rec_rebuild_d(const double U[NV], int dir, const R q[4], DirEvalT<R>& e) {
  const R ri = q[0];
  const R v1 = (R)U[1] * ri, v2 = (R)U[2] * ri, v3 = (R)U[3] * ri;
  const R b2 = (R)(U[4] * U[4] + U[5] * U[5] + U[6] * U[6]);
  flux_of<R, double>(U, dir, v1, v2, v3, q[1] + R(0.5) * b2, e.F);
  const R vn = dir ? v2 : v1;
  e.cf = q[2];
  e.vn = vn;
  e.sr = fabs(vn) + q[2];
  e.sq = q[3];
}

// State (field base sb) and directional evaluation (record base qb) of the
// tile point (ty, tx).
template <class R>
__device__ __forceinline__ void lean_pt(R (*s)[PB][PB], int sb, int qb, int ty, int tx, int dir, DirEvalT<R>& e,
                                        R U[NV]) {
  lds8(s, sb, ty, tx, U);
  R q[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) q[c] = s[qb + c][ty][tx];
  rec_rebuild(U, dir, q, e);
}

// Records of the tile's own points, FP64 states ua (-> LQ0) and ub (-> LQ1).
template <class R>
__device__ __forceinline__ void lean_records(R (*s)[PB][PB], const Geo& g, int ty, int tx, const double ua[NV],
                                             const double ub[NV], int dir) {
  R q[4];
  rec_eval(ua, g, dir, q);
#pragma unroll
  for (int c = 0; c < 4; ++c) s[LQ0 + c][ty][tx] = q[c];
  rec_eval(ub, g, dir, q);
#pragma unroll
  for (int c = 0; c < 4; ++c) s[LQ1 + c][ty][tx] = q[c];
}

// An empty asm that takes an accumulator as read and rewritten: its value is
// formed before this point, so the arithmetic of a family cannot be sunk
// past the next barrier with the LDS values it reads kept live instead.
template <class T>
__device__ __forceinline__ void pin8(T v[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) asm volatile("" : "+v"(v[c]));
}
template <class R>
__device__ __forceinline__ void pin_acc(PointAcc<R>& P) {
#pragma unroll
  for (int c = 0; c < NV; ++c) asm volatile("" : "+v"(P.h[c]), "+v"(P.l[c]));
  asm volatile("" : "+v"(P.divh), "+v"(P.divl));
}

// FVS line in direction dir through the tile point (ty, tx) of the type with
// state base so and record LQ0; the line's other type (state base sb, record
// LQ1) sits at -h/2 (point (ym, xm)) and +h/2 (the point itself), the own
// type's neighbours at -h (ym, xm) and +h (yp, xp).  alpha (the maximum
// spectral radius over the five) comes first, so that the FVS sums fold
// into one vector,
//   Q = F(-h) - 4F(-h/2) + 4F(+h/2) - F(+h)
//       + alpha (U(-h) - 4U(-h/2) + 6U - 4U(+h/2) + U(+h)),   h-part -= Q/(2h),
// and the outer neighbours (with their LLF fluxes, which need the point's
// own evaluation) come before the inner ones.  CENTRAL: the line's +h/2
// point (the tile point of the other type) also takes its central
// difference across this line, between this point and the +h neighbour,
// into P2 (families b and a), from the same evaluations.
template <class R>
__device__ __forceinline__ R lean_srad(R (*s)[PB][PB], int sb, int qb, int mn, int y, int x) {
  return fabs(s[sb + mn][y][x] * s[qb][y][x]) + s[qb + 2][y][x];
}

template <class R, bool CENTRAL>
__device__ __forceinline__ void lean_fvs(R (*s)[PB][PB], int dir, int so, int sb, int ty, int tx, int ym, int xm,
                                         int yp, int xp, R rh, R lam, PointAcc<R>& P, PointAcc<R>& P2) {
  const int bn = 4 + dir, mn = 1 + dir;
  R alpha = lean_srad(s, so, LQ0, mn, ty, tx);
  alpha = fmax(alpha, lean_srad(s, so, LQ0, mn, ym, xm));
  alpha = fmax(alpha, lean_srad(s, sb, LQ1, mn, ym, xm));
  alpha = fmax(alpha, lean_srad(s, sb, LQ1, mn, ty, tx));
  alpha = fmax(alpha, lean_srad(s, so, LQ0, mn, yp, xp));
  R Q[NV], dB, jl;
  DirEvalT<R> eo, e;
  R Uo[NV], U[NV];
  lean_pt(s, so, LQ0, ty, tx, dir, eo, Uo);
#pragma unroll
  for (int c = 0; c < NV; ++c) Q[c] = R(6) * alpha * Uo[c];
  // -h: LLF flux -F^LLF(U, Uo)
  lean_pt(s, so, LQ0, ym, xm, dir, e, U);
  R al = alpha_llf(e, eo, U, Uo);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    Q[c] += e.F[c] + alpha * U[c];
    P.l[c] += lam * (R(0.5) * (e.F[c] + eo.F[c] - al * (Uo[c] - U[c])));
  }
  dB = U[bn];
  jl = -U[bn];
  // +h: LLF flux F^LLF(Uo, U)
  lean_pt(s, so, LQ0, yp, xp, dir, e, U);
  al = alpha_llf(eo, e, Uo, U);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    Q[c] += alpha * U[c] - e.F[c];
    P.l[c] -= lam * (R(0.5) * (eo.F[c] + e.F[c] - al * (U[c] - Uo[c])));
  }
  dB -= U[bn];
  jl += U[bn];
  pin8(Q);
  pin8(P.l);
  {
    DirEvalT<R> ei;
    R Ui[NV];
    // -h/2, +h/2
    lean_pt(s, sb, LQ1, ym, xm, dir, ei, Ui);
#pragma unroll
    for (int c = 0; c < NV; ++c) Q[c] -= R(4) * (ei.F[c] + alpha * Ui[c]);
    dB -= R(4) * Ui[bn];
    lean_pt(s, sb, LQ1, ty, tx, dir, ei, Ui);
#pragma unroll
    for (int c = 0; c < NV; ++c) Q[c] += R(4) * (ei.F[c] - alpha * Ui[c]);
    dB += R(4) * Ui[bn];
    if constexpr (CENTRAL) {
      // the +h/2 point's central direction between this point (-h/2 from
      // it) and the +h neighbour (+h/2 from it), with their evaluations
      const R ad = alpha_llf(eo, ei, Uo, Ui), au = alpha_llf(ei, e, Ui, U);
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        P2.h[c] += eo.F[c] * rh;
        P2.l[c] += lam * (R(0.5) * (eo.F[c] + ei.F[c] - ad * (Ui[c] - Uo[c])));
      }
      P2.divh -= Uo[bn] * rh;
      P2.divl -= R(0.5) * rh * Uo[bn];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        P2.h[c] -= e.F[c] * rh;
        P2.l[c] -= lam * (R(0.5) * (ei.F[c] + e.F[c] - au * (U[c] - Ui[c])));
      }
      P2.divh += U[bn] * rh;
      P2.divl += R(0.5) * rh * U[bn];
    }
  }
  const R sh = R(0.5) * rh;
#pragma unroll
  for (int c = 0; c < NV; ++c) P.h[c] -= Q[c] * sh;
  P.divh += dB * sh;
  P.divl += jl * sh;
}

// (tx, ty): the thread's place in the tile.  live = false runs the tile's
// arithmetic and barriers but stores nothing and counts nothing (a
// workgroup that runs two tiles side by side and has only one to do).
template <class R>
__device__ __forceinline__ void points_tile_lean(const Geo& g, CState u, CState un, MState out,
                                                 double* __restrict__ src, double dt, double ca, double cb,
                                                 Counters* cn, int bx, int by, R (*s)[PB][PB],
                                                 double* __restrict__ wslot, int tx, int ty, bool live) {
  constexpr bool F32 = IsF32<R>::value;
  double wm = 0.0;
  double* const wmax = wslot ? &wm : nullptr;
  const int i0 = bx * (PB - 2) - 1, j0 = by * (PB - 2) - 1;
  const int i = clamp_pt(i0 + tx, g.nxp), j = clamp_pt(j0 + ty, g.nyp);
  const bool inner = live && tx >= 1 && tx < PB - 1 && ty >= 1 && ty < PB - 1;
  const bool outV = inner && i0 + tx < g.nxp && j0 + ty < g.nyp;
  const bool outX = inner && i0 + tx < g.nxp && j0 + ty < g.ny;
  const bool outY = inner && i0 + tx < g.nx && j0 + ty < g.nyp;
  const double lx = dt * g.rdx, ly = dt * g.rdy;
  const R rdx = (R)g.rdx, rdy = (R)g.rdy, lxr = (R)lx, lyr = (R)ly;
  const int txl = tx > 0 ? tx - 1 : tx, txr = tx < PB - 1 ? tx + 1 : tx;
  const int tyd = ty > 0 ? ty - 1 : ty, tyu = ty < PB - 1 ? ty + 1 : ty;
  // a thread's own FP64 states of type 0 V, 1 X, 2 Y: from LDS for the
  // FP64 stage; kept in registers from the tile load for the FP32-bulk one
  // (whose LDS holds FP32)
  double oV[F32 ? NV : 1], oX[F32 ? NV : 1], oY[F32 ? NV : 1];
  auto own = [&](int which, double U[NV]) {
    if constexpr (F32) {
#pragma unroll
      for (int c = 0; c < NV; ++c) U[c] = which == 0 ? oV[c] : which == 1 ? oX[c] : oY[c];
    } else {
      lds8(s, which == 0 ? SV_ : which == 1 ? SX_ : SY_, ty, tx, U);
    }
  };

  // 0: the tile's raw point values into LDS, and the records of family b
  //    (below) of the thread's own V and X, from the values loaded
  if constexpr (F32) {
    ldV(g, u.v, i, j, oV);
    sts8(s, SV_, ty, tx, oV);
    ldX(g, u.x, i, j, oX);
    sts8(s, SX_, ty, tx, oX);
    ldY(g, u.y, i, j, oY);
    sts8(s, SY_, ty, tx, oY);
    lean_records(s, g, ty, tx, oV, oX, 1);
  } else {
    double wv[NV], wx[NV], w[NV];
    ldV(g, u.v, i, j, wv);
    ldX(g, u.x, i, j, wx);
    ldY(g, u.y, i, j, w);
    sts8(s, SV_, ty, tx, wv);
    sts8(s, SX_, ty, tx, wx);
    sts8(s, SY_, ty, tx, w);
    lean_records(s, g, ty, tx, wv, wx, 1);
  }
  // the cell average of the centre value, in flight during family b
  double A[NV];
  ldA(g, u.a, i, j, A);
  __syncthreads();
  PointAcc<R> PV, PX, PY;

  // b: vertical lines through V and X.  V: FVS in y over V(l-1), X(l-1), V,
  // X(l), V(l+1).  X: central in y between V(k,j) and V(k,j+1).  It reads
  // no centre value, so it shares its barrier interval with phase 1.
  acc_zero(PV);
  acc_zero(PX);
  lean_fvs<R, true>(s, 1, SV_, SX_, ty, tx, tyd, tx, tyu, tx, rdy, lyr, PV, PX);
  pin_acc(PV);
  pin_acc(PX);

  // 1: centre values in FP64 (the last column/row's are never used), read
  //    by the line families c and d after the next barrier; the owner of a
  //    cell also writes the cell's nine-point source for the cell kernel.
  double C[NV];
  {
    double Uc[NV], f[NV], w[NV], q[NV];
    if constexpr (F32) {
#pragma unroll
      for (int c = 0; c < NV; ++c) f[c] = oX[c];
      ldX(g, u.x, i + 1, j, w);
#pragma unroll
      for (int c = 0; c < NV; ++c) Uc[c] = oY[c];
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
#pragma unroll
      for (int c = 0; c < NV; ++c) Uc[c] = oV[c];
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
    limit_centre(Uc, A, g.gm1, C, cn, owner);
    sts8(s, SC_, ty, tx, C);
    if (owner && src) {
      // the cell's nine-point source for the cell kernel, from the tile's
      // point values (in LDS since the barrier above) and this centre value
      auto Bat = [&](int a, int b, R& b1, R& b2) {
        if (a == 1 && b == 1) {
          b1 = (R)C[4];
          b2 = (R)C[5];
          return;
        }
        const int base = b == 1 ? SX_ : (a == 1 ? SY_ : SV_);
        const int yy = b == 2 ? tyu : ty, xx = a == 2 ? txr : tx;
        b1 = s[base + 4][yy][xx];
        b2 = s[base + 5][yy][xx];
      };
      auto Psiat = [&](int a, int b, R P[NV]) {
        if (a == 1 && b == 1) {
          psi(C, P);
          return;
        }
        const int base = b == 1 ? SX_ : (a == 1 ? SY_ : SV_);
        R w[NV];
        lds8(s, base, b == 2 ? tyu : ty, a == 2 ? txr : tx, w);
        psi(w, P);
      };
      R S[NV];
      source_nine<R>(Bat, Psiat, (R)g.rdx, (R)g.rdy, S);
#pragma unroll
      for (int c = 0; c < NV; ++c) src[c * g.sc + (long)j * g.nx + i] = (double)S[c];
    }
  }
  auto own_c = [&](double U[NV]) {
    if constexpr (F32) {
#pragma unroll
      for (int c = 0; c < NV; ++c) U[c] = C[c];
    } else {
      lds8(s, SC_, ty, tx, U);
    }
  };
  double w[NV], w2[NV];
  pin_acc(PV);
  pin_acc(PX);
  __syncthreads();

  // c: horizontal lines through X and C.  X: FVS in x over X(k-1), C(k-1),
  // X, C(k), X(k+1) -> X complete.
  own(1, w);
  own_c(w2);
  lean_records(s, g, ty, tx, w, w2, 0);
  __syncthreads();
  lean_fvs<R, false>(s, 0, SX_, SC_, ty, tx, ty, txl, ty, txr, rdx, lxr, PX, PX);
  // X is complete; its U^n is loaded now and X finished after the next
  // family's records, while the load is in flight
  double unp[NV];
  if (outX && ca != 0.0) ldX(g, un.x, i, j, unp);
  pin_acc(PV);
  pin_acc(PX);
  __syncthreads();

  // a: horizontal lines through V and Y.  V: FVS in x over V(k-1), Y(k-1),
  // V, Y(k), V(k+1) -> V complete.  Y: central in x between V(i,l) and
  // V(i+1,l).
  own(0, w);
  own(2, w2);
  lean_records(s, g, ty, tx, w, w2, 0);
  __syncthreads();
  if (outX) {
    own(1, w);
    finish(g, dt, w, PX, ca, cb, unp, out.x, g.sx, (long)j * g.nxp + i, cn, wmax);
  }
  acc_zero(PY);
  lean_fvs<R, true>(s, 0, SV_, SY_, ty, tx, ty, txl, ty, txr, rdx, lxr, PV, PY);
  pin_acc(PY);
  // V is complete: the same for V over the next family's records
  if (outV && ca != 0.0) ldV(g, un.v, i, j, unp);
  pin_acc(PV);
  __syncthreads();

  // d: vertical lines through Y and C.  Y: FVS in y over Y(l-1), C(l-1), Y,
  // C(l), Y(l+1) -> Y complete.
  own(2, w);
  own_c(w2);
  lean_records(s, g, ty, tx, w, w2, 1);
  __syncthreads();
  if (outV) {
    own(0, w);
    finish(g, dt, w, PV, ca, cb, unp, out.v, g.sv, (long)j * g.nxp + i, cn, wmax);
  }
  // Y's U^n: in flight during the family's line sums
  if (outY && ca != 0.0) ldY(g, un.y, i, j, unp);
  lean_fvs<R, false>(s, 1, SY_, SC_, ty, tx, tyd, tx, tyu, tx, rdy, lyr, PY, PY);
  if (outY) {
    own(2, w);
    finish(g, dt, w, PY, ca, cb, unp, out.y, g.sy, (long)j * g.nx + i, cn, wmax);
  }
  if (wslot) {
    __syncthreads();  // the LDS is reused as the reduction's scratch
    block_max_store(wm, ty * PB + tx, PNT, reinterpret_cast<double*>(&s[0][0][0]), wslot);
  }
}

// One tile of the point update (see above): FP64 stage (R = double) or
// FP32-bulk stage (R = float).
// wslot: null, or where the workgroup's maximum of rho_1/dx + rho_2/dy over
// the values it stores goes (a step's last stage).
template <class R>
__device__ __forceinline__ void points_tile(const Geo& g, CState u, CState un, MState out,
                                            double* __restrict__ src, double dt, double ca, double cb,
                                            Counters* cn, int bx, int by, R (*s)[PB][PB],
                                            double* __restrict__ wslot = nullptr) {
  points_tile_lean<R>(g, u, un, out, src, dt, ca, cb, cn, bx, by, s, wslot, (int)threadIdx.x, (int)threadIdx.y,
                      true);
}

// ------------------------------------------------------ fused cell update
// One launch computes the cell averages of the stage for a tile of
// (CBX-3) x (CBY-3) cells; the block's CBX x CBY threads cover the cells
// whose flux-limiter box is needed plus one trailing row/column whose left
// and bottom interfaces close the region.  Per thread (cell (i,j)):
//   1  shock-sensor indicators of the block's cells and one ring (LDS)
//   2  the cell's nine-point source (written by the point kernel; ghost
//      cells across an outflow boundary compute theirs)
//   3  x-interface at the cell's left: Simpson flux, LLF flux, sensor blend;
//      exchanged with the neighbouring lane so each cell has both of its
//      x-interfaces; then the same for the bottom y-interface, through LDS
//   4  LLF source, sensor blend of the source, flux-limiter steps (1)-(2)
//      -> Lambda
//   5  Lambda exchanged (lanes in x, LDS in y), unique interface
//      coefficients, and the limited update in flux form written as
//        A^new = G - dt S^Lim + sum_I theta_I H_I,
//      G = A - dt/dx (F^LLF_R - F^LLF_L) - dt/dy (F^LLF_U - F^LLF_D),
//      H_L = dt/dx (F^s_L - F^LLF_L), H_R = -dt/dx (F^s_R - F^LLF_R), ...
constexpr int CBX0 = 32, CBY0 = 16;  // the cell tile of the single-grid launch

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

// The nine-point source of cell (i,j) from global memory, the centre value
// C given (the cell kernel's ghost cells across an outflow boundary, whose
// mirrored stencil is a computation of its own).
template <class R>
__device__ void cell_source(const Geo& g, CState u, const double C[NV], int i, int j, R S[NV]) {
  auto at = [&](int a, int b, const double*& base, long& plane, long& off) {
    if (b == 1) {
      base = u.x, plane = g.sx, off = (long)map_cell(j, g.ny, g.bcy) * g.nxp + map_node(i + a / 2, g.nx, g.bcx);
    } else if (a == 1) {
      base = u.y, plane = g.sy, off = (long)map_node(j + b / 2, g.ny, g.bcy) * g.nx + map_cell(i, g.nx, g.bcx);
    } else {
      base = u.v, plane = g.sv,
      off = (long)map_node(j + b / 2, g.ny, g.bcy) * g.nxp + map_node(i + a / 2, g.nx, g.bcx);
    }
  };
  auto Bat = [&](int a, int b, R& b1, R& b2) {
    if (a == 1 && b == 1) {
      b1 = (R)C[4];
      b2 = (R)C[5];
      return;
    }
    const double* base;
    long plane, off;
    at(a, b, base, plane, off);
    b1 = (R)base[4 * plane + off];
    b2 = (R)base[5 * plane + off];
  };
  auto Psiat = [&](int a, int b, R P[NV]) {
    if (a == 1 && b == 1) {
      psi(C, P);
      return;
    }
    const double* base;
    long plane, off;
    at(a, b, base, plane, off);
    double w[NV];
    load8(base, plane, off, w);
    psi(w, P);
  };
  source_nine<R>(Bat, Psiat, (R)g.rdx, (R)g.rdy, S);
}

// The centre value of cell (i,j) from global memory (Section 2.1, limited
// as in remark rmk:cell_center), with the operations of the point tile's.
__device__ void centre_value(const Geo& g, CState u, int i, int j, double C[NV]) {
  double A[NV], Uc[NV], f[NV], w[NV], q[NV];
  ldA(g, u.a, i, j, A);
  ldX(g, u.x, i, j, f);
  ldX(g, u.x, i + 1, j, w);
  ldY(g, u.y, i, j, Uc);
  ldY(g, u.y, i, j + 1, q);
#pragma unroll
  for (int c = 0; c < NV; ++c) f[c] = -4.0 * ((f[c] + w[c]) + (Uc[c] + q[c]));
  ldV(g, u.v, i, j, Uc);
  ldV(g, u.v, i + 1, j, w);
#pragma unroll
  for (int c = 0; c < NV; ++c) Uc[c] += w[c];
  ldV(g, u.v, i, j + 1, q);
  ldV(g, u.v, i + 1, j + 1, w);
#pragma unroll
  for (int c = 0; c < NV; ++c) Uc[c] = (36.0 * A[c] + f[c] - (Uc[c] + (q[c] + w[c]))) * 0.0625;
  limit_centre(Uc, A, g.gm1, C, nullptr, false);
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

// theta^s at an interface between the cells whose indicators are a[q] and
// b[q] (q = phi1x, phi1y, phi2, phi3).
template <class R>
__device__ __forceinline__ R sensor_theta(R kappa, const R a[4], const R b[4], int dir) {
  const R p1 = fmax(a[dir], b[dir]), p2 = fmax(a[2], b[2]), p3 = fmax(a[3], b[3]);
  return exp_r(-kappa * (p1 * p2 + p3));
}

// LDS of one cell tile.  The Lambda exchange is FP64: for the FP64 stage it
// reuses the exchange buffer, for the FP32-bulk stage it has its own.
template <class R, int CBX, int CBY>
struct CellsLDS {
  R dfx[NV][CBY][CBX];  // theta^s (F_simpson - F^LLF) at the x-interface left of each cell
  R dfy[NV][CBY][CBX];  // ... at the y-interface below it; they give H_L, H_R, H_D, H_U
  R x[RF][CBY][CBX];    // exchange: primitives; records (0-3) and F^LLF (4-11); Lambda (FP64 stage)
  R ts[2][CBY][CBX];    // theta^s at the two interfaces
  R phi[4][CBY + 1][CBX + 1];  // indicator-major: a wavefront's lanes read consecutive words
  double lam[IsF32<R>::value ? 4 : 1][CBY][CBX];
};

// One tile of the cell update: CBX x CBY threads, (CBX-3) x (CBY-3) cells.
// src: the point kernel's nine-point sources, or null (every cell computes
// its own from the stage input, as the ghost cells do).
template <class R, int CBX, int CBY>
__device__ __forceinline__ void cells_tile(const Geo& g, CState u, const double* __restrict__ src,
                                           const double* __restrict__ un, double* __restrict__ out, double dt,
                                           double ca, double cb, Counters* cn, int bx, int by,
                                           CellsLDS<R, CBX, CBY>& L, double* __restrict__ wslot = nullptr) {
  constexpr int CNT = CBX * CBY;
  auto& s_dfx = L.dfx;
  auto& s_dfy = L.dfy;
  auto& s_x = L.x;
  auto& s_ts = L.ts;
  auto& s_phi = L.phi;
  double (*s_lam)[CBY][CBX];
  if constexpr (IsF32<R>::value) {
    s_lam = L.lam;
  } else {
    s_lam = reinterpret_cast<double (*)[CBY][CBX]>(&L.x[0][0][0]);
  }
  // thread (tx, ty) of the CBX x CBY tile: x fastest in the flat thread index
  const int tid = (int)(threadIdx.y * blockDim.x + threadIdx.x), tx = tid % CBX, ty = tid / CBX;
  const int i0 = bx * (CBX - 3) - 1, j0 = by * (CBY - 3) - 1;
  const int i = clamp_cell(i0 + tx, g.nx), j = clamp_cell(j0 + ty, g.ny);
  const bool output = tx >= 1 && tx < CBX - 2 && ty >= 1 && ty < CBY - 2 && i0 + tx < g.nx && j0 + ty < g.ny;
  const int txr = tx + 1 < CBX ? tx + 1 : tx, tyu = ty + 1 < CBY ? ty + 1 : ty;
  const double lx = dt * g.rdx, ly = dt * g.rdy;

  // 1a: sensor primitives on [i0-2, i0+CBX+1) x [j0-2, j0+CBY+1), aliased
  //     onto the exchange buffer
  constexpr int PW = CBX + 3, PH = CBY + 3;
  static_assert(5 * PW * PH <= RF * CBX * CBY, "primitives must fit the exchange buffer");
  R* prim = &s_x[0][0][0];
  {
    // one or two items per thread, the loads of both issued first
    static_assert(CNT < PW * PH && PW * PH <= 2 * CNT, "one or two primitive items per thread");
    const int it2 = tid + CNT;
    const bool two = it2 < PW * PH;
    double U[NV], U2[NV];
    R q[5];
    ldA(g, u.a, clamp_prim(i0 - 2 + tid % PW, g.nx), clamp_prim(j0 - 2 + tid / PW, g.ny), U);
    if (two) ldA(g, u.a, clamp_prim(i0 - 2 + it2 % PW, g.nx), clamp_prim(j0 - 2 + it2 / PW, g.ny), U2);
    sensor_prims(U, g.gamma, q);
#pragma unroll
    for (int m = 0; m < 5; ++m) prim[m * PW * PH + tid] = q[m];
    if (two) {
      sensor_prims(U2, g.gamma, q);
#pragma unroll
      for (int m = 0; m < 5; ++m) prim[m * PW * PH + it2] = q[m];
    }
  }
  __syncthreads();
  // div B of the LLF source (phase 4) from the neighbours' B1, B2: for the
  // FP64 stage from the sensor primitives (they hold B exactly), read before
  // the next barrier, after which the exchange buffer they share is
  // rewritten; for the FP32-bulk stage from memory in phase 4
  double divb = 0.0;
  if constexpr (!IsF32<R>::value) {
    const int pc = (ty + 2) * PW + (tx + 2);
    divb = (prim[3 * PW * PH + pc + 1] - prim[3 * PW * PH + pc - 1]) * (0.5 * g.rdx);
    divb += (prim[4 * PW * PH + pc + PW] - prim[4 * PW * PH + pc - PW]) * (0.5 * g.rdy);
  }
  // the cell's average, nine-point source and first edge point: loaded
  // now, in flight while the indicators are computed
  double A[NV], Sd[NV], w0[NV];
  ldA(g, u.a, i, j, A);
  if (src) ldA(g, src, i, j, Sd);
  ldV(g, u.v, i, j, w0);
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
    for (int q = 0; q < 4; ++q) s_phi[q][b][a] = ph[q];
  }
  __syncthreads();

  double G[NV];
  R S[NV];
  // 2: nine-point source: the point kernel's for the grid's cells; a ghost
  //    cell across an outflow boundary (its mirrored stencil differs from
  //    its image's) computes its own
  if (!src || (g.bcx && (i < 0 || i >= g.nx)) || (g.bcy && (j < 0 || j >= g.ny))) {
    double C[NV];
    centre_value(g, u, i, j, C);
    cell_source(g, u, C, i, j, S);
  } else {
#pragma unroll
    for (int c = 0; c < NV; ++c) S[c] = (R)Sd[c];
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) G[c] = A[c];

  // 3: interfaces.  dir 0: the x-interface left of the cell, dir 1: the
  //    y-interface below it.  The cell's record (1/rho, p, c_f, sqrt(rho))
  //    goes to the neighbour on the other side, which rebuilds the cell's
  //    directional evaluation from it and the average it loads anyway; the
  //    interface's LLF flux goes back for that cell's update.  In x the two
  //    cells are neighbouring lanes of one wavefront (a tile row is 16 or 32
  //    lanes), so both travel by lane shuffles, with no barrier; in y they
  //    go through LDS (fields 0-3 and 4-11 of the exchange buffer).
  const R kappa = (R)g.kappa;
  // w0 = V(i,j): the first edge point of both interfaces
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    R Fl[NV];
    {
      DirEvalT<R> eA, eN;
      double AN[NV], w1[NV], w2[NV];
      R q[4];
      // the neighbour's average and the interface's edge points are loaded
      // first, together: in flight across the record exchange
      if (dir == 0) {
        ldA(g, u.a, i - 1, j, AN);
        ldX(g, u.x, i, j, w1);
        ldV(g, u.v, i, j + 1, w2);
      } else {
        ldA(g, u.a, i, j - 1, AN);
        ldY(g, u.y, i, j, w1);
        ldV(g, u.v, i + 1, j, w2);
      }
      rec_eval(A, g, dir, q);
      if (dir == 1) {
#pragma unroll
        for (int c = 0; c < 4; ++c) s_x[c][ty][tx] = q[c];
      }
      rec_rebuild_d(A, dir, q, eA);
      if (dir == 0) {
        // the left neighbour's record: lane tx - 1 (meaningless for tx = 0,
        // which evaluates its neighbour itself)
#pragma unroll
        for (int c = 0; c < 4; ++c) q[c] = __shfl_up(q[c], 1);
      } else {
        __syncthreads();
        if (ty > 0) {
#pragma unroll
          for (int c = 0; c < 4; ++c) q[c] = s_x[c][ty - 1][tx];
        }
      }
      if ((dir == 0 ? tx : ty) > 0) {
        rec_rebuild_d(AN, dir, q, eN);
      } else {
        eval_dir(AN, g, dir, eN);
      }
      R dF[NV];
      R pa[4], pb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pa[q] = dir == 0 ? s_phi[q][ty + 1][tx] : s_phi[q][ty][tx + 1];
        pb[q] = s_phi[q][ty + 1][tx + 1];
      }
      const R ts = sensor_theta(kappa, pa, pb, dir);
      interface_flux(g, dir, w0, w1, w2, eN, AN, eA, A, ts, Fl, dF);
      s_ts[dir][ty][tx] = ts;
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        (dir == 0 ? s_dfx : s_dfy)[c][ty][tx] = dF[c];
        if (dir == 1) s_x[4 + c][ty][tx] = Fl[c];
      }
    }
    const double lam = dir == 0 ? lx : ly;
    if (dir == 0) {
      // the right neighbour's flux: lane tx + 1 (the last column, whose
      // update is never used, takes its own)
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        const R fr = __shfl_down(Fl[c], 1);
        G[c] += lam * (double)(Fl[c] - (tx + 1 < CBX ? fr : Fl[c]));
      }
    } else {
      __syncthreads();
#pragma unroll
      for (int c = 0; c < NV; ++c) G[c] += lam * (double)(Fl[c] - s_x[4 + c][tyu][tx]);
    }
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
  {
    R P[NV];
    if constexpr (IsF32<R>::value) {
      double AN[NV], b;
      ldA(g, u.a, i + 1, j, AN);
      b = AN[4];
      ldA(g, u.a, i - 1, j, AN);
      divb = (b - AN[4]) * (0.5 * g.rdx);
      ldA(g, u.a, i, j + 1, AN);
      b = AN[5];
      ldA(g, u.a, i, j - 1, AN);
      divb += (b - AN[5]) * (0.5 * g.rdy);
    }
    psi(A, P);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      Sl[c] = (R)divb * P[c];
      S[c] = tsmin * S[c] + (R(1) - tsmin) * Sl[c];
    }
  }
  double A1[NV], er, ep;
  const double th = source_step(G, S, Sl, dt, g.gm1, A1, er, ep, cn, output);
  double SL[NV];  // S^Lim
#pragma unroll
  for (int c = 0; c < NV; ++c) SL[c] = th * (double)S[c] + (1.0 - th) * (double)Sl[c];
  double Lam[4];
  limiter_box(A1, H, g.gm1, er, ep, Lam, cn, output);
  // 5: unique interface coefficients and the limited update: Lambda_R of
  //    the left neighbour and Lambda_L of the right one by lane shuffles,
  //    Lambda_U of the cell below and Lambda_D of the cell above through LDS
  const double lamR_left = __shfl_up(Lam[1], 1), lamL_right = __shfl_down(Lam[0], 1);
  s_lam[2][ty][tx] = Lam[2];
  s_lam[3][ty][tx] = Lam[3];
  __syncthreads();
  double wm = 0.0;
  if (output) {
  const double thL = fmin(lamR_left, Lam[0]);
  const double thR = fmin(Lam[1], lamL_right);
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
  if (!in_G_fast(An)) count(&cn->n_not_admissible);
  const long off = (long)j * g.nx + i;
  if (ca != 0.0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) An[c] = ca * un[c * g.sc + off] + cb * An[c];
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) out[c * g.sc + off] = An[c];
  if (wslot) wm = dt_speed(An, g);
  }
  if (wslot) {
    __syncthreads();  // the Lambda exchange is read; its LDS is the scratch
    block_max_store(wm, tid, CNT, reinterpret_cast<double*>(&L.ts[0][0][0]), wslot);
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


}  // namespace afm
