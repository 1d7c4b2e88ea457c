// af_adjoint_stage.h -- the entities of one recorded stage and of its
// reverse sweep (see af_adjoint.h for the entity list and conventions).
//
// A stage computes out = a Un + b FE(Uk, dt).  The recording forward writes
// the tape: the limited centre values, the interface fluxes and sensor
// coefficients, the sources, the limiter coefficients and Newton roots, and
// the decision bits of every limiter and of the sensor.  The reverse sweep
// takes lam_out (the adjoint of out) and accumulates
//   lam_n += a lam_out,   lam_k += b (dFE/dUk)^T lam_out
// with every decision read back from the tape.
#pragma once

#include "af_adjoint.h"

namespace afadj {

// Widths and heights of the extended entity grids.
struct Ext {
  int sw, sh;  // sensor cells [-2, nx+2) x [-2, ny+2)
  int xw, xh;  // x-interfaces [-1, nx+2) x [-1, ny+1)
  int yw, yh;  // y-interfaces [-1, nx+1) x [-1, ny+2)
  int ew, eh;  // limiter cells [-1, nx+1) x [-1, ny+1)
};
AF_HD Ext ext_of(const AGeo& g) { return {g.nx + 4, g.ny + 4, g.nx + 3, g.ny + 2, g.nx + 2, g.ny + 3, g.nx + 2, g.ny + 2}; }
AF_HD size_t sidx(const Ext& e, int i, int j) { return (size_t)(j + 2) * e.sw + (i + 2); }
AF_HD size_t xidx(const Ext& e, int k, int j) { return (size_t)(j + 1) * e.xw + (k + 1); }
AF_HD size_t yidx(const Ext& e, int i, int l) { return (size_t)(l + 1) * e.yw + (i + 1); }
AF_HD size_t eidx(const Ext& e, int i, int j) { return (size_t)(j + 1) * e.ew + (i + 1); }

// The tape of one stage.  Planes of 8 components are [8][entities].
struct Tape {
  double* C;           // [8][ny*nx] limited centre values
  uint32_t* cfl;       // [ny*nx] centre limiter decisions
  uint32_t* pfl[3];    // point limiter decisions of the X, Y, V sets
  double* phi;         // [4][ns] phi1x, phi1y, phi2, phi3
  uint32_t* sfl;       // [ns]
  double* xFh;         // [8][nxi] Simpson fluxes
  double* xFl;         // [8][nxi] LLF fluxes
  double* xts;         // [nxi] sensor coefficients
  uint32_t* xfl;       // [nxi]
  double* yFh;
  double* yFl;
  double* yts;
  uint32_t* yfl;
  double* S;           // [8][ne] high-order source
  double* Sllf;        // [8][ne] first-order source
  double* thsrc;       // [ne] source coefficient
  double* Lam;         // [4][ne] Lambda_L, R, D, U
  double* rk;          // [15][ne] vertex roots (1 where feasible)
  uint64_t* lfl;       // [ne] limiter decisions
};
// Adjoints of the intermediate quantities of the reverse sweep.
struct AdjBuf {
  double* lC;    // [8][ny*nx]
  double* lphi;  // [4][ns]
  double* xlFs;  // [8][nxi]
  double* xlFl;  // [8][nxi]
  double* xlts;  // [nxi]
  double* ylFs;
  double* ylFl;
  double* ylts;
  double* lLam;  // [4][ne]
  double* lth;   // [ne]
  double* lSs;   // [8][ne]
  double* lSll;  // [8][ne]
};

struct Sizes {
  size_t cells, ns, nxi, nyi, ne, set[4];
};
inline Sizes sizes_of(const AGeo& g) {
  const Ext e = ext_of(g);
  Sizes s;
  s.cells = (size_t)g.nx * g.ny;
  s.ns = (size_t)e.sw * e.sh;
  s.nxi = (size_t)e.xw * e.xh;
  s.nyi = (size_t)e.yw * e.yh;
  s.ne = (size_t)e.ew * e.eh;
  s.set[0] = (size_t)g.nx * g.ny;
  s.set[1] = (size_t)g.nxp * g.ny;
  s.set[2] = (size_t)g.nx * g.nyp;
  s.set[3] = (size_t)g.nxp * g.nyp;
  return s;
}
// Carve a tape out of base (nullptr: only measure).  Returns the bytes used.
inline size_t tape_layout(const AGeo& g, char* base, Tape* t) {
  const Sizes s = sizes_of(g);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  Tape x;
  x.C = (double*)take(8 * s.cells * sizeof(double));
  x.cfl = (uint32_t*)take(s.cells * sizeof(uint32_t));
  x.pfl[0] = (uint32_t*)take(s.set[1] * sizeof(uint32_t));
  x.pfl[1] = (uint32_t*)take(s.set[2] * sizeof(uint32_t));
  x.pfl[2] = (uint32_t*)take(s.set[3] * sizeof(uint32_t));
  x.phi = (double*)take(4 * s.ns * sizeof(double));
  x.sfl = (uint32_t*)take(s.ns * sizeof(uint32_t));
  x.xFh = (double*)take(8 * s.nxi * sizeof(double));
  x.xFl = (double*)take(8 * s.nxi * sizeof(double));
  x.xts = (double*)take(s.nxi * sizeof(double));
  x.xfl = (uint32_t*)take(s.nxi * sizeof(uint32_t));
  x.yFh = (double*)take(8 * s.nyi * sizeof(double));
  x.yFl = (double*)take(8 * s.nyi * sizeof(double));
  x.yts = (double*)take(s.nyi * sizeof(double));
  x.yfl = (uint32_t*)take(s.nyi * sizeof(uint32_t));
  x.S = (double*)take(8 * s.ne * sizeof(double));
  x.Sllf = (double*)take(8 * s.ne * sizeof(double));
  x.thsrc = (double*)take(s.ne * sizeof(double));
  x.Lam = (double*)take(4 * s.ne * sizeof(double));
  x.rk = (double*)take(15 * s.ne * sizeof(double));
  x.lfl = (uint64_t*)take(s.ne * sizeof(uint64_t));
  if (t) *t = x;
  return off;
}
inline size_t adjbuf_layout(const AGeo& g, char* base, AdjBuf* a) {
  const Sizes s = sizes_of(g);
  size_t off = 0;
  auto take = [&](size_t n) -> double* {
    double* p = base ? (double*)(base + off) : nullptr;
    off += (n * sizeof(double) + 255) & ~(size_t)255;
    return p;
  };
  AdjBuf x;
  x.lC = take(8 * s.cells);
  x.lphi = take(4 * s.ns);
  x.xlFs = take(8 * s.nxi);
  x.xlFl = take(8 * s.nxi);
  x.xlts = take(s.nxi);
  x.ylFs = take(8 * s.nyi);
  x.ylFl = take(8 * s.nyi);
  x.ylts = take(s.nyi);
  x.lLam = take(4 * s.ne);
  x.lth = take(s.ne);
  x.lSs = take(8 * s.ne);
  x.lSll = take(8 * s.ne);
  if (a) *a = x;
  return off;
}

struct StateC {
  const double *a, *x, *y, *v;
};
struct StateM {
  double *a, *x, *y, *v;
};

// A stencil slot of the reverse sweep: where a state is read and where its
// adjoint is added (the centre values come from the tape, their adjoints go
// to the workspace buffer).
struct Slot {
  const double* src;
  double* dst;
  Loc L;
};
template <class Add>
AF_HD void slot_put(const Slot& q, const double* l) {
  put<Add>(q.dst, q.L, l);
}

AF_HD void ldC(const AGeo& g, const Tape& t, int i, int j, double* u) {
  const size_t id = (size_t)mcell(j, g.ny, g.bcy) * g.nx + mcell(i, g.nx, g.bcx);
  for (int c = 0; c < NV; ++c) u[c] = t.C[id + c * (size_t)g.nx * g.ny];
}
template <class Add>
AF_HD void putC(const AGeo& g, double* lC, int i, int j, const double* l) {
  put<Add>(lC, locA(g, i, j), l);
}
AF_HD void ld8(const double* p, size_t id, size_t n, double* u) {
  for (int c = 0; c < NV; ++c) u[c] = p[id + c * n];
}
AF_HD void st8(double* p, size_t id, size_t n, const double* u) {
  for (int c = 0; c < NV; ++c) p[id + c * n] = u[c];
}
template <class Add>
AF_HD void add8(double* p, size_t id, size_t n, const double* u) {
  for (int c = 0; c < NV; ++c)
    if (u[c] != 0.0) Add::add(p + id + c * n, u[c]);
}
AF_HD double combine(double a, double b, double un, double fe) {
  return (a == 0.0 && b == 1.0) ? fe : a * un + b * fe;
}

// ------------------------------------------------------------ recording
// Centre (i, j), a real cell.
AF_HD void centre_inputs(const AGeo& g, const StateC& u, int i, int j, double in[9][NV]) {
  ld(u.a, locA(g, i, j), in[0]);
  ld(u.x, locX(g, i, j), in[1]);
  ld(u.x, locX(g, i + 1, j), in[2]);
  ld(u.y, locY(g, i, j), in[3]);
  ld(u.y, locY(g, i, j + 1), in[4]);
  ld(u.v, locV(g, i, j), in[5]);
  ld(u.v, locV(g, i + 1, j), in[6]);
  ld(u.v, locV(g, i, j + 1), in[7]);
  ld(u.v, locV(g, i + 1, j + 1), in[8]);
}
AF_HD void rec_centre(const AGeo& g, const StateC& u, const Tape& t, int i, int j) {
  double in[9][NV], Uc[NV], C[NV];
  centre_inputs(g, u, i, j, in);
  const double* p[9] = {in[0], in[1], in[2], in[3], in[4], in[5], in[6], in[7], in[8]};
  centre_raw(p, Uc);
  uint32_t fl = 0;
  centre_limit(in[0], Uc, g.gamma, C, fl);
  const size_t id = (size_t)j * g.nx + i, n = (size_t)g.nx * g.ny;
  st8(t.C, id, n, C);
  t.cfl[id] = fl;
}

// Point stencils.  kind 0: X(k,j), 1: Y(i,l), 2: V(k,l).
struct PointSt {
  double U[NV];
  double wx[5][NV], wy[5][NV];  // FVS lines (V: both; X: wx; Y: wy)
  double ca[NV], cb[NV];        // central states (X: V(k,j), V(k,j+1); Y: V(i,l), V(i+1,l))
  double L[NV], R[NV], D[NV], Up[NV];
};
AF_HD void point_stencil(const AGeo& g, const StateC& u, const Tape& t, int kind, int k, int l, PointSt& s) {
  if (kind == 0) {
    ld(u.x, locX(g, k, l), s.U);
    ld(u.x, locX(g, k - 1, l), s.wx[0]);
    ldC(g, t, k - 1, l, s.wx[1]);
    ld(u.x, locX(g, k, l), s.wx[2]);
    ldC(g, t, k, l, s.wx[3]);
    ld(u.x, locX(g, k + 1, l), s.wx[4]);
    ld(u.v, locV(g, k, l), s.ca);
    ld(u.v, locV(g, k, l + 1), s.cb);
    ld(u.x, locX(g, k - 1, l), s.L);
    ld(u.x, locX(g, k + 1, l), s.R);
    ld(u.v, locV(g, k, l), s.D);
    ld(u.v, locV(g, k, l + 1), s.Up);
  } else if (kind == 1) {
    ld(u.y, locY(g, k, l), s.U);
    ld(u.y, locY(g, k, l - 1), s.wy[0]);
    ldC(g, t, k, l - 1, s.wy[1]);
    ld(u.y, locY(g, k, l), s.wy[2]);
    ldC(g, t, k, l, s.wy[3]);
    ld(u.y, locY(g, k, l + 1), s.wy[4]);
    ld(u.v, locV(g, k, l), s.ca);
    ld(u.v, locV(g, k + 1, l), s.cb);
    ld(u.v, locV(g, k, l), s.L);
    ld(u.v, locV(g, k + 1, l), s.R);
    ld(u.y, locY(g, k, l - 1), s.D);
    ld(u.y, locY(g, k, l + 1), s.Up);
  } else {
    ld(u.v, locV(g, k, l), s.U);
    ld(u.v, locV(g, k - 1, l), s.wx[0]);
    ld(u.y, locY(g, k - 1, l), s.wx[1]);
    ld(u.v, locV(g, k, l), s.wx[2]);
    ld(u.y, locY(g, k, l), s.wx[3]);
    ld(u.v, locV(g, k + 1, l), s.wx[4]);
    ld(u.v, locV(g, k, l - 1), s.wy[0]);
    ld(u.x, locX(g, k, l - 1), s.wy[1]);
    ld(u.v, locV(g, k, l), s.wy[2]);
    ld(u.x, locX(g, k, l), s.wy[3]);
    ld(u.v, locV(g, k, l + 1), s.wy[4]);
    ld(u.v, locV(g, k - 1, l), s.L);
    ld(u.v, locV(g, k + 1, l), s.R);
    ld(u.v, locV(g, k, l - 1), s.D);
    ld(u.v, locV(g, k, l + 1), s.Up);
  }
}
// High-order point update U^H = U + dt (-R1 - R2 - div B Psi(U)).
AF_HD void point_high(const AGeo& g, int kind, const PointSt& s, double dt, double* H) {
  double R1[NV], R2[NV], d1, d2, P[NV];
  const double* wx[5] = {s.wx[0], s.wx[1], s.wx[2], s.wx[3], s.wx[4]};
  const double* wy[5] = {s.wy[0], s.wy[1], s.wy[2], s.wy[3], s.wy[4]};
  if (kind != 1) fvs_line(wx, g.gamma, 0, g.dx, R1, d1);
  if (kind != 0) fvs_line(wy, g.gamma, 1, g.dy, R2, d2);
  if (kind == 0) {
    double Fd[NV], Fu[NV];
    flux(s.ca, g.gamma, 1, Fd);
    flux(s.cb, g.gamma, 1, Fu);
    for (int c = 0; c < NV; ++c) R2[c] = (Fu[c] - Fd[c]) / g.dy;
    d2 = (s.cb[5] - s.ca[5]) / g.dy;
  } else if (kind == 1) {
    double Fl[NV], Fr[NV];
    flux(s.ca, g.gamma, 0, Fl);
    flux(s.cb, g.gamma, 0, Fr);
    for (int c = 0; c < NV; ++c) R1[c] = (Fr[c] - Fl[c]) / g.dx;
    d1 = (s.cb[4] - s.ca[4]) / g.dx;
  }
  const double divB = d1 + d2;
  psi(s.U, P);
  for (int c = 0; c < NV; ++c) H[c] = s.U[c] + dt * (-R1[c] - R2[c] - divB * P[c]);
}
AF_HD size_t point_id(const AGeo& g, int kind, int k, int l) {
  return kind == 0 ? (size_t)l * g.nxp + k : kind == 1 ? (size_t)l * g.nx + k : (size_t)l * g.nxp + k;
}
AF_HD size_t point_n(const AGeo& g, int kind) {
  return kind == 0 ? (size_t)g.nxp * g.ny : kind == 1 ? (size_t)g.nx * g.nyp : (size_t)g.nxp * g.nyp;
}
AF_HD void rec_point(const AGeo& g, const StateC& un, const StateC& u, const Tape& t, double* out, int kind, int k,
                     int l, double dt, double a, double b) {
  PointSt s;
  point_stencil(g, u, t, kind, k, l, s);
  double H[NV], Lf[NV], W[NV];
  point_high(g, kind, s, dt, H);
  point_llf(s.U, s.L, s.R, s.D, s.Up, dt, g, Lf);
  uint32_t fl = 0;
  point_limit(H, Lf, g.gamma, W, fl);
  const size_t id = point_id(g, kind, k, l), n = point_n(g, kind);
  const double* unp = kind == 0 ? un.x : kind == 1 ? un.y : un.v;
  for (int c = 0; c < NV; ++c) out[id + c * n] = combine(a, b, unp[id + c * n], W[c]);
  t.pfl[kind][id] = fl;
}

// Sensor of (possibly ghost) cell (i, j).
AF_HD void sensor_inputs(const AGeo& g, const StateC& u, int i, int j, double in[5][NV]) {
  ld(u.a, locA(g, i, j), in[0]);
  ld(u.a, locA(g, i - 1, j), in[1]);
  ld(u.a, locA(g, i + 1, j), in[2]);
  ld(u.a, locA(g, i, j - 1), in[3]);
  ld(u.a, locA(g, i, j + 1), in[4]);
}
AF_HD void rec_sensor(const AGeo& g, const StateC& u, const Tape& t, int i, int j) {
  const Ext e = ext_of(g);
  double in[5][NV], phi[4];
  sensor_inputs(g, u, i, j, in);
  uint32_t fl = 0;
  sensor(in[0], in[1], in[2], in[3], in[4], g, phi, fl);
  const size_t id = sidx(e, i, j), n = (size_t)e.sw * e.sh;
  for (int q = 0; q < 4; ++q) t.phi[id + q * n] = phi[q];
  t.sfl[id] = fl;
}
AF_HD void ldphi(const Ext& e, const double* phi, int i, int j, double* p) {
  const size_t id = sidx(e, i, j), n = (size_t)e.sw * e.sh;
  for (int q = 0; q < 4; ++q) p[q] = phi[id + q * n];
}

// Interface (dir 0: x-interface k of row j; dir 1: y-interface l of column i,
// called with (i, l)).  Simpson flux over the three points of the face, LLF
// flux of the adjacent cell averages, sensor coefficient.
AF_HD void iface_inputs(const AGeo& g, const StateC& u, int dir, int k, int j, double p[3][NV], double* Al,
                        double* Ar) {
  if (dir == 0) {
    ld(u.v, locV(g, k, j), p[0]);
    ld(u.x, locX(g, k, j), p[1]);
    ld(u.v, locV(g, k, j + 1), p[2]);
    ld(u.a, locA(g, k - 1, j), Al);
    ld(u.a, locA(g, k, j), Ar);
  } else {
    ld(u.v, locV(g, k, j), p[0]);
    ld(u.y, locY(g, k, j), p[1]);
    ld(u.v, locV(g, k + 1, j), p[2]);
    ld(u.a, locA(g, k, j - 1), Al);
    ld(u.a, locA(g, k, j), Ar);
  }
}
AF_HD void rec_iface(const AGeo& g, const StateC& u, const Tape& t, int dir, int k, int j) {
  const Ext e = ext_of(g);
  double p[3][NV], Al[NV], Ar[NV], Fa[NV], Fb[NV], Fc[NV], Fh[NV], Fl[NV], pL[4], pR[4];
  iface_inputs(g, u, dir, k, j, p, Al, Ar);
  flux(p[0], g.gamma, dir, Fa);
  flux(p[1], g.gamma, dir, Fb);
  flux(p[2], g.gamma, dir, Fc);
  for (int c = 0; c < NV; ++c) Fh[c] = (Fa[c] + 4.0 * Fb[c] + Fc[c]) / 6.0;
  llf(Al, Ar, g.gamma, dir, Fl);
  if (dir == 0) {
    ldphi(e, t.phi, k - 1, j, pL);
    ldphi(e, t.phi, k, j, pR);
  } else {
    ldphi(e, t.phi, k, j - 1, pL);
    ldphi(e, t.phi, k, j, pR);
  }
  uint32_t fl = 0;
  const double ts = sensor_theta(pL, pR, dir, g.kappa, fl);
  const size_t id = dir == 0 ? xidx(e, k, j) : yidx(e, k, j);
  const size_t n = dir == 0 ? (size_t)e.xw * e.xh : (size_t)e.yw * e.yh;
  st8(dir == 0 ? t.xFh : t.yFh, id, n, Fh);
  st8(dir == 0 ? t.xFl : t.yFl, id, n, Fl);
  (dir == 0 ? t.xts : t.yts)[id] = ts;
  (dir == 0 ? t.xfl : t.yfl)[id] = fl;
}
// Blended flux Fs = ts Fh + (1 - ts) Fl and Fl of an interface from the tape.
struct IfaceRef {
  size_t id, n;
  const double *Fh, *Fl, *ts;
};
AF_HD IfaceRef iref(const Ext& e, const Tape& t, int dir, int k, int j) {
  if (dir == 0) return {xidx(e, k, j), (size_t)e.xw * e.xh, t.xFh, t.xFl, t.xts};
  return {yidx(e, k, j), (size_t)e.yw * e.yh, t.yFh, t.yFl, t.yts};
}
AF_HD void ld_iface(const IfaceRef& r, double* Fs, double* Fl, double& ts) {
  ts = r.ts[r.id];
  for (int c = 0; c < NV; ++c) {
    const double fh = r.Fh[r.id + c * r.n];
    Fl[c] = r.Fl[r.id + c * r.n];
    Fs[c] = ts * fh + (1.0 - ts) * Fl[c];
  }
}
// The four interfaces of cell (i, j): L, R, D, U.
AF_HD void cell_irefs(const Ext& e, const Tape& t, int i, int j, IfaceRef r[4]) {
  r[0] = iref(e, t, 0, i, j);
  r[1] = iref(e, t, 0, i + 1, j);
  r[2] = iref(e, t, 1, i, j);
  r[3] = iref(e, t, 1, i, j + 1);
}
// Smallest of the four sensor coefficients, and which (L, R, D, U).
AF_HD double ts_min(const double ts[4], int& arg) {
  const int a1 = ts[1] < ts[0] ? 1 : 0, a2 = ts[3] < ts[2] ? 3 : 2;
  arg = ts[a2] < ts[a1] ? a2 : a1;
  return ts[arg];
}
// The nine points of cell (i, j) (a along x, b along y), centre from the tape.
AF_HD void nine_points(const AGeo& g, const StateC& u, const Tape& t, int i, int j, double P[3][3][NV]) {
  ld(u.v, locV(g, i, j), P[0][0]);
  ld(u.y, locY(g, i, j), P[1][0]);
  ld(u.v, locV(g, i + 1, j), P[2][0]);
  ld(u.x, locX(g, i, j), P[0][1]);
  ldC(g, t, i, j, P[1][1]);
  ld(u.x, locX(g, i + 1, j), P[2][1]);
  ld(u.v, locV(g, i, j + 1), P[0][2]);
  ld(u.y, locY(g, i, j + 1), P[1][2]);
  ld(u.v, locV(g, i + 1, j + 1), P[2][2]);
}
AF_HD double div_bbar(const AGeo& g, const StateC& u, int i, int j) {
  double Al[NV], Ar[NV], Ad[NV], Au[NV];
  ld(u.a, locA(g, i - 1, j), Al);
  ld(u.a, locA(g, i + 1, j), Ar);
  ld(u.a, locA(g, i, j - 1), Ad);
  ld(u.a, locA(g, i, j + 1), Au);
  return (Ar[4] - Al[4]) / (2.0 * g.dx) + (Au[5] - Ad[5]) / (2.0 * g.dy);
}
AF_HD void rec_limiter(const AGeo& g, const StateC& u, const Tape& t, int i, int j, double dt) {
  const Ext e = ext_of(g);
  CellIn w;
  ld(u.a, locA(g, i, j), w.A);
  IfaceRef r[4];
  cell_irefs(e, t, i, j, r);
  double ts[4];
  for (int I = 0; I < 4; ++I) ld_iface(r[I], w.Fs[I], w.Fl[I], ts[I]);
  double P[3][3][NV], S[NV], Q[NV];
  nine_points(g, u, t, i, j, P);
  const double* pp[3][3] = {{P[0][0], P[0][1], P[0][2]}, {P[1][0], P[1][1], P[1][2]}, {P[2][0], P[2][1], P[2][2]}};
  cell_source(pp, g, S);
  const double divb = div_bbar(g, u, i, j);
  psi(w.A, Q);
  int am = 0;
  const double tsc = ts_min(ts, am);
  for (int c = 0; c < NV; ++c) {
    w.Sllf[c] = divb * Q[c];
    w.Ss[c] = tsc * S[c] + (1.0 - tsc) * w.Sllf[c];
  }
  double th, Lam[4], rk[15];
  uint64_t fl = (uint64_t)am << 59;
  cell_limiter(w, dt, g, th, Lam, rk, fl);
  const size_t id = eidx(e, i, j), n = (size_t)e.ew * e.eh;
  st8(t.S, id, n, S);
  st8(t.Sllf, id, n, w.Sllf);
  t.thsrc[id] = th;
  for (int I = 0; I < 4; ++I) t.Lam[id + I * n] = Lam[I];
  for (int k = 0; k < 15; ++k) t.rk[id + k * n] = rk[k];
  t.lfl[id] = fl;
}
// Interface coefficients of cell (i, j): the smaller of the two adjacent
// cells' box entries, ties to the first (L: Lambda_R(i-1) vs Lambda_L(i)).
// src[I] = 0 when the first argument wins.
AF_HD void cell_thetas(const Ext& e, const Tape& t, int i, int j, double th[4], int src[4]) {
  const size_t n = (size_t)e.ew * e.eh;
  auto L = [&](int ii, int jj, int I) { return t.Lam[eidx(e, ii, jj) + I * n]; };
  const double a[4] = {L(i - 1, j, 1), L(i, j, 1), L(i, j - 1, 3), L(i, j, 3)};
  const double b[4] = {L(i, j, 0), L(i + 1, j, 0), L(i, j, 2), L(i, j + 1, 2)};
  for (int I = 0; I < 4; ++I) {
    src[I] = b[I] < a[I] ? 1 : 0;
    th[I] = src[I] ? b[I] : a[I];
  }
}
// The entity and component of Lambda behind interface coefficient I of cell
// (i, j) when taken from argument s (0 first, 1 second).
AF_HD void theta_owner(int i, int j, int I, int s, int& oi, int& oj, int& comp) {
  const int fi[4] = {i - 1, i, i, i}, fj[4] = {j, j, j - 1, j}, fc[4] = {1, 1, 3, 3};
  const int si[4] = {i, i + 1, i, i}, sj[4] = {j, j, j, j + 1}, sc[4] = {0, 0, 2, 2};
  oi = s ? si[I] : fi[I];
  oj = s ? sj[I] : fj[I];
  comp = s ? sc[I] : fc[I];
}
AF_HD void cell_sources(const Ext& e, const Tape& t, int i, int j, const double ts[4], double* Ss, double* Sllf) {
  const size_t id = eidx(e, i, j), n = (size_t)e.ew * e.eh;
  int am;
  const double tsc = ts_min(ts, am);
  for (int c = 0; c < NV; ++c) {
    Sllf[c] = t.Sllf[id + c * n];
    Ss[c] = tsc * t.S[id + c * n] + (1.0 - tsc) * Sllf[c];
  }
}
AF_HD void rec_update(const AGeo& g, const StateC& un, const StateC& u, const Tape& t, double* out, int i, int j,
                      double dt, double a, double b) {
  const Ext e = ext_of(g);
  double A[NV];
  ld(u.a, locA(g, i, j), A);
  IfaceRef r[4];
  cell_irefs(e, t, i, j, r);
  double Fs[4][NV], Fl[4][NV], ts[4], th[4], Ss[NV], Sllf[NV];
  int src[4];
  for (int I = 0; I < 4; ++I) ld_iface(r[I], Fs[I], Fl[I], ts[I]);
  cell_thetas(e, t, i, j, th, src);
  cell_sources(e, t, i, j, ts, Ss, Sllf);
  const double thsrc = t.thsrc[eidx(e, i, j)];
  const double ldx = dt / g.dx, ldy = dt / g.dy;
  const size_t id = (size_t)j * g.nx + i, n = (size_t)g.nx * g.ny;
  for (int c = 0; c < NV; ++c) {
    const double FL = th[0] * Fs[0][c] + (1.0 - th[0]) * Fl[0][c];
    const double FR = th[1] * Fs[1][c] + (1.0 - th[1]) * Fl[1][c];
    const double FD = th[2] * Fs[2][c] + (1.0 - th[2]) * Fl[2][c];
    const double FU = th[3] * Fs[3][c] + (1.0 - th[3]) * Fl[3][c];
    const double S = thsrc * Ss[c] + (1.0 - thsrc) * Sllf[c];
    const double An = A[c] - ldx * (FR - FL) - ldy * (FU - FD) - dt * S;
    out[id + c * n] = combine(a, b, un.a[id + c * n], An);
  }
}

// ------------------------------------------------------------ reverse
// Update of real cell (i, j).
template <class Add>
AF_HD void adj_update(const AGeo& g, const Tape& t, const AdjBuf& ab, const StateC& lo, const StateM& ln,
                      const StateM& lk, int i, int j, double dt, double a, double b) {
  const Ext e = ext_of(g);
  const size_t cid = (size_t)j * g.nx + i, cn = (size_t)g.nx * g.ny;
  double lam[NV];
  for (int c = 0; c < NV; ++c) {
    const double l = lo.a[cid + c * cn];
    if (a != 0.0) Add::add(ln.a + cid + c * cn, a * l);
    lam[c] = b * l;
  }
  add8<Add>(lk.a, cid, cn, lam);
  IfaceRef r[4];
  cell_irefs(e, t, i, j, r);
  double Fs[4][NV], Fl[4][NV], ts[4], th[4], Ss[NV], Sllf[NV];
  int src[4];
  for (int I = 0; I < 4; ++I) ld_iface(r[I], Fs[I], Fl[I], ts[I]);
  cell_thetas(e, t, i, j, th, src);
  cell_sources(e, t, i, j, ts, Ss, Sllf);
  const double ldx = dt / g.dx, ldy = dt / g.dy;
  const double coef[4] = {ldx, -ldx, ldy, -ldy};
  const size_t en = (size_t)e.ew * e.eh;
  for (int I = 0; I < 4; ++I) {
    double lFs[NV], lFl[NV], lth = 0.0;
    for (int c = 0; c < NV; ++c) {
      const double lF = coef[I] * lam[c];
      lth += lF * (Fs[I][c] - Fl[I][c]);
      lFs[c] = th[I] * lF;
      lFl[c] = (1.0 - th[I]) * lF;
    }
    int oi, oj, comp;
    theta_owner(i, j, I, src[I], oi, oj, comp);
    if (lth != 0.0) Add::add(ab.lLam + eidx(e, oi, oj) + comp * en, lth);
    add8<Add>(I < 2 ? ab.xlFs : ab.ylFs, r[I].id, r[I].n, lFs);
    add8<Add>(I < 2 ? ab.xlFl : ab.ylFl, r[I].id, r[I].n, lFl);
  }
  const size_t eid = eidx(e, i, j);
  const double thsrc = t.thsrc[eid];
  double lthsrc = 0.0, lSs[NV], lSl[NV];
  for (int c = 0; c < NV; ++c) {
    const double lS = -dt * lam[c];
    lthsrc += lS * (Ss[c] - Sllf[c]);
    lSs[c] = thsrc * lS;
    lSl[c] = (1.0 - thsrc) * lS;
  }
  if (lthsrc != 0.0) Add::add(ab.lth + eid, lthsrc);
  add8<Add>(ab.lSs, eid, en, lSs);
  add8<Add>(ab.lSll, eid, en, lSl);
}

// The nine points of cell (i, j) as slots (a along x, b along y).
AF_HD void nine_slots(const AGeo& g, const StateC& u, const Tape& t, const AdjBuf& ab, const StateM& lk, int i, int j,
                      Slot q[3][3]) {
  q[0][0] = Slot{u.v, lk.v, locV(g, i, j)};
  q[1][0] = Slot{u.y, lk.y, locY(g, i, j)};
  q[2][0] = Slot{u.v, lk.v, locV(g, i + 1, j)};
  q[0][1] = Slot{u.x, lk.x, locX(g, i, j)};
  q[1][1] = Slot{t.C, ab.lC, locA(g, i, j)};
  q[2][1] = Slot{u.x, lk.x, locX(g, i + 1, j)};
  q[0][2] = Slot{u.v, lk.v, locV(g, i, j + 1)};
  q[1][2] = Slot{u.y, lk.y, locY(g, i, j + 1)};
  q[2][2] = Slot{u.v, lk.v, locV(g, i + 1, j + 1)};
}
// Reverse of the nine-point source, one point at a time: pass 1 forms the
// nine div B values from the normal field components and the adjoints of
// the nine div B's (which need Psi at each point); pass 2 scatters each
// point's adjoint once (its Psi part plus its share of every div B).
template <class Add>
AF_HD void source_reverse(const AGeo& g, const Slot q[3][3], const double* lS) {
  const double w[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  double B1[3][3], B2[3][3], dv[3][3], ldv[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      B1[a][b] = q[a][b].src[q[a][b].L.i + 4 * q[a][b].L.s];
      B2[a][b] = q[a][b].src[q[a][b].L.i + 5 * q[a][b].L.s];
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      dv[a][b] = d3(a, B1[0][b], B1[1][b], B1[2][b]) / g.dx + d3(b, B2[a][0], B2[a][1], B2[a][2]) / g.dy;
      double U[NV], Q[NV];
      ld(q[a][b].src, q[a][b].L, U);
      psi(U, Q);
      double s = 0.0;
      for (int c = 0; c < NV; ++c) s += w[a] * w[b] * lS[c] * Q[c];
      ldv[a][b] = s;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double U[NV], lQ[NV], lU[NV];
      ld(q[a][b].src, q[a][b].L, U);
      for (int c = 0; c < NV; ++c) lQ[c] = w[a] * w[b] * dv[a][b] * lS[c];
      zero8(lU);
      psi_vjp(U, lQ, lU);
      // this point is entry a of row b (B1 derivatives) and entry b of column a (B2)
      double l4 = 0.0, l5 = 0.0;
      for (int p = 0; p < 3; ++p) {
        l4 += d3c(p, a) * ldv[p][b] / g.dx;
        l5 += d3c(p, b) * ldv[a][p] / g.dy;
      }
      lU[4] += l4;
      lU[5] += l5;
      slot_put<Add>(q[a][b], lU);
    }
}

// Reverse of steps (1)-(2) of a limiter cell whose coefficients depend on
// the state (rare).  Scatters the adjoints of A and of the
// four interfaces' fluxes, and adds those of Ss, Sllf to oSs, oSll.
template <class Add>
AF_HD void limiter_active_vjp(const AGeo& g, const StateC& u, const Tape& t, const AdjBuf& ab, const StateM& lk,
                                    int i, int j, double dt, uint64_t fl, double* oSs, double* oSll) {
  const Ext e = ext_of(g);
  const size_t eid = eidx(e, i, j), en = (size_t)e.ew * e.eh;
  CellIn w;
  ld(u.a, locA(g, i, j), w.A);
  IfaceRef r[4];
  cell_irefs(e, t, i, j, r);
  double ts[4];
  for (int I = 0; I < 4; ++I) ld_iface(r[I], w.Fs[I], w.Fl[I], ts[I]);
  cell_sources(e, t, i, j, ts, w.Ss, w.Sllf);
  double rk[15], lLam[4];
  for (int k = 0; k < 15; ++k) rk[k] = t.rk[eid + k * en];
  for (int I = 0; I < 4; ++I) lLam[I] = ab.lLam[eid + I * en];
  CellAdj o;
  zero8(o.A);
  zero8(o.Ss);
  zero8(o.Sllf);
  for (int I = 0; I < 4; ++I) {
    zero8(o.Fs[I]);
    zero8(o.Fl[I]);
  }
  cell_limiter_vjp(w, dt, g, rk, fl, ab.lth[eid], lLam, o);
  for (int I = 0; I < 4; ++I) {
    add8<Add>(I < 2 ? ab.xlFs : ab.ylFs, r[I].id, r[I].n, o.Fs[I]);
    add8<Add>(I < 2 ? ab.xlFl : ab.ylFl, r[I].id, r[I].n, o.Fl[I]);
  }
  put<Add>(lk.a, locA(g, i, j), o.A);
  for (int c = 0; c < NV; ++c) {
    oSs[c] += o.Ss[c];
    oSll[c] += o.Sllf[c];
  }
}

// Limiter cell (i, j), extended range.
template <class Add>
AF_HD void adj_limiter(const AGeo& g, const StateC& u, const Tape& t, const AdjBuf& ab, const StateM& lk, int i, int j,
                       double dt) {
  const Ext e = ext_of(g);
  const size_t eid = eidx(e, i, j), en = (size_t)e.ew * e.eh;
  const uint64_t fl = t.lfl[eid];
  double oSs[NV], oSll[NV];
  ld8(ab.lSs, eid, en, oSs);
  ld8(ab.lSll, eid, en, oSll);
  if (fl & LM_ACTIVE) limiter_active_vjp<Add>(g, u, t, ab, lk, i, j, dt, fl, oSs, oSll);
  // Ss = tsc S + (1 - tsc) Sllf, tsc the smallest sensor coefficient of the cell
  const int am = lm_tsmin(fl);
  const IfaceRef r = iref(e, t, am < 2 ? 0 : 1, am == 1 ? i + 1 : i, am == 3 ? j + 1 : j);
  const double tsc = r.ts[r.id];
  double S[NV], Sllf[NV], lS[NV], ltsc = 0.0;
  ld8(t.S, eid, en, S);
  ld8(t.Sllf, eid, en, Sllf);
  for (int c = 0; c < NV; ++c) {
    ltsc += oSs[c] * (S[c] - Sllf[c]);
    lS[c] = tsc * oSs[c];
    oSll[c] += (1.0 - tsc) * oSs[c];
  }
  if (ltsc != 0.0) Add::add((am < 2 ? ab.xlts : ab.ylts) + r.id, ltsc);
  // Sllf = div Bbar Psi(A)
  double A[NV], Q[NV], lQ[NV], lA[NV], ldiv = 0.0;
  ld(u.a, locA(g, i, j), A);
  psi(A, Q);
  const double divb = div_bbar(g, u, i, j);
  for (int c = 0; c < NV; ++c) {
    ldiv += oSll[c] * Q[c];
    lQ[c] = divb * oSll[c];
  }
  zero8(lA);
  psi_vjp(A, lQ, lA);
  put<Add>(lk.a, locA(g, i, j), lA);
  if (ldiv != 0.0) {
    const Loc Lr = locA(g, i + 1, j), Ll = locA(g, i - 1, j), Lu = locA(g, i, j + 1), Ld = locA(g, i, j - 1);
    Add::add(lk.a + Lr.i + 4 * Lr.s, ldiv / (2.0 * g.dx));
    Add::add(lk.a + Ll.i + 4 * Ll.s, -ldiv / (2.0 * g.dx));
    Add::add(lk.a + Lu.i + 5 * Lu.s, ldiv / (2.0 * g.dy));
    Add::add(lk.a + Ld.i + 5 * Ld.s, -ldiv / (2.0 * g.dy));
  }
  bool any = false;
  for (int c = 0; c < NV; ++c) any = any || lS[c] != 0.0;
  if (any) {
    Slot q[3][3];
    nine_slots(g, u, t, ab, lk, i, j, q);
    source_reverse<Add>(g, q, lS);
  }
}

// Interface, extended range.
template <class Add>
AF_HD void adj_iface(const AGeo& g, const StateC& u, const Tape& t, const AdjBuf& ab, const StateM& lk, int dir, int k,
                     int j) {
  const Ext e = ext_of(g);
  const IfaceRef r = iref(e, t, dir, k, j);
  const double* lFsb = dir == 0 ? ab.xlFs : ab.ylFs;
  const double* lFlb = dir == 0 ? ab.xlFl : ab.ylFl;
  double lFs[NV], lFl[NV], lFh[NV];
  ld8(lFsb, r.id, r.n, lFs);
  ld8(lFlb, r.id, r.n, lFl);
  double lts = (dir == 0 ? ab.xlts : ab.ylts)[r.id];
  const double ts = r.ts[r.id];
  for (int c = 0; c < NV; ++c) {
    const double fh = r.Fh[r.id + c * r.n], fl = r.Fl[r.id + c * r.n];
    lts += lFs[c] * (fh - fl);
    lFh[c] = ts * lFs[c];
    lFl[c] += (1.0 - ts) * lFs[c];
  }
  double p[3][NV], Al[NV], Ar[NV];
  iface_inputs(g, u, dir, k, j, p, Al, Ar);
  double l0[NV], l1[NV], l2[NV], lh[NV], lh4[NV], lAl[NV], lAr[NV];
  zero8(l0);
  zero8(l1);
  zero8(l2);
  zero8(lAl);
  zero8(lAr);
  for (int c = 0; c < NV; ++c) {
    lh[c] = lFh[c] / 6.0;
    lh4[c] = 4.0 * lFh[c] / 6.0;
  }
  flux_vjp(p[0], g.gamma, dir, lh, l0);
  flux_vjp(p[1], g.gamma, dir, lh4, l1);
  flux_vjp(p[2], g.gamma, dir, lh, l2);
  bool anyl = false;
  for (int c = 0; c < NV; ++c) anyl = anyl || lFl[c] != 0.0;
  if (anyl) llf_vjp(Al, Ar, g.gamma, dir, lFl, lAl, lAr);
  if (dir == 0) {
    put<Add>(lk.v, locV(g, k, j), l0);
    put<Add>(lk.x, locX(g, k, j), l1);
    put<Add>(lk.v, locV(g, k, j + 1), l2);
    put<Add>(lk.a, locA(g, k - 1, j), lAl);
    put<Add>(lk.a, locA(g, k, j), lAr);
  } else {
    put<Add>(lk.v, locV(g, k, j), l0);
    put<Add>(lk.y, locY(g, k, j), l1);
    put<Add>(lk.v, locV(g, k + 1, j), l2);
    put<Add>(lk.a, locA(g, k, j - 1), lAl);
    put<Add>(lk.a, locA(g, k, j), lAr);
  }
  if (lts != 0.0 && g.kappa != 0.0) {
    double pL[4], pR[4], lpL[4] = {0.0, 0.0, 0.0, 0.0}, lpR[4] = {0.0, 0.0, 0.0, 0.0};
    const int li = dir == 0 ? k - 1 : k, lj = dir == 0 ? j : j - 1;
    ldphi(e, t.phi, li, lj, pL);
    ldphi(e, t.phi, k, j, pR);
    const uint32_t fl = (dir == 0 ? t.xfl : t.yfl)[r.id];
    sensor_theta_vjp(pL, pR, dir, g.kappa, fl, ts, lts, lpL, lpR);
    const size_t sn = (size_t)e.sw * e.sh, sl = sidx(e, li, lj), sr = sidx(e, k, j);
    for (int q = 0; q < 4; ++q) {
      if (lpL[q] != 0.0) Add::add(ab.lphi + sl + q * sn, lpL[q]);
      if (lpR[q] != 0.0) Add::add(ab.lphi + sr + q * sn, lpR[q]);
    }
  }
}

// Sensor cell, extended range.
template <class Add>
AF_HD void adj_sensor(const AGeo& g, const StateC& u, const Tape& t, const AdjBuf& ab, const StateM& lk, int i, int j) {
  const Ext e = ext_of(g);
  const size_t id = sidx(e, i, j), n = (size_t)e.sw * e.sh;
  double lphi[4];
  bool any = false;
  for (int q = 0; q < 4; ++q) {
    lphi[q] = ab.lphi[id + q * n];
    any = any || lphi[q] != 0.0;
  }
  if (!any) return;
  double in[5][NV], l[5][NV];
  sensor_inputs(g, u, i, j, in);
  for (int q = 0; q < 5; ++q) zero8(l[q]);
  sensor_vjp(in[0], in[1], in[2], in[3], in[4], g, t.sfl[id], lphi, l[0], l[1], l[2], l[3], l[4]);
  put<Add>(lk.a, locA(g, i, j), l[0]);
  put<Add>(lk.a, locA(g, i - 1, j), l[1]);
  put<Add>(lk.a, locA(g, i + 1, j), l[2]);
  put<Add>(lk.a, locA(g, i, j - 1), l[3]);
  put<Add>(lk.a, locA(g, i, j + 1), l[4]);
}

// The FVS lines and central pair of a point.  kind 0: X(k,l) (x line, y
// pair V(k,l), V(k,l+1)); 1: Y(k,l) (y line, x pair V(k,l), V(k+1,l));
// 2: V(k,l) (both lines).
AF_HD void point_slots(const AGeo& g, const StateC& u, const Tape& t, const AdjBuf& ab, const StateM& lk, int kind,
                       int k, int l, Slot lx[5], Slot ly[5], Slot pair[2]) {
  auto X = [&](int a, int b) { return Slot{u.x, lk.x, locX(g, a, b)}; };
  auto Y = [&](int a, int b) { return Slot{u.y, lk.y, locY(g, a, b)}; };
  auto V = [&](int a, int b) { return Slot{u.v, lk.v, locV(g, a, b)}; };
  auto C = [&](int a, int b) { return Slot{t.C, ab.lC, locA(g, a, b)}; };
  if (kind == 0) {
    lx[0] = X(k - 1, l); lx[1] = C(k - 1, l); lx[2] = X(k, l); lx[3] = C(k, l); lx[4] = X(k + 1, l);
    pair[0] = V(k, l); pair[1] = V(k, l + 1);
  } else if (kind == 1) {
    ly[0] = Y(k, l - 1); ly[1] = C(k, l - 1); ly[2] = Y(k, l); ly[3] = C(k, l); ly[4] = Y(k, l + 1);
    pair[0] = V(k, l); pair[1] = V(k + 1, l);
  } else {
    lx[0] = V(k - 1, l); lx[1] = Y(k - 1, l); lx[2] = V(k, l); lx[3] = Y(k, l); lx[4] = V(k + 1, l);
    ly[0] = V(k, l - 1); ly[1] = X(k, l - 1); ly[2] = V(k, l); ly[3] = X(k, l); ly[4] = V(k, l + 1);
  }
}
// Pass 1 over an FVS line: alpha (largest spectral radius, first on ties),
// its slot, and 1/2 (D+ B_n + D- B_n).
AF_HD void line_scan(const Slot q[5], double gm, int n, double h, double& alpha, int& am, double& dB) {
  alpha = 0.0;
  am = -1;
  double b[5];
  for (int m = 0; m < 5; ++m) {
    double w[NV];
    ld(q[m].src, q[m].L, w);
    const double r = srad(w, gm, n);
    if (alpha < r) {
      alpha = r;
      am = m;
    }
    b[m] = w[4 + n];
  }
  dB = 0.5 * ((b[0] - 4.0 * b[1] + 3.0 * b[2]) / h + (-3.0 * b[2] + 4.0 * b[3] - b[4]) / h);
}
// Passes 2 and 3: the reverse of R = sum_m [sp_m F(w_m) + sd_m alpha w_m]
// and of dB, one state at a time, then of alpha at its argmax.  The middle
// slot is the point itself: its adjoint goes to self (scattered later with
// the point's other terms) instead of memory.
template <class Add>
AF_HD void line_reverse(const Slot q[5], double gm, int n, double h, double alpha, int am, const double* lR,
                        double ldB, double* self) {
  const double cp[5] = {1.0, -4.0, 3.0, 0.0, 0.0};
  const double cm[5] = {0.0, 0.0, -3.0, 4.0, -1.0};
  double lal = 0.0;
  for (int m = 0; m < 5; ++m) {
    const double sp = 0.5 * (cp[m] + cm[m]) / h, sd = 0.5 * (cp[m] - cm[m]) / h;
    double w[NV], lF[NV], lw[NV];
    ld(q[m].src, q[m].L, w);
    for (int c = 0; c < NV; ++c) {
      lF[c] = sp * lR[c];
      lw[c] = sd * alpha * lR[c];
      lal += sd * lR[c] * w[c];
    }
    flux_vjp(w, gm, n, lF, lw);
    lw[4 + n] += sp * ldB;
    if (m == 2)
      for (int c = 0; c < NV; ++c) self[c] += lw[c];
    else
      slot_put<Add>(q[m], lw);
  }
  if (am >= 0 && lal != 0.0) {
    double w[NV], lw[NV];
    ld(q[am].src, q[am].L, w);
    zero8(lw);
    srad_vjp(w, gm, n, lal, lw);
    if (am == 2)
      for (int c = 0; c < NV; ++c) self[c] += lw[c];
    else
      slot_put<Add>(q[am], lw);
  }
}

// Reverse of a point's scaling limiter and first-order LLF state where the
// limiter acted (rare).  Writes the adjoint of U^H to lH and scatters the LLF
// state's adjoints.
template <class Add>
AF_HD void point_limited_vjp(const AGeo& g, const StateC& u, const Tape& t, const StateM& lk, int kind, int k,
                                   int l, double dt, uint32_t fl, const double* lam, double* lH) {
  PointSt s;
  point_stencil(g, u, t, kind, k, l, s);
  double H[NV], Lf[NV], lLf[NV], lU[NV], lL[NV], lR[NV], lD[NV], lUp[NV];
  point_high(g, kind, s, dt, H);
  point_llf(s.U, s.L, s.R, s.D, s.Up, dt, g, Lf);
  zero8(lH);
  zero8(lLf);
  point_limit_vjp(H, Lf, g.gamma, fl, lam, lH, lLf);
  zero8(lU);
  zero8(lL);
  zero8(lR);
  zero8(lD);
  zero8(lUp);
  point_llf_vjp(s.U, s.L, s.R, s.D, s.Up, dt, g, lLf, lU, lL, lR, lD, lUp);
  if (kind == 0) {
    put<Add>(lk.x, locX(g, k, l), lU);
    put<Add>(lk.x, locX(g, k - 1, l), lL);
    put<Add>(lk.x, locX(g, k + 1, l), lR);
    put<Add>(lk.v, locV(g, k, l), lD);
    put<Add>(lk.v, locV(g, k, l + 1), lUp);
  } else if (kind == 1) {
    put<Add>(lk.y, locY(g, k, l), lU);
    put<Add>(lk.v, locV(g, k, l), lL);
    put<Add>(lk.v, locV(g, k + 1, l), lR);
    put<Add>(lk.y, locY(g, k, l - 1), lD);
    put<Add>(lk.y, locY(g, k, l + 1), lUp);
  } else {
    put<Add>(lk.v, locV(g, k, l), lU);
    put<Add>(lk.v, locV(g, k - 1, l), lL);
    put<Add>(lk.v, locV(g, k + 1, l), lR);
    put<Add>(lk.v, locV(g, k, l - 1), lD);
    put<Add>(lk.v, locV(g, k, l + 1), lUp);
  }
}

// Point of kind (0 X, 1 Y, 2 V), real.
template <class Add>
AF_HD void adj_point(const AGeo& g, const StateC& u, const Tape& t, const AdjBuf& ab, const StateC& lo, const StateM& ln,
                     const StateM& lk, int kind, int k, int l, double dt, double a, double b) {
  const size_t id = point_id(g, kind, k, l), n = point_n(g, kind);
  const double* lop = kind == 0 ? lo.x : kind == 1 ? lo.y : lo.v;
  double* lnp = kind == 0 ? ln.x : kind == 1 ? ln.y : ln.v;
  double lam[NV];
  bool any = false;
  for (int c = 0; c < NV; ++c) {
    const double x = lop[id + c * n];
    if (a != 0.0 && x != 0.0) Add::add(lnp + id + c * n, a * x);
    lam[c] = b * x;
    any = any || lam[c] != 0.0;
  }
  if (!any) return;
  const uint32_t fl = t.pfl[kind][id];
  double lH[NV];
  if (fl & (BL_T1 | BL_T2 | BL_SHIFT | BL_ZERO))
    point_limited_vjp<Add>(g, u, t, lk, kind, k, l, dt, fl, lam, lH);
  else
    for (int c = 0; c < NV; ++c) lH[c] = lam[c];  // limiter inactive: the output is U^H
  // H = U + dt (-R1 - R2 - div B Psi(U))
  Slot lx[5], ly[5], pair[2];
  point_slots(g, u, t, ab, lk, kind, k, l, lx, ly, pair);
  double ax = 0.0, ay = 0.0, d1 = 0.0, d2 = 0.0;
  int mx = -1, my = -1;
  if (kind != 1) line_scan(lx, g.gamma, 0, g.dx, ax, mx, d1);
  if (kind != 0) line_scan(ly, g.gamma, 1, g.dy, ay, my, d2);
  if (kind == 0) d2 = (pair[1].src[pair[1].L.i + 5 * pair[1].L.s] - pair[0].src[pair[0].L.i + 5 * pair[0].L.s]) / g.dy;
  if (kind == 1) d1 = (pair[1].src[pair[1].L.i + 4 * pair[1].L.s] - pair[0].src[pair[0].L.i + 4 * pair[0].L.s]) / g.dx;
  const double divB = d1 + d2;
  {
    double U[NV], P[NV], lP[NV], lU[NV];
    const Loc LU = kind == 0 ? locX(g, k, l) : kind == 1 ? locY(g, k, l) : locV(g, k, l);
    const double* src = kind == 0 ? u.x : kind == 1 ? u.y : u.v;
    ld(src, LU, U);
    psi(U, P);
    double ldiv = 0.0;
    for (int c = 0; c < NV; ++c) {
      lU[c] = lH[c];
      ldiv -= dt * lH[c] * P[c];
      lP[c] = -dt * divB * lH[c];
    }
    psi_vjp(U, lP, lU);
    double lR[NV];
    for (int c = 0; c < NV; ++c) lR[c] = -dt * lH[c];
    if (kind != 1) line_reverse<Add>(lx, g.gamma, 0, g.dx, ax, mx, lR, ldiv, lU);
    if (kind != 0) line_reverse<Add>(ly, g.gamma, 1, g.dy, ay, my, lR, ldiv, lU);
    put<Add>(kind == 0 ? lk.x : kind == 1 ? lk.y : lk.v, LU, lU);
    if (kind != 2) {
      // central pair: R = (F(pair1) - F(pair0)) / h in the transverse direction
      const int dir = kind == 0 ? 1 : 0;
      const double h = kind == 0 ? g.dy : g.dx;
      for (int q = 0; q < 2; ++q) {
        double w[NV], lF[NV], lw[NV];
        ld(pair[q].src, pair[q].L, w);
        const double sgnq = q ? 1.0 : -1.0;
        for (int c = 0; c < NV; ++c) lF[c] = sgnq * lR[c] / h;
        zero8(lw);
        flux_vjp(w, g.gamma, dir, lF, lw);
        lw[4 + dir] += sgnq * ldiv / h;
        slot_put<Add>(pair[q], lw);
      }
    }
  }
}

// Centre of real cell (i, j), first pass: the adjoint of the limited
// centre back to A (added here; the last kernel of the sweep, so this
// thread is the only writer of A(i,j)'s adjoint) and to the raw
// reconstruction C~, whose adjoint replaces lC(i,j) in place for the gather.
template <class Add>
AF_HD void adj_centre(const AGeo& g, const StateC& u, const Tape& t, const AdjBuf& ab, const StateM& lk, int i, int j) {
  const size_t id = (size_t)j * g.nx + i, n = (size_t)g.nx * g.ny;
  double lC[NV];
  ld8(ab.lC, id, n, lC);
  bool any = false;
  for (int c = 0; c < NV; ++c) any = any || lC[c] != 0.0;
  if (!any) return;
  double lA[NV], lUc[NV];
  zero8(lA);
  zero8(lUc);
  if (t.cfl[id] & (BL_T1 | BL_T2 | BL_SHIFT | BL_ZERO)) {
    double in[9][NV], Uc[NV];
    centre_inputs(g, u, i, j, in);
    const double* p[9] = {in[0], in[1], in[2], in[3], in[4], in[5], in[6], in[7], in[8]};
    centre_raw(p, Uc);
    centre_limit_vjp(in[0], Uc, g.gamma, t.cfl[id], lC, lA, lUc);
  } else {
    for (int c = 0; c < NV; ++c) lUc[c] = lC[c];  // C = C~
  }
  for (int c = 0; c < NV; ++c) lA[c] += 36.0 / 16.0 * lUc[c];
  st8(ab.lC, id, n, lUc);
  double* pa = lk.a + id;
  for (int c = 0; c < NV; ++c) pa[c * n] += lA[c];
}

// Second pass, one thread per point of kind (0 X, 1 Y, 2 V): gathers the
// reconstruction adjoints of the cells whose centre contains the point
// (-4/16 for a face, -1/16 for a vertex).  A real cell's centre reads its
// points at node indices 0..n (never mirrored), so a point's cells are its
// real neighbours: i-1 and i along x for a node index i (wrapped when
// periodic), the cell itself along a cell index.
AF_HD void adj_centre_gather(const AGeo& g, const AdjBuf& ab, const StateM& lk, int kind, int k, int l) {
  const size_t n = (size_t)g.nx * g.ny;
  int ci[2], cj[2], nci = 0, ncj = 0;
  auto nodes = [](int k_, int nc, int bc, int* out, int& cnt) {
    cnt = 0;
    if (bc == 0) {
      out[cnt++] = k_ % nc;
      out[cnt++] = (k_ - 1 + nc) % nc;
    } else {
      if (k_ < nc) out[cnt++] = k_;
      if (k_ - 1 >= 0) out[cnt++] = k_ - 1;
    }
  };
  if (kind == 0 || kind == 2)
    nodes(k, g.nx, g.bcx, ci, nci);
  else {
    ci[0] = k;
    nci = 1;
  }
  if (kind == 1 || kind == 2)
    nodes(l, g.ny, g.bcy, cj, ncj);
  else {
    cj[0] = l;
    ncj = 1;
  }
  const double w = kind == 2 ? -1.0 / 16.0 : -4.0 / 16.0;
  double sum[NV];
  zero8(sum);
  for (int a = 0; a < nci; ++a)
    for (int b = 0; b < ncj; ++b) {
      const size_t id = (size_t)cj[b] * g.nx + ci[a];
      for (int c = 0; c < NV; ++c) sum[c] += ab.lC[id + c * n];
    }
  const size_t pid = point_id(g, kind, k, l), pn = point_n(g, kind);
  double* p = kind == 0 ? lk.x : kind == 1 ? lk.y : lk.v;
  for (int c = 0; c < NV; ++c) p[pid + c * pn] += w * sum[c];
}

}  // namespace afadj
