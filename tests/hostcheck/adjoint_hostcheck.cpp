// Host build of the adjoint's entity functions (the code the HIP kernels of
// af_adjoint.hip run, one thread per entity), driven by plain loops in the
// kernels' launch order and with plain adds for the scatters.  Test
// infrastructure: it lets the reverse sweep be checked against the tangent
// oracle on a machine without a GPU.  Never part of the library.
#include <cmath>
#include <cstring>
#include <vector>
using std::exp;
using std::fabs;
using std::sqrt;
#define AF_HD inline
#include "af_adjoint_stage.h"

using namespace afadj;

namespace {
struct HostAdd {
  static void add(double* p, double v) { *p += v; }
};
const double RK_A[3] = {0.0, 0.75, 1.0 / 3.0};
const double RK_B[3] = {1.0, 0.25, 2.0 / 3.0};
}  // namespace

extern "C" {

typedef struct {
  int nx, ny, bc_x, bc_y;
  double dx, dy, gamma, kappa;
} hc_params;

static AGeo geo(const hc_params* p) {
  AGeo g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.bcx = p->bc_x;
  g.bcy = p->bc_y;
  g.nxp = p->nx + (p->bc_x ? 1 : 0);
  g.nyp = p->ny + (p->bc_y ? 1 : 0);
  g.dx = p->dx;
  g.dy = p->dy;
  g.gamma = p->gamma;
  g.kappa = p->kappa;
  return g;
}

size_t hc_tape_bytes(const hc_params* p) { return tape_layout(geo(p), nullptr, nullptr); }
size_t hc_adjbuf_bytes(const hc_params* p) { return adjbuf_layout(geo(p), nullptr, nullptr); }

void hc_record(const hc_params* p, int k, const double* const* un, const double* const* uk, double* const* out,
               double dt, void* tape) {
  const AGeo g = geo(p);
  const Ext e = ext_of(g);
  Tape t;
  tape_layout(g, (char*)tape, &t);
  const StateC u{uk[0], uk[1], uk[2], uk[3]};
  const StateC n = k == 0 ? u : StateC{un[0], un[1], un[2], un[3]};
  const double a = RK_A[k], b = RK_B[k];
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) rec_centre(g, u, t, i, j);
  for (int j = -2; j < g.ny + 2; ++j)
    for (int i = -2; i < g.nx + 2; ++i) rec_sensor(g, u, t, i, j);
  for (int j = -1; j < g.ny + 1; ++j)
    for (int kk = -1; kk < g.nx + 2; ++kk) rec_iface(g, u, t, 0, kk, j);
  for (int l = -1; l < g.ny + 2; ++l)
    for (int i = -1; i < g.nx + 1; ++i) rec_iface(g, u, t, 1, i, l);
  for (int j = -1; j < g.ny + 1; ++j)
    for (int i = -1; i < g.nx + 1; ++i) rec_limiter(g, u, t, i, j, dt);
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) rec_update(g, n, u, t, out[0], i, j, dt, a, b);
  for (int l = 0; l < g.ny; ++l)
    for (int kk = 0; kk < g.nxp; ++kk) rec_point(g, n, u, t, out[1], 0, kk, l, dt, a, b);
  for (int l = 0; l < g.nyp; ++l)
    for (int i = 0; i < g.nx; ++i) rec_point(g, n, u, t, out[2], 1, i, l, dt, a, b);
  for (int l = 0; l < g.nyp; ++l)
    for (int kk = 0; kk < g.nxp; ++kk) rec_point(g, n, u, t, out[3], 2, kk, l, dt, a, b);
}

void hc_adjoint(const hc_params* p, int k, const double* const* uk, const void* tape, double dt,
                const double* const* lam_out, double* const* lam_n, double* const* lam_k, void* adjbuf) {
  const AGeo g = geo(p);
  Tape t;
  tape_layout(g, (char*)tape, &t);
  AdjBuf ab;
  const size_t nb = adjbuf_layout(g, (char*)adjbuf, &ab);
  std::memset(adjbuf, 0, nb);
  const StateC u{uk[0], uk[1], uk[2], uk[3]};
  const StateC lo{lam_out[0], lam_out[1], lam_out[2], lam_out[3]};
  const StateM lk{lam_k[0], lam_k[1], lam_k[2], lam_k[3]};
  const StateM ln = k == 0 ? lk : StateM{lam_n[0], lam_n[1], lam_n[2], lam_n[3]};
  const double a = RK_A[k], b = RK_B[k];
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) adj_update<HostAdd>(g, t, ab, lo, ln, lk, i, j, dt, a, b);
  for (int j = -1; j < g.ny + 1; ++j)
    for (int i = -1; i < g.nx + 1; ++i) adj_limiter<HostAdd>(g, u, t, ab, lk, i, j, dt);
  for (int j = -1; j < g.ny + 1; ++j)
    for (int kk = -1; kk < g.nx + 2; ++kk) adj_iface<HostAdd>(g, u, t, ab, lk, 0, kk, j);
  for (int l = -1; l < g.ny + 2; ++l)
    for (int i = -1; i < g.nx + 1; ++i) adj_iface<HostAdd>(g, u, t, ab, lk, 1, i, l);
  for (int j = -2; j < g.ny + 2; ++j)
    for (int i = -2; i < g.nx + 2; ++i) adj_sensor<HostAdd>(g, u, t, ab, lk, i, j);
  for (int l = 0; l < g.ny; ++l)
    for (int kk = 0; kk < g.nxp; ++kk) adj_point<HostAdd>(g, u, t, ab, lo, ln, lk, 0, kk, l, dt, a, b);
  for (int l = 0; l < g.nyp; ++l)
    for (int i = 0; i < g.nx; ++i) adj_point<HostAdd>(g, u, t, ab, lo, ln, lk, 1, i, l, dt, a, b);
  for (int l = 0; l < g.nyp; ++l)
    for (int kk = 0; kk < g.nxp; ++kk) adj_point<HostAdd>(g, u, t, ab, lo, ln, lk, 2, kk, l, dt, a, b);
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) adj_centre<HostAdd>(g, u, t, ab, lk, i, j);
  for (int l = 0; l < g.ny; ++l)
    for (int kk = 0; kk < g.nxp; ++kk) adj_centre_gather(g, ab, lk, 0, kk, l);
  for (int l = 0; l < g.nyp; ++l)
    for (int i = 0; i < g.nx; ++i) adj_centre_gather(g, ab, lk, 1, i, l);
  for (int l = 0; l < g.nyp; ++l)
    for (int kk = 0; kk < g.nxp; ++kk) adj_centre_gather(g, ab, lk, 2, kk, l);
}

}  // extern "C"

// ---- the limiters alone (function-level checks)
extern "C" {

void hc_point_limit(const double* UH, const double* UL, double g, double* out, uint32_t* fl) {
  uint32_t f = 0;
  point_limit(UH, UL, g, out, f);
  *fl = f;
}
void hc_point_limit_vjp(const double* UH, const double* UL, double g, uint32_t fl, const double* lout, double* lUH,
                        double* lUL) {
  for (int c = 0; c < NV; ++c) lUH[c] = lUL[c] = 0.0;
  point_limit_vjp(UH, UL, g, fl, lout, lUH, lUL);
}
static CellIn cell_in(const double* x) {
  CellIn w;
  for (int c = 0; c < NV; ++c) {
    w.A[c] = x[c];
    for (int I = 0; I < 4; ++I) {
      w.Fs[I][c] = x[8 + 8 * I + c];
      w.Fl[I][c] = x[40 + 8 * I + c];
    }
    w.Ss[c] = x[72 + c];
    w.Sllf[c] = x[80 + c];
  }
  return w;
}
// x[88] = A, FsL..FsU, FlL..FlU, S_s, S_llf
void hc_cell_limiter(const double* x, double dt, double dx, double dy, double g, double* th, double* Lam, double* rk,
                     uint64_t* fl) {
  AGeo geo{};
  geo.dx = dx;
  geo.dy = dy;
  geo.gamma = g;
  uint64_t f = 0;
  cell_limiter(cell_in(x), dt, geo, *th, Lam, rk, f);
  *fl = f;
}
void hc_cell_limiter_vjp(const double* x, double dt, double dx, double dy, double g, const double* rk, uint64_t fl,
                         double lth, const double* lLam, double* lx) {
  AGeo geo{};
  geo.dx = dx;
  geo.dy = dy;
  geo.gamma = g;
  CellAdj o;
  std::memset(&o, 0, sizeof(o));
  cell_limiter_vjp(cell_in(x), dt, geo, rk, fl, lth, lLam, o);
  for (int c = 0; c < NV; ++c) {
    lx[c] = o.A[c];
    for (int I = 0; I < 4; ++I) {
      lx[8 + 8 * I + c] = o.Fs[I][c];
      lx[40 + 8 * I + c] = o.Fl[I][c];
    }
    lx[72 + c] = o.Ss[c];
    lx[80 + c] = o.Sllf[c];
  }
}

}  // extern "C"
