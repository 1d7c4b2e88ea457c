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
}

}  // extern "C"
