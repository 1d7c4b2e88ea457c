// af_stage.hip -- kernels of one SSP-RK3 stage of the PP Active Flux scheme
// for 2D ideal MHD with the Godunov-Powell source (gfx950), and the C ABI
// declared in include/af_mhd.h.
//
// A stage (forward Euler on U^(k), then out = a_k U^n + b_k FE) is two
// launches that read only U^(k) (and U^n for the combination):
//   k_points  point values (Section 2.3): centre values (Section 2.1,
//             remark rmk:cell_center), LLF flux-vector splitting with the
//             central div B source, first-order LLF safe state and scaling
//             limiter (Section 3.3), SSP combination; and each cell's
//             nine-point Powell source (Section 2.2) from the tile's points
//   k_cells   cell averages (Sections 2.2, 3.1-3.4): Simpson and LLF fluxes,
//             shock sensor, LLF Powell source, parametrized flux limiter,
//             limited update in flux form, SSP combination
// Both are LDS-tiled: a tile's states and the costly per-point quantities
// are computed once and shared through LDS, cheap ones (fluxes) rebuilt
// where they are used; only the nine-point sources pass through HBM.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "af_device.h"
#include "af_tiles.h"
#include "af_mhd.h"

using namespace afm;

namespace {

struct WS {                 // workspace pointers
  double* partial;          // reduction partials
  Counters* cnt;
  double* scratch[2][4];    // two RK scratch states
  double* src;              // nine-point sources of the stage input's cells, [8][ny][nx]
  double* wpart;            // per-workgroup wave-speed maxima of a step's last stage
  int nwpart;               // point-kernel grid + cell-kernel grid
};

inline int points_tiles_x(const Geo& g) { return (g.nxp + PB - 3) / (PB - 2); }
inline int points_tiles_y(const Geo& g) { return (g.nyp + PB - 3) / (PB - 2); }
inline int cells_tiles_x(const Geo& g) { return (g.nx + CBX0 - 4) / (CBX0 - 3); }
inline int cells_tiles_y(const Geo& g) { return (g.ny + CBY0 - 4) / (CBY0 - 3); }

// wpart: null, or one slot per workgroup for the maximum of rho_1/dx +
// rho_2/dy over the values it stores (a step's last stage; padding
// workgroups store 0).
// WDT: a step's last stage, whose epilogue also writes the wave-speed maxima.
template <class R, bool WDT>
__global__ __launch_bounds__(PNT, 2) void k_points(Geo g, CState u, CState un, MState out,
                                                   double* __restrict__ src, const double* dtp, double ca,
                                                   double cb, Counters* cn, int ntx, int nty,
                                                   double* __restrict__ wpart) {
  __shared__ R s[point_fields<R>()][PB][PB];
  int bx, by;
  if (!xcd_tile(ntx, nty, bx, by)) {
    if (WDT && threadIdx.x == 0 && threadIdx.y == 0) wpart[blockIdx.x] = 0.0;
    return;
  }
  points_tile<R>(g, u, un, out, src, *dtp, ca, cb, cn, bx, by, s, WDT ? wpart + blockIdx.x : nullptr);
}

template <class R, bool WDT>
__global__ __launch_bounds__(CBX0 * CBY0) void k_cells(Geo g, CState u, const double* __restrict__ src,
                                                       const double* __restrict__ un, double* __restrict__ out,
                                                       const double* dtp, double ca, double cb, Counters* cn,
                                                       int ntx, int nty, double* __restrict__ wpart) {
  __shared__ CellsLDS<R, CBX0, CBY0> L;
  int bx, by;
  if (!xcd_tile(ntx, nty, bx, by)) {
    if (WDT && threadIdx.x == 0 && threadIdx.y == 0) wpart[blockIdx.x] = 0.0;
    return;
  }
  cells_tile<R, CBX0, CBY0>(g, u, src, un, out, *dtp, ca, cb, cn, bx, by, L, WDT ? wpart + blockIdx.x : nullptr);
}

__global__ __launch_bounds__(BLK) void k_dt_partial(Geo g, CState u, double* partial) {
  const long n = g.sc + g.sx + g.sy + g.sv;
  double m = 0.0;
  // four DoFs per trip: their loads are in flight together
#pragma unroll 4
  for (long t = (long)blockIdx.x * BLK + threadIdx.x; t < n; t += (long)gridDim.x * BLK) {
    const double* base;
    long plane, off;
    dof_ptr(g, u, t, base, plane, off);
    double U[NV];
    load8(base, plane, off, U);
    m = fmax(m, dt_speed(U, g));
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

// dt from the per-workgroup maxima a step's last stage left (one workgroup
// of 1024 threads).
constexpr int DT_PARTS_BLK = 1024;
__global__ __launch_bounds__(DT_PARTS_BLK) void k_dt_from_parts(const double* wpart, int n, double cfl,
                                                                double t_rem, double* dt) {
  __shared__ double sh[DT_PARTS_BLK / 64];
  double m = 0.0;
#pragma unroll 4
  for (int t = threadIdx.x; t < n; t += DT_PARTS_BLK) m = fmax(m, wpart[t]);
  block_max_store(m, (int)threadIdx.x, DT_PARTS_BLK, sh, sh);
  if (threadIdx.x == 0) {
    double d = cfl / sh[0];
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

// The two discrete divergences recorded for the Orszag-Tang example
// (Section 4), per cell, summed in a fixed order (deterministic):
//   div1: sum over the nine points of |div B| w_a w_b dx dy, with the
//         derivatives and weights of the source of eq. (semi_av_src) and
//         the limited centre value;
//   div2: one sixth of |Simpson edge integral of B . n| dx dy, as printed.
__global__ __launch_bounds__(BLK) void k_divb_partial(Geo g, CState u, double* partial) {
  double s1 = 0.0, s2 = 0.0;
  for (long t = (long)blockIdx.x * BLK + threadIdx.x; t < g.sc; t += (long)gridDim.x * BLK) {
    const int i = (int)(t % g.nx), j = (int)(t / g.nx);
    double A[NV], Uc[NV], f[NV], w[NV], q[NV], C[NV];
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
    double B1[3][3], B2[3][3];  // [a][b]: a along x, b along y
    auto put = [&](int a, int b, const double* U) {
      B1[a][b] = U[4];
      B2[a][b] = U[5];
    };
    ldV(g, u.v, i, j, w);         put(0, 0, w);
    ldY(g, u.y, i, j, w);         put(1, 0, w);
    ldV(g, u.v, i + 1, j, w);     put(2, 0, w);
    ldX(g, u.x, i, j, w);         put(0, 1, w);
    put(1, 1, C);
    ldX(g, u.x, i + 1, j, w);     put(2, 1, w);
    ldV(g, u.v, i, j + 1, w);     put(0, 2, w);
    ldY(g, u.y, i, j + 1, w);     put(1, 2, w);
    ldV(g, u.v, i + 1, j + 1, w); put(2, 2, w);
    const double wq[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    double c1 = 0.0;
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
        c1 += fabs(dx1 * g.rdx + dy2 * g.rdy) * wq[a] * wq[b];
      }
    const double right = B1[2][0] + 4.0 * B1[2][1] + B1[2][2], left = B1[0][0] + 4.0 * B1[0][1] + B1[0][2];
    const double top = B2[0][2] + 4.0 * B2[1][2] + B2[2][2], bottom = B2[0][0] + 4.0 * B2[1][0] + B2[2][0];
    s1 += c1 * (g.dx * g.dy);
    s2 += fabs((right - left) + (top - bottom)) * (1.0 / 6.0) * (g.dx * g.dy);
  }
  __shared__ double sh[2][BLK];
  sh[0][threadIdx.x] = s1;
  sh[1][threadIdx.x] = s2;
  __syncthreads();
  for (int st = BLK / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) partial[threadIdx.x * gridDim.x + blockIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_divb_final(const double* partial, int nparts, double* out) {
  if (threadIdx.x < 2) {
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += partial[threadIdx.x * nparts + b];
    out[threadIdx.x] = s;
  }
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
  bool f32 = false;        // AF_FLAG_FP32_BULK
  bool fused_dt = false;   // AF_FLAG_FUSED_DT
  // the state whose wave-speed maxima ws.wpart holds (left by the last
  // stage of af_mhd_step on it), or null
  const double* wpart_for[4] = {nullptr, nullptr, nullptr, nullptr};
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
  return (p->flags & ~(uint32_t)(AF_FLAG_KERNEL_TIMING | AF_FLAG_FP32_BULK | AF_FLAG_FUSED_DT)) == 0;
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
  w.src = take(8 * sizes[0]);
  w.nwpart = xcd_grid(points_tiles_x(g), points_tiles_y(g)) + xcd_grid(cells_tiles_x(g), cells_tiles_y(g));
  w.wpart = take((size_t)w.nwpart);
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

// wpart: null, or the slots for the workgroups' wave-speed maxima of the
// stage's outputs (point-kernel grid, then cell-kernel grid).
int run_stage(af_mhd_ctx* c, int k, const af_mhd_state* un, const af_mhd_state* uk, af_mhd_state* out,
              const double* dt_dev, double* wpart = nullptr) {
  static const double A[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double B[3] = {1.0, 0.25, 2.0 / 3.0};
  const Geo& g = c->g;
  hipStream_t s = c->stream;
  const CState u = cstate(uk);
  const CState n = cstate(k == 0 ? uk : un);  // not read when a_k = 0
  const MState o{out->cell, out->xface, out->yface, out->vert};
  const int ptx = points_tiles_x(g), pty = points_tiles_y(g);
  double* const wcells = wpart ? wpart + xcd_grid(ptx, pty) : nullptr;
  hipEvent_t end;
  hipError_t e = timer_begin(c, KernelTimer::POINTS, &end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  {
    if (c->f32)
      (wpart ? k_points<float, true> : k_points<float, false>)<<<xcd_grid(ptx, pty), dim3(PB, PB), 0, s>>>(
          g, u, n, o, c->ws.src, dt_dev, A[k], B[k], c->ws.cnt, ptx, pty, wpart);
    else
      (wpart ? k_points<double, true> : k_points<double, false>)<<<xcd_grid(ptx, pty), dim3(PB, PB), 0, s>>>(
          g, u, n, o, c->ws.src, dt_dev, A[k], B[k], c->ws.cnt, ptx, pty, wpart);
  }
  e = timer_end(c, end);
  if (e == hipSuccess) e = timer_begin(c, KernelTimer::CELLS, &end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  const int ctx_ = cells_tiles_x(g), cty = cells_tiles_y(g);
  if (c->f32)
    (wcells ? k_cells<float, true> : k_cells<float, false>)<<<xcd_grid(ctx_, cty), dim3(CBX0, CBY0), 0, s>>>(
        g, u, c->ws.src, n.a, o.a, dt_dev, A[k], B[k], c->ws.cnt, ctx_, cty, wcells);
  else
    (wcells ? k_cells<double, true> : k_cells<double, false>)<<<xcd_grid(ctx_, cty), dim3(CBX0, CBY0), 0, s>>>(
        g, u, c->ws.src, n.a, o.a, dt_dev, A[k], B[k], c->ws.cnt, ctx_, cty, wcells);
  e = timer_end(c, end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  return check_hip(c, "stage launch");
}

bool same_state(const double* const a[4], const af_mhd_state* u) {
  return a[0] == u->cell && a[1] == u->xface && a[2] == u->yface && a[3] == u->vert;
}

// dt from the wave-speed maxima the last stage of the previous step left.
int run_dt_from_parts(af_mhd_ctx* c, double t_rem, double* dt_dev) {
  hipEvent_t end;
  hipError_t e = timer_begin(c, KernelTimer::DT, &end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  k_dt_from_parts<<<1, DT_PARTS_BLK, 0, c->stream>>>(c->ws.wpart, c->ws.nwpart, c->g.cfl, t_rem, dt_dev);
  e = timer_end(c, end);
  if (e != hipSuccess) return fail(c, AF_EHIP, hipGetErrorString(e));
  return check_hip(c, "dt launch");
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
  c->fused_dt = (p->flags & AF_FLAG_FUSED_DT) != 0;
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
  for (auto& p : c->wpart_for) p = nullptr;  // the stage may write the state the maxima belong to
  return run_stage(c, k, un, uk, out, dt_dev);
}

int af_mhd_step(af_mhd_ctx* c, af_mhd_state* u, double t_remaining, double* dt_dev) {
  if (!c) return AF_EINVAL;
  if (!valid_state(u) || !aligned8(dt_dev) || !(t_remaining > 0.0)) return fail(c, AF_EINVAL, "af_mhd_step: bad argument");
  af_mhd_state s1{c->ws.scratch[0][0], c->ws.scratch[0][1], c->ws.scratch[0][2], c->ws.scratch[0][3]};
  af_mhd_state s2{c->ws.scratch[1][0], c->ws.scratch[1][1], c->ws.scratch[1][2], c->ws.scratch[1][3]};
  const bool reuse = c->fused_dt && same_state(c->wpart_for, u);
  for (auto& p : c->wpart_for) p = nullptr;
  int rc = reuse ? run_dt_from_parts(c, t_remaining, dt_dev) : run_dt(c, u, t_remaining, dt_dev);
  if (rc == AF_OK) rc = run_stage(c, 0, u, u, &s1, dt_dev);
  if (rc == AF_OK) rc = run_stage(c, 1, u, &s1, &s2, dt_dev);
  if (rc == AF_OK) rc = run_stage(c, 2, u, &s2, u, dt_dev, c->fused_dt ? c->ws.wpart : nullptr);
  if (rc == AF_OK && c->fused_dt) {
    c->wpart_for[0] = u->cell;
    c->wpart_for[1] = u->xface;
    c->wpart_for[2] = u->yface;
    c->wpart_for[3] = u->vert;
  }
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

int af_mhd_divb(af_mhd_ctx* c, const af_mhd_state* u, double* divb_dev) {
  if (!c) return AF_EINVAL;
  if (!valid_state(u) || !aligned8(divb_dev)) return fail(c, AF_EINVAL, "af_mhd_divb: bad argument");
  const Geo& g = c->g;
  const int nb = (int)std::min<long>(RED_BLOCKS, std::max<long>(1, nblocks(g.sc)));
  k_divb_partial<<<nb, BLK, 0, c->stream>>>(g, cstate(u), c->ws.partial);
  k_divb_final<<<1, 64, 0, c->stream>>>(c->ws.partial, nb, divb_dev);
  return check_hip(c, "af_mhd_divb launch");
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

// ------------------------------------------------ the step without allocation
// af_mhd_step_noalloc keeps the step's scratch (reduction partials, counters,
// two RK scratch states, nine-point sources, wave-speed maxima: the workspace
// layout above) in one file-scope device array per GPU instead of a
// caller-owned workspace.  In host code the array's name is only a stand-in:
// its device address, one per GPU, comes from hipGetSymbolAddress on the
// first call on that device (with the device current) and is kept here.
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)48 << 20;  // 48 MiB per GPU
__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
char* scratch_dev[NOALLOC_MAX_DEVICES];  // each device's copy of the array; null until looked up
std::mutex scratch_mu;

}  // namespace

extern "C" int af_mhd_step_noalloc(const af_mhd_params* p, af_mhd_state* u, double t_remaining, double* dt_dev,
                                   void* hip_stream) {
  init_err.clear();
  if (!valid_params(p) || (p->flags & (AF_FLAG_KERNEL_TIMING | AF_FLAG_FUSED_DT)))
    return init_fail(AF_EINVAL, "af_mhd_step_noalloc: invalid parameters");
  if (!valid_state(u) || !aligned8(dt_dev) || !(t_remaining > 0.0))
    return init_fail(AF_EINVAL, "af_mhd_step_noalloc: bad argument");
  af_mhd_ctx c;
  make_geo(p, c.g);
  if (layout(c.g, nullptr, nullptr) > NOALLOC_SCRATCH_BYTES)
    return init_fail(AF_EINVAL, "af_mhd_step_noalloc: grid too large for the 48 MiB static scratch "
                                "(about 256 x 256 cells at most)");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return init_fail(AF_EHIP, std::string("af_mhd_step_noalloc: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return init_fail(AF_EINVAL, "af_mhd_step_noalloc: device index too large");
  char* base;
  {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return init_fail(AF_EHIP, std::string("af_mhd_step_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
      scratch_dev[dev] = static_cast<char*>(ptr);
    }
    base = scratch_dev[dev];
  }
  layout(c.g, base, &c.ws);
  c.stream = static_cast<hipStream_t>(hip_stream);
  c.f32 = (p->flags & AF_FLAG_FP32_BULK) != 0;
  (void)hipGetLastError();
  // the counters start at zero on every call (a fill kernel, no memset)
  k_zero_counters<<<1, 64, 0, c.stream>>>(c.ws.cnt);
  int rc = check_hip(&c, "af_mhd_step_noalloc");
  af_mhd_state s1{c.ws.scratch[0][0], c.ws.scratch[0][1], c.ws.scratch[0][2], c.ws.scratch[0][3]};
  af_mhd_state s2{c.ws.scratch[1][0], c.ws.scratch[1][1], c.ws.scratch[1][2], c.ws.scratch[1][3]};
  if (rc == AF_OK) rc = run_dt(&c, u, t_remaining, dt_dev);
  if (rc == AF_OK) rc = run_stage(&c, 0, u, u, &s1, dt_dev);
  if (rc == AF_OK) rc = run_stage(&c, 1, u, &s1, &s2, dt_dev);
  if (rc == AF_OK) rc = run_stage(&c, 2, u, &s2, u, dt_dev);
  if (rc != AF_OK) init_fail(rc, c.err);
  return rc;
}
