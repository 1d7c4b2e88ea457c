// af_batch.hip -- batched ensembles: many independent grids, of any sizes,
// advanced together.  Per SSP-RK3 step: one launch for the dt of every
// instance (plus its per-instance finish), then per stage either
//   - one launch (AF_BATCH_FUSED) over the point tiles of all instances
//     (two 16 x 16 tiles per 512-thread workgroup) and their cell tiles,
//     which compute their own nine-point sources so that nothing in the
//     launch waits on anything, or
//   - one launch of the point update over the (instance, tile) work items
//     of all instances and one launch of the cell update over theirs, with
//     persistent workgroups (AF_BATCH_PERSISTENT) or one item per workgroup
//     (AF_BATCH_FLAT).
// Cell tiles are 32 x 16 or 16 x 32 (the shape tuned for most of the
// batch's cells).  The mode is the fastest on the batch's stage 0, measured
// at init, unless the caller sets one.  The step is captured once into a
// hipGraph and replayed.  The cell-tile shape of each grid size is chosen
// by measurement (autotune) and kept in a text table that later runs reuse.
//
// Each instance computes exactly what a single-grid context computes on it
// (same arithmetic per DoF; max reductions are order-independent), so its
// results are bitwise equal to its single-grid run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "af_device.h"
#include "af_mhd.h"
#include "af_tiles.h"

using namespace afm;

namespace {

// Cell-tile shapes the autotuner chooses from (threads = cells + ring).
constexpr int NSHAPE = 2;
const int SHAPE_X[NSHAPE] = {32, 16};
const int SHAPE_Y[NSHAPE] = {16, 32};

struct BInst {          // one instance in one launch of one stage
  Geo g;
  CState u;             // stage input U^(k)
  CState un;            // U^n (read when a_k != 0)
  MState out;           // stage output
  double* src;          // nine-point sources of U^(k)'s cells
  const double* dt;     // the instance's time step (device)
  int first;            // first work item of the instance in this launch
  int ntx;              // tiles per row in this launch
};

struct BDt {            // one instance in the dt launch
  Geo g;
  CState u;
  int first;            // first partial of the instance
  int nparts;           // partials of the instance
  double cfl;
};

constexpr int DT_CHUNK = BLK * 4;   // DoFs per dt work item
constexpr int TUNE_COPIES = 64;     // most copies of one instance's items in a tuning launch
constexpr int TUNE_ITEMS = 4096;    // tuning launches carry about this many items

// Work item -> instance: binary search over the first-item offsets.
template <class T>
__device__ __forceinline__ int find_inst(const T* __restrict__ I, int n, int it) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (I[mid].first <= it) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Item order.  Workgroup b runs on XCD b % 8, and XCD x takes the
// contiguous item range [x per, (x+1) per): the tiles an XCD works on
// together are neighbours and share halos in its L2.  Persistent launches
// (gridDim.x a multiple of 8, about one resident wave of workgroups) step
// through the range by gridDim.x / 8; flat launches (8 per workgroups) take
// one item each.  Returns false when the workgroup has no item.
template <bool PERSIST>
__device__ __forceinline__ bool item_range(int items, int& first, int& end, int& step) {
  const int b = (int)blockIdx.x, x = b % NXCD, r = b / NXCD, per = (items + NXCD - 1) / NXCD;
  first = x * per + r;
  if constexpr (PERSIST) {
    end = min(items, (x + 1) * per);
    step = (int)gridDim.x / NXCD;
  } else {
    end = first + 1;
    step = 1;
  }
  return first < items && first < (x + 1) * per;
}
inline int flat_grid(int items) { return NXCD * ((items + NXCD - 1) / NXCD); }

template <class R, bool PERSIST>
__global__ __launch_bounds__(PNT, 2) void kb_points(const BInst* __restrict__ I, int n,
                                                                          int items, double ca, double cb,
                                                                          Counters* cn) {
  __shared__ R s[point_fields<R>()][PB][PB];
  int it, end, step;
  if (!item_range<PERSIST>(items, it, end, step)) return;
  for (; it < end; it += step) {
    const int m = find_inst(I, n, it);
    const Geo g = I[m].g;
    const int t = it - I[m].first, ntx = I[m].ntx;
    __syncthreads();  // the previous item's LDS reads are done
    points_tile<R>(g, I[m].u, I[m].un, I[m].out, I[m].src, *I[m].dt, ca, cb, cn, t % ntx, t / ntx, s);
  }
}

// The cell update of every instance in one launch, on CBX x CBY tiles
// (the batch's tuned shape).
template <class R, int CBX, int CBY, bool PERSIST>
__global__ __launch_bounds__(CBX * CBY) void kb_cells(const BInst* __restrict__ I, int n, int items, double ca,
                                                      double cb, Counters* cn) {
  __shared__ CellsLDS<R, CBX, CBY> L;
  int it, end, step;
  if (!item_range<PERSIST>(items, it, end, step)) return;
  for (; it < end; it += step) {
    const int m = find_inst(I, n, it);
    const Geo g = I[m].g;
    const int t = it - I[m].first, ntx = I[m].ntx;
    __syncthreads();
    cells_tile<R, CBX, CBY>(g, I[m].u, I[m].src, I[m].un.a, I[m].out.a, *I[m].dt, ca, cb, cn, t % ntx,
                            t / ntx, L);
  }
}

// One stage of every instance in one launch (AF_BATCH_FUSED): workgroups
// [0, npairs) take pairs of point tiles (tiles 2q and 2q+1 of the batch's
// point list, run side by side by the two halves of the 512-thread
// workgroup; an odd last tile leaves the second half recomputing the first
// half's tile without storing anything), workgroups [npairs, npairs +
// citems) cell tiles.  The two kinds share nothing within the stage: the
// cell tiles compute their cells' nine-point sources themselves, from the
// stage input, instead of reading the point tiles' (which would make a cell
// tile wait for its neighbours' point tiles), so the launch has no
// inter-workgroup synchronisation at all.
constexpr int FUSED_THREADS = 512;

template <class R, int CBX, int CBY>
__global__ __launch_bounds__(FUSED_THREADS) void kb_stage(const BInst* __restrict__ P, const BInst* __restrict__ C,
                                                          int n, int pitems, int citems, double ca, double cb,
                                                          Counters* cn) {
  static_assert(CBX * CBY == FUSED_THREADS, "one cell tile per workgroup");
  union Lds {
    R pts[2][point_fields<R>()][PB][PB];
    CellsLDS<R, CBX, CBY> cells;
  };
  __shared__ Lds L;
  const int tid = (int)(threadIdx.y * blockDim.x + threadIdx.x);
  const int npairs = (pitems + 1) / 2;
  const int it = (int)blockIdx.x;
  if (it < npairs) {
    const int half = tid / PNT, ltid = tid % PNT;
    const int t0 = 2 * it + half;
    const bool live = t0 < pitems;
    const int t = live ? t0 : 2 * it;
    const int m = find_inst(P, n, t);
    const Geo g = P[m].g;
    const int tt = t - P[m].first, ntx = P[m].ntx;
    points_tile_lean<R>(g, P[m].u, P[m].un, P[m].out, nullptr, *P[m].dt, ca, cb, cn, tt % ntx, tt / ntx,
                        L.pts[half], nullptr, ltid % PB, ltid / PB, live);
    return;
  }
  const int c = it - npairs;
  if (c >= citems) return;
  const int m = find_inst(C, n, c);
  const int t = c - C[m].first, ntx = C[m].ntx;
  cells_tile<R, CBX, CBY>(C[m].g, C[m].u, nullptr, C[m].un.a, C[m].out.a, *C[m].dt, ca, cb, cn, t % ntx, t / ntx,
                          L.cells);
}

// dt: partial maxima of rho_1/dx + rho_2/dy over DT_CHUNK DoFs per item,
// then one workgroup per instance.
__global__ __launch_bounds__(BLK) void kb_dt_partial(const BDt* __restrict__ D, int n, int items,
                                                     double* partial) {
  int it, end, step;
  if (!item_range<true>(items, it, end, step)) return;
  for (; it < end; it += step) {
    const int m = find_inst(D, n, it);
    const Geo g = D[m].g;
    const CState u = D[m].u;
    const long ndof = g.sc + g.sx + g.sy + g.sv;
    const long t0 = (long)(it - D[m].first) * DT_CHUNK;
    double mx = 0.0;
    for (long t = t0 + threadIdx.x; t < ndof && t < t0 + DT_CHUNK; t += BLK) {
      const double* base;
      long plane, off;
      dof_ptr(g, u, t, base, plane, off);
      double U[NV];
      load8(base, plane, off, U);
      mx = fmax(mx, dt_speed(U, g));
    }
    mx = block_max(mx);
    if (threadIdx.x == 0) partial[it] = mx;
  }
}

__global__ __launch_bounds__(BLK) void kb_dt_final(const BDt* __restrict__ D, const double* partial,
                                                   const double* t_rem, double* dt) {
  const int m = (int)blockIdx.x;
  double mx = 0.0;
  for (int t = threadIdx.x; t < D[m].nparts; t += BLK) mx = fmax(mx, partial[D[m].first + t]);
  mx = block_max(mx);
  if (threadIdx.x == 0) {
    const double d = D[m].cfl / mx;
    const double r = t_rem ? t_rem[m] : d;
    dt[m] = d > r ? r : d;
  }
}

__global__ void kb_zero_counters(Counters* cn) {
  if (threadIdx.x == 0) {
    cn->n_llf_not_admissible = cn->n_newton = cn->newton_iters_max = cn->n_fallback = cn->n_not_admissible = 0;
    cn->n_theta_active = cn->n_point_limited = cn->n_centre_limited = cn->n_source_limited = 0;
    cn->min_theta_bits = (unsigned long long)__double_as_longlong(1.0);
  }
}

// Launch helpers for a cell-tile shape and launch mode chosen at run time;
// grid is the persistent grid (flat launches size their own).
template <class R, bool P>
void launch_cells_m(int shape, int grid, hipStream_t s, const BInst* I, int n, int items, double ca, double cb,
                    Counters* cn) {
  const int g = P ? grid : flat_grid(items);
  if (shape == 0) kb_cells<R, 32, 16, P><<<g, dim3(32, 16), 0, s>>>(I, n, items, ca, cb, cn);
  else kb_cells<R, 16, 32, P><<<g, dim3(16, 32), 0, s>>>(I, n, items, ca, cb, cn);
}
template <class R>
void launch_cells(bool persist, int shape, int grid, hipStream_t s, const BInst* I, int n, int items, double ca,
                  double cb, Counters* cn) {
  if (persist) launch_cells_m<R, true>(shape, grid, s, I, n, items, ca, cb, cn);
  else launch_cells_m<R, false>(shape, grid, s, I, n, items, ca, cb, cn);
}
template <class R>
void launch_points(bool persist, int grid, hipStream_t s, const BInst* I, int n, int items, double ca, double cb,
                   Counters* cn) {
  if (persist) kb_points<R, true><<<grid, dim3(PB, PB), 0, s>>>(I, n, items, ca, cb, cn);
  else kb_points<R, false><<<flat_grid(items), dim3(PB, PB), 0, s>>>(I, n, items, ca, cb, cn);
}

template <class R>
void launch_fused(int shape, hipStream_t s, const BInst* P, const BInst* C, int n, int pitems, int citems,
                  double ca, double cb, Counters* cn) {
  const int grid = (pitems + 1) / 2 + citems;  // one work item per workgroup
  if (shape == 0) kb_stage<R, 32, 16><<<grid, dim3(32, 16), 0, s>>>(P, C, n, pitems, citems, ca, cb, cn);
  else kb_stage<R, 16, 32><<<grid, dim3(32, 16), 0, s>>>(P, C, n, pitems, citems, ca, cb, cn);
}
template <class R>
const void* cells_fn(int shape) {
  return shape == 0 ? reinterpret_cast<const void*>(&kb_cells<R, 32, 16, true>)
                    : reinterpret_cast<const void*>(&kb_cells<R, 16, 32, true>);
}

int cell_tiles_x(const Geo& g, int shape) { return (g.nx + SHAPE_X[shape] - 4) / (SHAPE_X[shape] - 3); }
int cell_tiles_y(const Geo& g, int shape) { return (g.ny + SHAPE_Y[shape] - 4) / (SHAPE_Y[shape] - 3); }
int point_tiles_x(const Geo& g) { return (g.nxp + PB - 3) / (PB - 2); }
int point_tiles_y(const Geo& g) { return (g.nyp + PB - 3) / (PB - 2); }

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct af_mhd_batch {
  int n = 0;
  bool f32 = false;
  hipStream_t stream = nullptr;
  std::vector<Geo> geo;
  std::vector<af_mhd_state> user;       // the bound states
  std::vector<af_mhd_state> s1, s2;     // RK scratch per instance
  std::vector<double*> src;             // nine-point source buffer per instance
  std::vector<int> shape;               // tuned cell-tile shape of each instance's size class
  int cshape = 0;                       // the shape of the batch's one cell launch
  double* dt = nullptr;                 // caller's dt array
  const double* t_rem = nullptr;        // caller's t_remaining array or null
  // device tables
  BInst* pts[3] = {nullptr, nullptr, nullptr};
  BInst* cls[3] = {nullptr, nullptr, nullptr};  // every instance, grouped by shape
  int pts_items = 0;
  int cls_items = 0;
  BDt* dts = nullptr;
  BInst* tune = nullptr;                // TUNE_COPIES entries for the autotuner
  int dt_items = 0;
  double* partial = nullptr;
  Counters* cnt = nullptr;
  int grid_points = 0, grid_cells = 0, grid_dt = 0;
  int mode = AF_BATCH_FLAT;             // launch mode of the stages
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string err;
  ~af_mhd_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

thread_local std::string batch_init_err;

bool valid_one(const af_mhd_params* p) {
  if (!p) return false;
  if (p->nx < 4 || p->ny < 4 || p->nx > (1 << 16) || p->ny > (1 << 16)) return false;
  if (!(p->x1 > p->x0) || !(p->y1 > p->y0) || !(p->gamma > 1.0)) return false;
  if (!(p->cfl > 0.0 && p->cfl <= 1.0) || !(p->kappa >= 0.0)) return false;
  if ((p->bc_x != AF_BC_PERIODIC && p->bc_x != AF_BC_OUTFLOW) ||
      (p->bc_y != AF_BC_PERIODIC && p->bc_y != AF_BC_OUTFLOW))
    return false;
  return (p->flags & ~(uint32_t)AF_FLAG_FP32_BULK) == 0;
}

void geo_of(const af_mhd_params* p, Geo& g) {
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

size_t state_doubles(const Geo& g) { return 8 * (size_t)(g.sc + g.sx + g.sy + g.sv); }

int dt_parts(const Geo& g) { return (int)((g.sc + g.sx + g.sy + g.sv + DT_CHUNK - 1) / DT_CHUNK); }

// Device workspace: per instance two scratch states and a nine-point source buffer,
// then the dt partials, the counters and the launch tables.
size_t batch_layout(const af_mhd_params* p, int n, char* base, af_mhd_batch* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* ptr = base ? base + off : nullptr;
    off += al256(bytes);
    return ptr;
  };
  int parts = 0;
  for (int m = 0; m < n; ++m) {
    Geo g;
    geo_of(&p[m], g);
    for (int k = 0; k < 2; ++k) {
      double* a = reinterpret_cast<double*>(take(8 * sizeof(double) * g.sc));
      double* x = reinterpret_cast<double*>(take(8 * sizeof(double) * g.sx));
      double* y = reinterpret_cast<double*>(take(8 * sizeof(double) * g.sy));
      double* v = reinterpret_cast<double*>(take(8 * sizeof(double) * g.sv));
      if (b) (k ? b->s2 : b->s1).push_back(af_mhd_state{a, x, y, v});
    }
    double* c = reinterpret_cast<double*>(take(8 * sizeof(double) * g.sc));
    if (b) b->src.push_back(c);
    parts += dt_parts(g);
  }
  double* partial = reinterpret_cast<double*>(take(sizeof(double) * parts));
  Counters* cnt = reinterpret_cast<Counters*>(take(sizeof(Counters)));
  char* tabs = take(sizeof(BInst) * (size_t)n * 3 * 2 + sizeof(BDt) * (size_t)n);
  char* tune = take(sizeof(BInst) * (size_t)TUNE_COPIES);
  if (b) {
    b->partial = partial;
    b->cnt = cnt;
    BInst* t = reinterpret_cast<BInst*>(tabs);
    for (int k = 0; k < 3; ++k) {
      b->pts[k] = t;
      t += n;
      b->cls[k] = t;
      t += n;
    }
    b->dts = reinterpret_cast<BDt*>(t);
    b->tune = reinterpret_cast<BInst*>(tune);
  }
  return off;
}

int bfail(af_mhd_batch* b, int code, const std::string& msg) {
  b->err = msg;
  return code;
}

int bcheck(af_mhd_batch* b, hipError_t e, const char* where) {
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) return AF_OK;
  return bfail(b, AF_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Persistent grid: as many workgroups as fit on the device at once, a
// multiple of 8 (at least 8).
int persistent_grid(const void* fn, int threads) {
  int dev = 0, cus = 256, per = 1;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, 0) != hipSuccess || per < 1) per = 1;
  const int g = cus * per;
  return std::max(NXCD, (g / NXCD) * NXCD);
}

// Fill the launch tables of every stage for the current shapes.
int build_tables(af_mhd_batch* b) {
  const int n = b->n;
  std::vector<BInst> pts(n), cls;
  std::vector<BDt> dts(n);
  for (int k = 0; k < 3; ++k) {
    int pfirst = 0, cfirst = 0;
    cls.clear();
    const int q = b->cshape;
    for (int m = 0; m < n; ++m) {
      const Geo& g = b->geo[m];
      const af_mhd_state& U = b->user[m];
      const af_mhd_state& in = k == 0 ? U : (k == 1 ? b->s1[m] : b->s2[m]);
      const af_mhd_state& out = k == 0 ? b->s1[m] : (k == 1 ? b->s2[m] : U);
      BInst r;
      r.g = g;
      r.u = CState{in.cell, in.xface, in.yface, in.vert};
      r.un = CState{U.cell, U.xface, U.yface, U.vert};
      r.out = MState{out.cell, out.xface, out.yface, out.vert};
      r.src = b->src[m];
      r.dt = b->dt + m;
      r.first = cfirst;
      r.ntx = cell_tiles_x(g, q);
      cls.push_back(r);
      cfirst += cell_tiles_x(g, q) * cell_tiles_y(g, q);
    }
    for (int m = 0; m < n; ++m) {
      const Geo& g = b->geo[m];
      const af_mhd_state& U = b->user[m];
      const af_mhd_state& in = k == 0 ? U : (k == 1 ? b->s1[m] : b->s2[m]);
      const af_mhd_state& out = k == 0 ? b->s1[m] : (k == 1 ? b->s2[m] : U);
      BInst r;
      r.g = g;
      r.u = CState{in.cell, in.xface, in.yface, in.vert};
      r.un = CState{U.cell, U.xface, U.yface, U.vert};
      r.out = MState{out.cell, out.xface, out.yface, out.vert};
      r.src = b->src[m];
      r.dt = b->dt + m;
      r.first = pfirst;
      r.ntx = point_tiles_x(g);
      pts[m] = r;
      pfirst += point_tiles_x(g) * point_tiles_y(g);
    }
    b->pts_items = pfirst;
    b->cls_items = cfirst;
    hipError_t e = hipMemcpyAsync(b->pts[k], pts.data(), sizeof(BInst) * n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->cls[k], cls.data(), sizeof(BInst) * n, hipMemcpyHostToDevice, b->stream);
    // the host vectors are reused for the next stage: the copies must be done
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bcheck(b, e, "batch tables");
  }
  int first = 0;
  for (int m = 0; m < n; ++m) {
    const Geo& g = b->geo[m];
    const af_mhd_state& U = b->user[m];
    dts[m].g = g;
    dts[m].u = CState{U.cell, U.xface, U.yface, U.vert};
    dts[m].first = first;
    dts[m].nparts = dt_parts(g);
    dts[m].cfl = g.cfl;
    first += dts[m].nparts;
  }
  b->dt_items = first;
  hipError_t e = hipMemcpyAsync(b->dts, dts.data(), sizeof(BDt) * n, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return bcheck(b, e, "batch tables");
}

// The launches of stage k in the batch's mode.
void enqueue_stage(af_mhd_batch* b, int k, double a, double c) {
  hipStream_t s = b->stream;
  if (b->mode == AF_BATCH_FUSED) {
    if (b->f32)
      launch_fused<float>(b->cshape, s, b->pts[k], b->cls[k], b->n, b->pts_items, b->cls_items, a, c, b->cnt);
    else
      launch_fused<double>(b->cshape, s, b->pts[k], b->cls[k], b->n, b->pts_items, b->cls_items, a, c, b->cnt);
    return;
  }
  const bool persist = b->mode == AF_BATCH_PERSISTENT;
  if (b->f32) launch_points<float>(persist, b->grid_points, s, b->pts[k], b->n, b->pts_items, a, c, b->cnt);
  else launch_points<double>(persist, b->grid_points, s, b->pts[k], b->n, b->pts_items, a, c, b->cnt);
  if (b->f32) launch_cells<float>(persist, b->cshape, b->grid_cells, s, b->cls[k], b->n, b->cls_items, a, c, b->cnt);
  else launch_cells<double>(persist, b->cshape, b->grid_cells, s, b->cls[k], b->n, b->cls_items, a, c, b->cnt);
}

// The launches of one step (also what the graph records).
int enqueue_step(af_mhd_batch* b) {
  static const double A[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double B[3] = {1.0, 0.25, 2.0 / 3.0};
  hipStream_t s = b->stream;
  kb_dt_partial<<<b->grid_dt, BLK, 0, s>>>(b->dts, b->n, b->dt_items, b->partial);
  kb_dt_final<<<b->n, BLK, 0, s>>>(b->dts, b->partial, b->t_rem, b->dt);
  for (int k = 0; k < 3; ++k) enqueue_stage(b, k, A[k], B[k]);
  return bcheck(b, hipSuccess, "batch step launch");
}

// ------------------------------------------------------------- autotuner
// Key of a size class: grid size, boundaries and precision.
std::string class_key(const Geo& g, bool f32) {
  char buf[96];
  std::snprintf(buf, sizeof buf, "%d %d %d %d %s", g.nx, g.ny, g.bcx, g.bcy, f32 ? "fp32" : "fp64");
  return buf;
}

std::map<std::string, int> read_table(const char* path) {
  std::map<std::string, int> t;
  FILE* f = path ? std::fopen(path, "r") : nullptr;
  if (!f) return t;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    int nx, ny, bx, by, q;
    char prec[8];
    if (std::sscanf(line, "%d %d %d %d %7s %d", &nx, &ny, &bx, &by, prec, &q) == 6 && q >= 0 && q < NSHAPE) {
      char key[96];
      std::snprintf(key, sizeof key, "%d %d %d %d %s", nx, ny, bx, by, prec);
      t[key] = q;
    }
  }
  std::fclose(f);
  return t;
}

// Throughput of the cell update of instance m under each shape: its work
// items repeated until a launch carries about TUNE_ITEMS of them (a filled
// device, as in a batch), computing stage 0 into the instance's scratch
// state (the copies write identical values); the point update runs first so
// that the source buffer is valid.  Returns the fastest shape; us[] gets
// the time per instance-launch of each shape.
int tune_instance(af_mhd_batch* b, int m, double us[NSHAPE]) {
  const Geo& g = b->geo[m];
  const af_mhd_state& U = b->user[m];
  BInst r;
  r.g = g;
  r.u = CState{U.cell, U.xface, U.yface, U.vert};
  r.un = r.u;
  r.out = MState{b->s1[m].cell, b->s1[m].xface, b->s1[m].yface, b->s1[m].vert};
  r.src = b->src[m];
  r.dt = b->dt + m;
  hipStream_t s = b->stream;
  // a valid dt for the instances first
  kb_dt_partial<<<b->grid_dt, BLK, 0, s>>>(b->dts, b->n, b->dt_items, b->partial);
  kb_dt_final<<<b->n, BLK, 0, s>>>(b->dts, b->partial, nullptr, b->dt);
  BInst* dev = b->tune;
  r.first = 0;
  r.ntx = point_tiles_x(g);
  hipError_t e = hipMemcpyAsync(dev, &r, sizeof r, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return -1;
  const int pitems = point_tiles_x(g) * point_tiles_y(g);
  if (b->f32) launch_points<float>(false, 0, s, dev, 1, pitems, 0.0, 1.0, b->cnt);
  else launch_points<double>(false, 0, s, dev, 1, pitems, 0.0, 1.0, b->cnt);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1;
  }
  int best = 0;
  std::vector<BInst> copies;
  for (int q = 0; q < NSHAPE && e == hipSuccess; ++q) {
    const int items = cell_tiles_x(g, q) * cell_tiles_y(g, q);
    const int reps = std::max(1, std::min(TUNE_COPIES, TUNE_ITEMS / items));
    copies.assign(reps, r);
    for (int c = 0; c < reps; ++c) {
      copies[c].first = c * items;
      copies[c].ntx = cell_tiles_x(g, q);
    }
    e = hipMemcpyAsync(dev, copies.data(), sizeof(BInst) * reps, hipMemcpyHostToDevice, s);
    float best_ms = 1e30f;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, s);
      if (b->f32) launch_cells<float>(false, q, 0, s, dev, reps, reps * items, 0.0, 1.0, b->cnt);
      else launch_cells<double>(false, q, 0, s, dev, reps, reps * items, 0.0, 1.0, b->cnt);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) best_ms = std::min(best_ms, ms);  // the first launch warms up
    }
    us[q] = 1e3 * best_ms / reps;
    if (us[q] < us[best]) best = q;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e == hipSuccess ? best : -1;
}

// Time the launches of stage 0 (dt, point and cell updates into the
// scratch states; the caller's states are only read) in the current mode.
double time_stage0(af_mhd_batch* b, int reps) {
  static const double A0 = 0.0, B0 = 1.0;
  hipStream_t s = b->stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  float best = 1e30f;
  hipError_t e = hipSuccess;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, s);
    kb_dt_partial<<<b->grid_dt, BLK, 0, s>>>(b->dts, b->n, b->dt_items, b->partial);
    kb_dt_final<<<b->n, BLK, 0, s>>>(b->dts, b->partial, b->t_rem, b->dt);
    enqueue_stage(b, 0, A0, B0);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (r > 0) best = std::min(best, ms);  // the first round warms up
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e == hipSuccess ? (double)best : -1.0;
}

}  // namespace

extern "C" {

size_t af_mhd_batch_workspace_bytes(const af_mhd_params* p, int n) {
  if (!p || n < 1 || n > (1 << 20)) return 0;
  for (int m = 0; m < n; ++m)
    if (!valid_one(&p[m]) || p[m].flags != p[0].flags) return 0;
  return batch_layout(p, n, nullptr, nullptr);
}

int af_mhd_batch_init(const af_mhd_params* p, int n, const af_mhd_state* states, double* dt_dev,
                      const double* t_remaining_dev, void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                      const char* tune_table, af_mhd_batch** out) {
  batch_init_err.clear();
  auto ifail = [](int code, const char* msg) {
    batch_init_err = msg;
    return code;
  };
  if (!out || !states || !dt_dev || ((uintptr_t)dt_dev & 7)) return ifail(AF_EINVAL, "af_mhd_batch_init: bad argument");
  const size_t need = af_mhd_batch_workspace_bytes(p, n);
  if (need == 0) return ifail(AF_EINVAL, "af_mhd_batch_init: invalid parameters");
  if (!workspace_dev || ((uintptr_t)workspace_dev & 255))
    return ifail(AF_EINVAL, "af_mhd_batch_init: workspace null or not 256-byte aligned");
  if (workspace_bytes < need) return ifail(AF_EWORKSPACE, "af_mhd_batch_init: workspace too small");
  for (int m = 0; m < n; ++m) {
    const af_mhd_state& s = states[m];
    for (const double* q : {s.cell, s.xface, s.yface, s.vert})
      if (!q || ((uintptr_t)q & 7)) return ifail(AF_EINVAL, "af_mhd_batch_init: state pointer null or misaligned");
  }
  af_mhd_batch* b = new (std::nothrow) af_mhd_batch();
  if (!b) return ifail(AF_EINVAL, "af_mhd_batch_init: out of host memory");
  b->n = n;
  b->f32 = (p[0].flags & AF_FLAG_FP32_BULK) != 0;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->dt = dt_dev;
  b->t_rem = t_remaining_dev;
  for (int m = 0; m < n; ++m) {
    Geo g;
    geo_of(&p[m], g);
    b->geo.push_back(g);
    b->user.push_back(states[m]);
  }
  batch_layout(p, n, static_cast<char*>(workspace_dev), b);
  b->grid_points = b->f32 ? persistent_grid(reinterpret_cast<const void*>(&kb_points<float, true>), PNT)
                          : persistent_grid(reinterpret_cast<const void*>(&kb_points<double, true>), PNT);
  b->grid_cells = persistent_grid(b->f32 ? cells_fn<float>(0) : cells_fn<double>(0), 512);  // 512 threads either shape
  b->grid_dt = persistent_grid(reinterpret_cast<const void*>(&kb_dt_partial), BLK);
  (void)hipGetLastError();
  kb_zero_counters<<<1, 64, 0, b->stream>>>(b->cnt);
  // shapes: from the table, by measurement for classes it lacks, else 0
  b->shape.assign(n, 0);
  int rc = build_tables(b);
  if (rc == AF_OK && tune_table) {
    std::map<std::string, int> table = read_table(tune_table);
    std::map<std::string, std::vector<double>> measured;
    for (int m = 0; m < n && rc == AF_OK; ++m) {
      const std::string key = class_key(b->geo[m], b->f32);
      auto it = table.find(key);
      if (it == table.end()) {
        double us[NSHAPE];
        const int q = tune_instance(b, m, us);
        if (q < 0) {
          rc = bcheck(b, hipErrorUnknown, "autotune");
          break;
        }
        table[key] = q;
        measured[key] = std::vector<double>(us, us + NSHAPE);
        it = table.find(key);
      }
      b->shape[m] = it->second;
    }
    if (rc == AF_OK && !measured.empty()) {
      FILE* f = std::fopen(tune_table, "a");
      if (f) {
        for (auto& kv : measured) {
          std::fprintf(f, "%s %d  # us:", kv.first.c_str(), table[kv.first]);
          for (int q = 0; q < NSHAPE; ++q) std::fprintf(f, " %dx%d=%.2f", SHAPE_X[q], SHAPE_Y[q], kv.second[q]);
          std::fprintf(f, "\n");
        }
        std::fclose(f);
      }
    }
    if (rc == AF_OK) {
      // the batch's one cell launch takes the shape tuned for most of its cells
      long cells[NSHAPE] = {0, 0};
      for (int m = 0; m < n; ++m) cells[b->shape[m]] += (long)b->geo[m].nx * b->geo[m].ny;
      b->cshape = cells[1] > cells[0] ? 1 : 0;
      rc = build_tables(b);
    }
  }
  if (rc == AF_OK && tune_table) {
    // launch mode of the whole batch: the fastest of the three on stage 0
    double best = -1.0;
    int best_mode = AF_BATCH_FLAT;
    for (int mode : {AF_BATCH_FUSED, AF_BATCH_PERSISTENT, AF_BATCH_FLAT}) {
      b->mode = mode;
      const double t = time_stage0(b, 3);
      if (t < 0.0) {
        rc = bcheck(b, hipErrorUnknown, "autotune (launch mode)");
        break;
      }
      if (best < 0.0 || t < best) {
        best = t;
        best_mode = mode;
      }
    }
    b->mode = best_mode;
    kb_zero_counters<<<1, 64, 0, b->stream>>>(b->cnt);
    if (rc == AF_OK) rc = bcheck(b, hipStreamSynchronize(b->stream), "autotune");
  }
  if (rc != AF_OK) {
    batch_init_err = b->err;
    delete b;
    return rc;
  }
  *out = b;
  return AF_OK;
}

int af_mhd_batch_step(af_mhd_batch* b, int use_graph) {
  if (!b) return AF_EINVAL;
  if (!use_graph) return enqueue_step(b);
  hipError_t e = hipSuccess;
  if (!b->exec) {
    e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bcheck(b, e, "graph capture");
    enqueue_step(b);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bcheck(b, e, "graph instantiate");
  }
  e = hipGraphLaunch(b->exec, b->stream);
  return bcheck(b, e, "graph launch");
}

int af_mhd_batch_tile(const af_mhd_batch* b, int m, int* tile_x, int* tile_y) {
  if (!b || m < 0 || m >= b->n || !tile_x || !tile_y) return AF_EINVAL;
  *tile_x = SHAPE_X[b->cshape];
  *tile_y = SHAPE_Y[b->cshape];
  return AF_OK;
}

int af_mhd_batch_counters(af_mhd_batch* b, af_mhd_stats_t* out) {
  if (!b || !out) return AF_EINVAL;
  Counters cn;
  hipError_t e = hipMemcpyAsync(&cn, b->cnt, sizeof cn, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bcheck(b, e, "af_mhd_batch_counters");
  std::memset(out, 0, sizeof *out);
  double mt;
  std::memcpy(&mt, &cn.min_theta_bits, sizeof mt);
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
  b->err.clear();
  return AF_OK;
}

int af_mhd_batch_launch_mode(const af_mhd_batch* b, int* mode) {
  if (!b || !mode) return AF_EINVAL;
  *mode = b->mode;
  return AF_OK;
}

int af_mhd_batch_set_launch_mode(af_mhd_batch* b, int mode) {
  if (!b) return AF_EINVAL;
  if (mode != AF_BATCH_FLAT && mode != AF_BATCH_PERSISTENT && mode != AF_BATCH_FUSED)
    return bfail(b, AF_EINVAL, "af_mhd_batch_set_launch_mode: unknown mode");
  if (mode == b->mode) return AF_OK;
  // the captured step is the old mode's: drop it, the next graph step records the new one
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->mode = mode;
  b->err.clear();
  return AF_OK;
}


void af_mhd_batch_destroy(af_mhd_batch* b) { delete b; }

const char* af_mhd_batch_last_error(const af_mhd_batch* b) { return b ? b->err.c_str() : batch_init_err.c_str(); }

}  // extern "C"
