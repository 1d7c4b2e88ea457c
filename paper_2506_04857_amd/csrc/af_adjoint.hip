// af_adjoint.hip -- kernels and C ABI of the recorded stage and of its
// discrete adjoint (the transposed Jacobian of one SSP-RK3 stage with the
// limiter and sensor decisions frozen as the forward took them).
//
// One thread per entity (centre, point, sensor cell, interface, limiter
// cell, update cell); launches run in dependency order on the context's
// stream.  The reverse sweep scatters with hardware FP64 atomics into the
// adjoint states and into the intermediate adjoint buffers of the
// workspace (the centre's adjoint is gathered by the points instead), so
// its sums are order-dependent at the rounding level (not bitwise
// reproducible run to run).
// No contraction of a*b+c into fused multiply-adds in this translation unit
// (it must precede the includes to cover the entity functions): the
// recording forward and the reverse sweep then round like the FP64 oracle,
// so exact cancellations on symmetric data stay exact and the branches taken
// at them (|0|, max ties) are the oracle's.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <new>
#include <string>

#include "af_adjoint_stage.h"
#include "af_mhd.h"

using namespace afadj;

namespace {

constexpr int ABLK = 256;

struct DevAdd {
  __device__ static void add(double* p, double v) { unsafeAtomicAdd(p, v); }
};

__device__ __forceinline__ long gtid() { return (long)blockIdx.x * ABLK + threadIdx.x; }
inline int nblk(long n) { return (int)((n + ABLK - 1) / ABLK); }

// ---------------------------------------------------------------- record
__global__ __launch_bounds__(ABLK) void kr_centre(AGeo g, StateC u, Tape t) {
  const long q = gtid();
  if (q >= (long)g.nx * g.ny) return;
  rec_centre(g, u, t, (int)(q % g.nx), (int)(q / g.nx));
}
__global__ __launch_bounds__(ABLK) void kr_sensor(AGeo g, StateC u, Tape t) {
  const Ext e = ext_of(g);
  const long q = gtid();
  if (q >= (long)e.sw * e.sh) return;
  rec_sensor(g, u, t, (int)(q % e.sw) - 2, (int)(q / e.sw) - 2);
}
__global__ __launch_bounds__(ABLK) void kr_iface(AGeo g, StateC u, Tape t) {
  const Ext e = ext_of(g);
  const long nx = (long)e.xw * e.xh, q = gtid();
  if (q < nx)
    rec_iface(g, u, t, 0, (int)(q % e.xw) - 1, (int)(q / e.xw) - 1);
  else if (q < nx + (long)e.yw * e.yh)
    rec_iface(g, u, t, 1, (int)((q - nx) % e.yw) - 1, (int)((q - nx) / e.yw) - 1);
}
__global__ __launch_bounds__(ABLK) void kr_limiter(AGeo g, StateC u, Tape t, const double* dt) {
  const Ext e = ext_of(g);
  const long q = gtid();
  if (q >= (long)e.ew * e.eh) return;
  rec_limiter(g, u, t, (int)(q % e.ew) - 1, (int)(q / e.ew) - 1, *dt);
}
__global__ __launch_bounds__(ABLK) void kr_update(AGeo g, StateC un, StateC u, Tape t, double* out, const double* dt,
                                                  double a, double b) {
  const long q = gtid();
  if (q >= (long)g.nx * g.ny) return;
  rec_update(g, un, u, t, out, (int)(q % g.nx), (int)(q / g.nx), *dt, a, b);
}
// Points of the three sets in one launch: X, then Y, then V.
__device__ __forceinline__ bool point_of(const AGeo& g, long q, int& kind, int& k, int& l) {
  const long nX = (long)g.nxp * g.ny, nY = (long)g.nx * g.nyp, nV = (long)g.nxp * g.nyp;
  if (q < nX) {
    kind = 0;
    k = (int)(q % g.nxp);
    l = (int)(q / g.nxp);
  } else if (q < nX + nY) {
    q -= nX;
    kind = 1;
    k = (int)(q % g.nx);
    l = (int)(q / g.nx);
  } else if (q < nX + nY + nV) {
    q -= nX + nY;
    kind = 2;
    k = (int)(q % g.nxp);
    l = (int)(q / g.nxp);
  } else {
    return false;
  }
  return true;
}
__global__ __launch_bounds__(ABLK) void kr_points(AGeo g, StateC un, StateC u, Tape t, StateM out, const double* dt,
                                                  double a, double b) {
  int kind, k, l;
  if (!point_of(g, gtid(), kind, k, l)) return;
  double* o = kind == 0 ? out.x : kind == 1 ? out.y : out.v;
  rec_point(g, un, u, t, o, kind, k, l, *dt, a, b);
}

// --------------------------------------------------------------- reverse
__global__ __launch_bounds__(ABLK) void ka_zero(double* p, long n) {
  for (long q = gtid(); q < n; q += (long)gridDim.x * ABLK) p[q] = 0.0;
}
__global__ __launch_bounds__(ABLK) void ka_update(AGeo g, Tape t, AdjBuf ab, StateC lo, StateM ln, StateM lk,
                                                  const double* dt, double a, double b) {
  const long q = gtid();
  if (q >= (long)g.nx * g.ny) return;
  adj_update<DevAdd>(g, t, ab, lo, ln, lk, (int)(q % g.nx), (int)(q / g.nx), *dt, a, b);
}
__global__ __launch_bounds__(ABLK) void ka_limiter(AGeo g, StateC u, Tape t, AdjBuf ab, StateM lk, const double* dt) {
  const Ext e = ext_of(g);
  const long q = gtid();
  if (q >= (long)e.ew * e.eh) return;
  adj_limiter<DevAdd>(g, u, t, ab, lk, (int)(q % e.ew) - 1, (int)(q / e.ew) - 1, *dt);
}
__global__ __launch_bounds__(ABLK) void ka_iface(AGeo g, StateC u, Tape t, AdjBuf ab, StateM lk) {
  const Ext e = ext_of(g);
  const long nx = (long)e.xw * e.xh, q = gtid();
  if (q < nx)
    adj_iface<DevAdd>(g, u, t, ab, lk, 0, (int)(q % e.xw) - 1, (int)(q / e.xw) - 1);
  else if (q < nx + (long)e.yw * e.yh)
    adj_iface<DevAdd>(g, u, t, ab, lk, 1, (int)((q - nx) % e.yw) - 1, (int)((q - nx) / e.yw) - 1);
}
__global__ __launch_bounds__(ABLK) void ka_sensor(AGeo g, StateC u, Tape t, AdjBuf ab, StateM lk) {
  const Ext e = ext_of(g);
  const long q = gtid();
  if (q >= (long)e.sw * e.sh) return;
  adj_sensor<DevAdd>(g, u, t, ab, lk, (int)(q % e.sw) - 2, (int)(q / e.sw) - 2);
}
__global__ __launch_bounds__(ABLK) void ka_points(AGeo g, StateC u, Tape t, AdjBuf ab, StateC lo, StateM ln, StateM lk,
                                                  const double* dt, double a, double b) {
  int kind, k, l;
  if (!point_of(g, gtid(), kind, k, l)) return;
  adj_point<DevAdd>(g, u, t, ab, lo, ln, lk, kind, k, l, *dt, a, b);
}
__global__ __launch_bounds__(ABLK) void ka_centre(AGeo g, StateC u, Tape t, AdjBuf ab, StateM lk) {
  const long q = gtid();
  if (q >= (long)g.nx * g.ny) return;
  adj_centre<DevAdd>(g, u, t, ab, lk, (int)(q % g.nx), (int)(q / g.nx));
}
__global__ __launch_bounds__(ABLK) void ka_centre_gather(AGeo g, AdjBuf ab, StateM lk) {
  int kind, k, l;
  if (!point_of(g, gtid(), kind, k, l)) return;
  adj_centre_gather(g, ab, lk, kind, k, l);
}

thread_local std::string adj_init_err;

bool valid_params(const af_mhd_params* p) {
  if (!p) return false;
  if (p->nx < 4 || p->ny < 4 || p->nx > (1 << 16) || p->ny > (1 << 16)) return false;
  if (!(p->x1 > p->x0) || !(p->y1 > p->y0) || !(p->gamma > 1.0)) return false;
  if (!(p->cfl > 0.0 && p->cfl <= 1.0) || !(p->kappa >= 0.0)) return false;
  if ((p->bc_x != AF_BC_PERIODIC && p->bc_x != AF_BC_OUTFLOW) || (p->bc_y != AF_BC_PERIODIC && p->bc_y != AF_BC_OUTFLOW))
    return false;
  return p->flags == 0;  // FP64 only
}
AGeo make_ageo(const af_mhd_params* p) {
  AGeo g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.bcx = p->bc_x;
  g.bcy = p->bc_y;
  g.nxp = p->nx + (p->bc_x == AF_BC_OUTFLOW ? 1 : 0);
  g.nyp = p->ny + (p->bc_y == AF_BC_OUTFLOW ? 1 : 0);
  g.dx = (p->x1 - p->x0) / p->nx;
  g.dy = (p->y1 - p->y0) / p->ny;
  g.gamma = p->gamma;
  g.kappa = p->kappa;
  return g;
}
bool aligned8(const void* p) { return p && ((uintptr_t)p & 7) == 0; }
bool valid_state(const af_mhd_state* s) {
  return s && aligned8(s->cell) && aligned8(s->xface) && aligned8(s->yface) && aligned8(s->vert);
}
StateC sc(const af_mhd_state* s) { return StateC{s->cell, s->xface, s->yface, s->vert}; }
StateM sm(const af_mhd_state* s) { return StateM{s->cell, s->xface, s->yface, s->vert}; }
bool same_state(const af_mhd_state* a, const af_mhd_state* b) {
  return a->cell == b->cell || a->xface == b->xface || a->yface == b->yface || a->vert == b->vert;
}

const double RK_A[3] = {0.0, 0.75, 1.0 / 3.0};
const double RK_B[3] = {1.0, 0.25, 2.0 / 3.0};

}  // namespace

struct af_mhd_adj {
  AGeo g;
  AdjBuf ab;
  double* ab_base;
  size_t ab_doubles;
  size_t tape_bytes;
  hipStream_t stream;
  // The reverse of the point update runs on an auxiliary stream beside the
  // reverse of the cell update: the two only add into the shared adjoint
  // buffers (atomics), and the centre kernels that read them wait for both.
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::string err;
  ~af_mhd_adj() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (aux) (void)hipStreamDestroy(aux);
  }
};

namespace {
int fail(af_mhd_adj* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}
int check_hip(af_mhd_adj* c, const char* where) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return AF_OK;
  return fail(c, AF_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}
}  // namespace

extern "C" {

size_t af_mhd_adj_tape_bytes(const af_mhd_params* p) {
  if (!valid_params(p)) return 0;
  return tape_layout(make_ageo(p), nullptr, nullptr);
}

size_t af_mhd_adj_workspace_bytes(const af_mhd_params* p) {
  if (!valid_params(p)) return 0;
  return adjbuf_layout(make_ageo(p), nullptr, nullptr);
}

int af_mhd_adj_init(const af_mhd_params* p, void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                    af_mhd_adj** out) {
  adj_init_err.clear();
  if (!out) return adj_init_err = "af_mhd_adj_init: null output", AF_EINVAL;
  if (!valid_params(p)) return adj_init_err = "af_mhd_adj_init: invalid parameters (FP64 only)", AF_EINVAL;
  if (!workspace_dev || ((uintptr_t)workspace_dev & 255))
    return adj_init_err = "af_mhd_adj_init: workspace null or not 256-byte aligned", AF_EINVAL;
  const AGeo g = make_ageo(p);
  const size_t need = adjbuf_layout(g, nullptr, nullptr);
  if (workspace_bytes < need) return adj_init_err = "af_mhd_adj_init: workspace too small", AF_EWORKSPACE;
  af_mhd_adj* c = new (std::nothrow) af_mhd_adj();
  if (!c) return adj_init_err = "af_mhd_adj_init: out of host memory", AF_EINVAL;
  c->g = g;
  adjbuf_layout(g, static_cast<char*>(workspace_dev), &c->ab);
  c->ab_base = static_cast<double*>(workspace_dev);
  c->ab_doubles = need / sizeof(double);
  c->tape_bytes = tape_layout(g, nullptr, nullptr);
  c->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join, hipEventDisableTiming);
  if (e != hipSuccess) {
    adj_init_err = std::string("af_mhd_adj_init: ") + hipGetErrorString(e);
    delete c;
    return AF_EHIP;
  }
  *out = c;
  return AF_OK;
}

int af_mhd_adj_record(af_mhd_adj* c, int k, const af_mhd_state* un, const af_mhd_state* uk, af_mhd_state* out,
                      const double* dt_dev, void* tape_dev, size_t tape_bytes) {
  if (!c) return AF_EINVAL;
  if (k < 0 || k > 2 || !valid_state(uk) || !valid_state(out) || (k > 0 && !valid_state(un)) || !aligned8(dt_dev) ||
      !tape_dev || ((uintptr_t)tape_dev & 255))
    return fail(c, AF_EINVAL, "af_mhd_adj_record: bad argument");
  if (tape_bytes < c->tape_bytes) return fail(c, AF_EWORKSPACE, "af_mhd_adj_record: tape too small");
  if (same_state(out, uk)) return fail(c, AF_EINVAL, "af_mhd_adj_record: out aliases uk");
  const AGeo& g = c->g;
  const Ext e = ext_of(g);
  Tape t;
  tape_layout(g, static_cast<char*>(tape_dev), &t);
  const StateC u = sc(uk), n = sc(k == 0 ? uk : un);
  const StateM o = sm(out);
  const double a = RK_A[k], b = RK_B[k];
  hipStream_t s = c->stream;
  (void)hipGetLastError();
  kr_centre<<<nblk((long)g.nx * g.ny), ABLK, 0, s>>>(g, u, t);
  // fork: the points need only the centre values; they run on the
  // auxiliary stream beside the cell chain (disjoint outputs and tape fields)
  hipError_t he = hipEventRecord(c->fork, s);
  if (he == hipSuccess) he = hipStreamWaitEvent(c->aux, c->fork, 0);
  if (he != hipSuccess) return fail(c, AF_EHIP, std::string("af_mhd_adj_record: ") + hipGetErrorString(he));
  kr_points<<<nblk((long)g.nxp * g.ny + (long)g.nx * g.nyp + (long)g.nxp * g.nyp), ABLK, 0, c->aux>>>(
      g, n, u, t, o, dt_dev, a, b);
  he = hipEventRecord(c->join, c->aux);
  kr_sensor<<<nblk((long)e.sw * e.sh), ABLK, 0, s>>>(g, u, t);
  kr_iface<<<nblk((long)e.xw * e.xh + (long)e.yw * e.yh), ABLK, 0, s>>>(g, u, t);
  kr_limiter<<<nblk((long)e.ew * e.eh), ABLK, 0, s>>>(g, u, t, dt_dev);
  kr_update<<<nblk((long)g.nx * g.ny), ABLK, 0, s>>>(g, n, u, t, o.a, dt_dev, a, b);
  // join: the stage's output and tape are complete on s
  if (he == hipSuccess) he = hipStreamWaitEvent(s, c->join, 0);
  if (he != hipSuccess) return fail(c, AF_EHIP, std::string("af_mhd_adj_record: ") + hipGetErrorString(he));
  return check_hip(c, "af_mhd_adj_record");
}

int af_mhd_adj_stage(af_mhd_adj* c, int k, const af_mhd_state* uk, const void* tape_dev, size_t tape_bytes,
                     const double* dt_dev, const af_mhd_state* lam_out, af_mhd_state* lam_n, af_mhd_state* lam_k) {
  if (!c) return AF_EINVAL;
  if (k < 0 || k > 2 || !valid_state(uk) || !valid_state(lam_out) || !valid_state(lam_k) ||
      (k > 0 && !valid_state(lam_n)) || !aligned8(dt_dev) || !tape_dev || ((uintptr_t)tape_dev & 255))
    return fail(c, AF_EINVAL, "af_mhd_adj_stage: bad argument");
  if (tape_bytes < c->tape_bytes) return fail(c, AF_EWORKSPACE, "af_mhd_adj_stage: tape too small");
  if (same_state(lam_out, lam_k) || (k > 0 && same_state(lam_out, lam_n)))
    return fail(c, AF_EINVAL, "af_mhd_adj_stage: lam_out aliases an accumulator");
  const AGeo& g = c->g;
  const Ext e = ext_of(g);
  Tape t;
  tape_layout(g, static_cast<char*>(const_cast<void*>(tape_dev)), &t);
  const StateC u = sc(uk), lo = sc(lam_out);
  const StateM lk = sm(lam_k), ln = sm(k == 0 ? lam_k : lam_n);  // a_0 = 0: lam_n untouched
  const double a = RK_A[k], b = RK_B[k];
  hipStream_t s = c->stream;
  (void)hipGetLastError();
  ka_zero<<<nblk((long)c->ab_doubles) < 4096 ? nblk((long)c->ab_doubles) : 4096, ABLK, 0, s>>>(c->ab_base,
                                                                                                (long)c->ab_doubles);
  // fork: the points' reverse on the auxiliary stream, the cells' on s
  hipError_t he = hipEventRecord(c->fork, s);
  if (he == hipSuccess) he = hipStreamWaitEvent(c->aux, c->fork, 0);
  if (he != hipSuccess) return fail(c, AF_EHIP, std::string("af_mhd_adj_stage: ") + hipGetErrorString(he));
  ka_points<<<nblk((long)g.nxp * g.ny + (long)g.nx * g.nyp + (long)g.nxp * g.nyp), ABLK, 0, c->aux>>>(
      g, u, t, c->ab, lo, ln, lk, dt_dev, a, b);
  he = hipEventRecord(c->join, c->aux);
  ka_update<<<nblk((long)g.nx * g.ny), ABLK, 0, s>>>(g, t, c->ab, lo, ln, lk, dt_dev, a, b);
  ka_limiter<<<nblk((long)e.ew * e.eh), ABLK, 0, s>>>(g, u, t, c->ab, lk, dt_dev);
  ka_iface<<<nblk((long)e.xw * e.xh + (long)e.yw * e.yh), ABLK, 0, s>>>(g, u, t, c->ab, lk);
  ka_sensor<<<nblk((long)e.sw * e.sh), ABLK, 0, s>>>(g, u, t, c->ab, lk);
  // join: the centre kernels read what both sides added
  if (he == hipSuccess) he = hipStreamWaitEvent(s, c->join, 0);
  if (he != hipSuccess) return fail(c, AF_EHIP, std::string("af_mhd_adj_stage: ") + hipGetErrorString(he));
  ka_centre<<<nblk((long)g.nx * g.ny), ABLK, 0, s>>>(g, u, t, c->ab, lk);
  ka_centre_gather<<<nblk((long)g.nxp * g.ny + (long)g.nx * g.nyp + (long)g.nxp * g.nyp), ABLK, 0, s>>>(g, c->ab, lk);
  return check_hip(c, "af_mhd_adj_stage");
}

void af_mhd_adj_destroy(af_mhd_adj* c) { delete c; }

const char* af_mhd_adj_last_error(const af_mhd_adj* c) { return c ? c->err.c_str() : adj_init_err.c_str(); }

}  // extern "C"
