// af_limiters.hip -- the stage's positivity limiters applied to given inputs
// (af_mhd_limiters_apply): one thread per item, calling the very device
// functions the stage kernels call -- the point scaling limiter (Section
// 3.3), the centre-value limiter (remark rmk:cell_center), steps (1) and (2)
// of the parametrized flux limiter (Section 3.2), each with the round-off
// fallback of the closing remark of Section 4.  A verification aid: on
// identical inputs they can be compared bit for bit with a reference.
#include <hip/hip_runtime.h>

#include "af_device.h"
#include "af_mhd.h"

using namespace afm;

static_assert(sizeof(af_mhd_counters_t) == sizeof(Counters), "counter layouts agree");

namespace {

constexpr int LBLK = 64;

template <bool SHORTCUT>
__global__ __launch_bounds__(LBLK) void k_limiters(int kind, long n, double gm1, const double* __restrict__ in,
                                                   double* __restrict__ out, Counters* cn) {
  const long t = (long)blockIdx.x * LBLK + threadIdx.x;
  if (t >= n) return;
  if (kind == AF_LIM_POINT || kind == AF_LIM_CENTRE) {
    const double* q = in + 16 * t;
    double a[NV], b[NV], w[NV];
    for (int c = 0; c < NV; ++c) {
      a[c] = q[c];
      b[c] = q[NV + c];
    }
    if (kind == AF_LIM_POINT)
      limit_point(a, b, gm1, w, cn, true);
    else
      limit_centre(a, b, gm1, w, cn, true);
    for (int c = 0; c < NV; ++c) out[8 * t + c] = w[c];
  } else if (kind == AF_LIM_SOURCE) {
    const double* q = in + 25 * t;
    double G[NV], S[NV], Sl[NV], A1[NV], er, ep;
    for (int c = 0; c < NV; ++c) {
      G[c] = q[c];
      S[c] = q[NV + c];
      Sl[c] = q[2 * NV + c];
    }
    const double th = source_step(G, S, Sl, q[3 * NV], gm1, A1, er, ep, cn, true);
    for (int c = 0; c < NV; ++c) out[9 * t + c] = A1[c];
    out[9 * t + NV] = th;
  } else {
    const double* q = in + 42 * t;
    double A1[NV], Lam[4];
    for (int c = 0; c < NV; ++c) A1[c] = q[c];
    const double* Hq = q + NV;
    auto H = [&](int I, int c) -> double { return Hq[NV * I + c]; };
    limiter_box<decltype(H), SHORTCUT>(A1, H, gm1, q[5 * NV], q[5 * NV + 1], Lam, cn, true);
    for (int I = 0; I < 4; ++I) out[4 * t + I] = Lam[I];
  }
}

}  // namespace

extern "C" int af_mhd_limiters_apply(int kind, int64_t n, double gamma, const double* in_dev, double* out_dev,
                                     uint32_t flags, af_mhd_counters_t* counts_dev, void* hip_stream) {
  if (kind < AF_LIM_POINT || kind > AF_LIM_BOX || n < 0 || !(gamma > 1.0) || (flags & ~AF_LIM_NO_SHORTCUT))
    return AF_EINVAL;
  if (n == 0) return AF_OK;
  if (!in_dev || !out_dev || !counts_dev || ((uintptr_t)in_dev & 7) || ((uintptr_t)out_dev & 7) ||
      ((uintptr_t)counts_dev & 7))
    return AF_EINVAL;
  const long blocks = (long)((n + LBLK - 1) / LBLK);
  if (blocks > 0x7fffffffL) return AF_EINVAL;
  (void)hipGetLastError();
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Counters* cn = reinterpret_cast<Counters*>(counts_dev);
  if (flags & AF_LIM_NO_SHORTCUT)
    k_limiters<false><<<(unsigned)blocks, LBLK, 0, s>>>(kind, (long)n, gamma - 1.0, in_dev, out_dev, cn);
  else
    k_limiters<true><<<(unsigned)blocks, LBLK, 0, s>>>(kind, (long)n, gamma - 1.0, in_dev, out_dev, cn);
  return hipGetLastError() == hipSuccess ? AF_OK : AF_EHIP;
}
