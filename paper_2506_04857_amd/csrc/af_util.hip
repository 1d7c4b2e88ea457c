// af_util.hip -- a plain device-to-device stream copy, the measurement aid
// against which the stage kernels' HBM bandwidth is compared (the attainable
// copy bandwidth of the device, next to its 8 TB/s specification).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "af_mhd.h"

namespace {

constexpr int CBLK = 256;

// One 16-byte element per thread over a grid that covers the buffer: the
// fastest of the shapes measured on MI355X (6.2 TB/s on 1 GiB, against
// 4.2-5.2 TB/s for grid-stride loops with 4-16 loads in flight per thread).
__global__ __launch_bounds__(CBLK) void k_stream_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                      long n16) {
  const long q = (long)blockIdx.x * CBLK + threadIdx.x;
  if (q < n16) dst[q] = src[q];
}

}  // namespace

extern "C" int af_mhd_stream_copy(const double* src, double* dst, size_t n, void* hip_stream) {
  if (!src || !dst || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15) || (n & 1)) return AF_EINVAL;
  const long n16 = (long)(n / 2);
  if (n16 == 0) return AF_OK;
  const long blocks = (n16 + CBLK - 1) / CBLK;
  if (blocks > 0x7fffffffL) return AF_EINVAL;
  (void)hipGetLastError();
  k_stream_copy<<<(unsigned)blocks, CBLK, 0, static_cast<hipStream_t>(hip_stream)>>>(
      reinterpret_cast<const double2*>(src), reinterpret_cast<double2*>(dst), n16);
  return hipGetLastError() == hipSuccess ? AF_OK : AF_EHIP;
}
