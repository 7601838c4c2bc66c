// Memory-bandwidth probe: the realizable HBM bandwidth against which the
// solve's kernels are judged (Performance Measurements: kernels are rated
// against the bandwidth a STREAM triad achieves, and called roofline-bound
// above 70% of it).
//
// dst[i] = src[0][i] + s * sum_{k>=1} src[k][i], src = NIN contiguous arrays
// of n doubles. NIN = 1 is a copy, 2 the STREAM triad, 7 the read:write mix
// of the FP64 local Laplacian (u and six geometric factors in, A_L u out).
//
// Each lane handles two consecutive doubles per array (one 16-byte load per
// array, 1 KiB per wave instruction), all NIN loads issued before the sum,
// non-temporal like the Ax kernel's streams.
#include <hip/hip_runtime.h>

#include "sem_internal.h"

namespace sem {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));

template <int NIN>
__global__ __launch_bounds__(256) void k_stream(const double* __restrict__ src, double* __restrict__ dst, double s,
                                                int64_t n) {
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  if (i >= n) return;  // n is even: lanes below n own a full pair
  d2 v[NIN];
#pragma unroll
  for (int k = 0; k < NIN; ++k)
    v[k] = __builtin_nontemporal_load(reinterpret_cast<const d2*>(src + (int64_t)k * n + i));
  d2 acc = v[0];
  if (NIN > 1) {
    d2 t = v[1];
#pragma unroll
    for (int k = 2; k < NIN; ++k) t += v[k];
    acc += s * t;
  }
  __builtin_nontemporal_store(acc, reinterpret_cast<d2*>(dst + i));
}

template <int NIN>
void launch(const double* src, double* dst, double s, int64_t n, hipStream_t st) {
  const int64_t blocks = (n + 511) / 512;
  k_stream<NIN><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(src, dst, s, n);
}

}  // namespace
}  // namespace sem

using namespace sem;

extern "C" int sem_stream(int n_in, const double* src, double* dst, double s, int64_t n, void* stream) {
  return guarded([&] {
    if (n_in < 1 || n_in > 8) fail(SEM_EINVAL, "sem_stream: n_in = %d outside 1..8", n_in);
    if (n < 0 || (n & 1)) fail(SEM_EINVAL, "sem_stream: n = %lld must be even and >= 0", (long long)n);
    if (n == 0) return;
    if (!src || !dst) fail(SEM_EINVAL, "sem_stream: NULL pointer");
    if (((uintptr_t)src | (uintptr_t)dst) & 15) fail(SEM_EINVAL, "sem_stream: pointers must be 16-byte aligned");
    if ((n + 511) / 512 > 0x7fffffffLL) fail(SEM_EINVAL, "sem_stream: n too large for one launch");
    hipStream_t st = (hipStream_t)stream;
    switch (n_in) {
      case 1: launch<1>(src, dst, s, n, st); break;
      case 2: launch<2>(src, dst, s, n, st); break;
      case 3: launch<3>(src, dst, s, n, st); break;
      case 4: launch<4>(src, dst, s, n, st); break;
      case 5: launch<5>(src, dst, s, n, st); break;
      case 6: launch<6>(src, dst, s, n, st); break;
      case 7: launch<7>(src, dst, s, n, st); break;
      default: launch<8>(src, dst, s, n, st); break;
    }
    SEM_HIP(hipGetLastError());
  });
}
