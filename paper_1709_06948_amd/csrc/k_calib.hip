// k_calib.hip -- microbenchmarks of the rooflines the evaluator is held
// against: LDS 32- and 64-bit atomic add, LDS compare-and-swap, HBM stream
// read and FP64 VALU issue.  Each kernel does a known number of operations in
// a known pattern; the caller times it (HIP events) and divides.  The results
// are written to a device buffer so that no work is optimised away.
#include <algorithm>

#include <algorithm>

#include "mi_device.h"
#include "mi_internal.h"

#pragma clang fp contract(off)

namespace mi {

constexpr int kCalibLds = 16384;  // u32 words of LDS per workgroup (64 KiB)

// Every lane adds to its own bank-distinct word (lane + 64 * wave, wrapping):
// conflict-free LDS atomic traffic.  iters rounds of 8 atomics per lane.
__global__ void __launch_bounds__(1024) k_calib_lds_u32(uint32_t *out, int iters) {
  __shared__ uint32_t w[kCalibLds];
  for (int i = threadIdx.x; i < kCalibLds; i += blockDim.x) w[i] = 0u;
  __syncthreads();
  const int base = threadIdx.x & (kCalibLds - 1);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) atomicAdd(&w[(base + j * 1024) & (kCalibLds - 1)], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = w[0];
}

__global__ void __launch_bounds__(1024) k_calib_lds_u64(unsigned long long *out, int iters) {
  __shared__ unsigned long long w[kCalibLds / 2];
  for (int i = threadIdx.x; i < kCalibLds / 2; i += blockDim.x) w[i] = 0ull;
  __syncthreads();
  const int base = threadIdx.x & (kCalibLds / 2 - 1);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) atomicAdd(&w[(base + j * 1024) & (kCalibLds / 2 - 1)], 1ull);
  }
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = w[0];
}

// Compare-and-swap that always succeeds (each lane swaps its own word from the
// value it last wrote), returning the old value like the hash's claim does.
__global__ void __launch_bounds__(1024) k_calib_lds_cas(uint32_t *out, int iters) {
  __shared__ uint32_t w[kCalibLds];
  for (int i = threadIdx.x; i < kCalibLds; i += blockDim.x) w[i] = 0u;
  __syncthreads();
  const int base = threadIdx.x & (kCalibLds - 1);
  uint32_t v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = 0u;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t old = atomicCAS(&w[(base + j * 1024) & (kCalibLds - 1)], v[j], v[j] + 1u);
      v[j] = old + 1u;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = w[0] + v[0];
}

// Stream read of n 16-byte words, grid-strided, with a reduction kept live.
__global__ void __launch_bounds__(256) k_calib_hbm_read(const uint4 *__restrict__ p, int64_t n,
                                                        uint32_t *out) {
  uint32_t acc = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint4 v = p[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9e3779b9u) out[0] = acc;  // practically never: keeps the loads
}

// FP64 VALU issue: 8 independent chains of dependent multiply-adds written as
// separate multiply and add (no contraction), iters rounds of 16 FP64 ops.
__global__ void __launch_bounds__(256) k_calib_fp64(double *out, int iters, double a, double b) {
  double x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = (double)(threadIdx.x + j);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = x[j] * a + b;
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += x[j];
  if (s == 1.2345) out[0] = s;  // practically never: keeps the arithmetic
}

}  // namespace mi

using namespace mi;

// kind: 0 LDS u32 add, 1 LDS u64 add, 2 LDS CAS, 3 HBM read, 4 FP64 VALU.
// Returns the operations (lane operations or bytes) the launch performs in
// *ops, and launches it on `stream`; the caller times the launch.
extern "C" mi_status mi_calibrate_launch(int32_t kind, int64_t size, void *scratch,
                                         int64_t scratch_bytes, void *stream, double *ops) {
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return MI_E_DEVICE;
  if (!ops || size <= 0 || !scratch) return MI_E_INVALID;
  const int iters = (int)std::min<int64_t>(size, 1 << 20);
  const unsigned blocks = (unsigned)(cus * 2);
  switch (kind) {
    case 0:
      if (scratch_bytes < (int64_t)blocks * 4) return MI_E_WORKSPACE;
      k_calib_lds_u32<<<blocks, 1024, 0, s>>>((uint32_t *)scratch, iters);
      *ops = (double)blocks * 1024.0 * 8.0 * iters;
      break;
    case 1:
      if (scratch_bytes < (int64_t)blocks * 8) return MI_E_WORKSPACE;
      k_calib_lds_u64<<<blocks, 1024, 0, s>>>((unsigned long long *)scratch, iters);
      *ops = (double)blocks * 1024.0 * 8.0 * iters;
      break;
    case 2:
      if (scratch_bytes < (int64_t)blocks * 4) return MI_E_WORKSPACE;
      k_calib_lds_cas<<<blocks, 1024, 0, s>>>((uint32_t *)scratch, iters);
      *ops = (double)blocks * 1024.0 * 8.0 * iters;
      break;
    case 3: {
      const int64_t n = scratch_bytes / 16 - 1;  // the last word holds the result
      if (n < 1024) return MI_E_WORKSPACE;
      k_calib_hbm_read<<<(unsigned)(cus * 8), 256, 0, s>>>((const uint4 *)scratch, n,
                                                          (uint32_t *)((uint4 *)scratch + n));
      *ops = (double)n * 16.0;
      break;
    }
    case 4:
      if (scratch_bytes < 8) return MI_E_WORKSPACE;
      k_calib_fp64<<<(unsigned)(cus * 16), 256, 0, s>>>((double *)scratch, iters, 0.999999, 1e-7);
      *ops = (double)cus * 16.0 * 256.0 * 16.0 * iters;
      break;
    default:
      return MI_E_INVALID;
  }
  return hipGetLastError() == hipSuccess ? MI_OK : MI_E_DEVICE;
}
