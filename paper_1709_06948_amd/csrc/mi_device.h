// mi_device.h -- device helpers shared by the kernels of libmi355.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mi.h"

namespace mi {

typedef unsigned __int128 u128;

// Load through the global address space (tables reached through pointers held
// in memory are otherwise generic, and generic loads also hold up LDS waits).
template <class T>
__device__ __forceinline__ T ldg(const T *p) {
  return *(const __attribute__((address_space(1))) T *)p;
}

// Raw buffer access: a 32-bit byte offset from a uniform base, checked by the
// hardware against the buffer's size (a read past it returns 0, a write past
// it is dropped).  Descriptor word 3 of a plain 32-bit raw buffer on gfx9.
typedef __amdgpu_buffer_rsrc_t brsrc;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ brsrc buf_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float buf_f32(brsrc r, uint32_t off, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
__device__ __forceinline__ uint32_t buf_u8(brsrc r, uint32_t off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}
__device__ __forceinline__ u32x2 buf_u32x2(brsrc r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
}
__device__ __forceinline__ void buf_store_u32x2(u32x2 v, brsrc r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
}

// Point-count feature (Sec. III-A, number of points in the voxel):
// bin = #{j : n >= e[j]} over nb-1 non-decreasing edges (binary search).
__device__ __forceinline__ int bin_count_dev(uint32_t n, int nb, const uint32_t *e) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (n >= e[mid - 1]) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// z-height variance feature (Sec. III-A, variance of z in the voxel) on the
// fixed-point heights q: empty -> 0, else 1 + #{j : n*S2 - S1^2 >= E[j]*n^2}
// over nb-2 non-decreasing edges, decided exactly in 128-bit integers.
// The search runs on r = D / n^2 in FP64 (relative error below 2^-50) against
// the edges as doubles (exact: edges stay below 2^53); only when an edge lies
// within a relative 2^-30 of r is the count redone with the exact comparison.
__device__ __forceinline__ int bin_zvar_exact(u128 D, u128 n2, int m, const uint64_t *E) {
  int lo = 0, hi = m;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (D >= (u128)E[mid - 1] * n2) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int bin_zvar_dev(uint32_t n, uint64_t s1, uint64_t s2, int nb,
                                            const uint64_t *E) {
  if (n == 0) return 0;
  const u128 D = (u128)n * (u128)s2 - (u128)s1 * (u128)s1;
  const double nd = (double)n;
  const double r = ((double)(uint64_t)(D >> 64) * 18446744073709551616.0 + (double)(uint64_t)D) /
                   (nd * nd);
  const int m = nb - 2;
  int lo = 0, hi = m;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (r >= (double)E[mid - 1]) lo = mid; else hi = mid - 1;
  }
  const double tol = 0x1p-30;
  const bool near_lo = lo > 0 && r - (double)E[lo - 1] <= tol * (double)E[lo - 1];
  const bool near_hi = lo < m && (double)E[lo] - r <= tol * (double)E[lo];
  if (near_lo || near_hi) lo = bin_zvar_exact(D, (u128)n * (u128)n, m, E);
  return 1 + lo;
}

// The same z-variance bin without a division: the search compares FP64
// D = n*S2 - S1^2 (relative error below 2^-51) against E[j] * n^2 (Ed holds the
// edges as doubles, exact below 2^53), and only when an edge product lies
// within a relative 2^-40 of D is the count redone with the exact 128-bit
// comparison.  Identical to bin_zvar_dev for every input.
__device__ __forceinline__ int bin_zvar_nodiv(uint32_t n, uint64_t s1, uint64_t s2, int nb,
                                              const double *Ed, const uint64_t *E) {
  if (n == 0) return 0;
  const u128 D = (u128)n * (u128)s2 - (u128)s1 * (u128)s1;
  const double Dd = (double)(uint64_t)(D >> 64) * 18446744073709551616.0 + (double)(uint64_t)D;
  const double nd = (double)n;
  const double n2 = nd * nd;
  const int m = nb - 2;
  int lo = 0, hi = m;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (Ed[mid - 1] * n2 <= Dd) lo = mid; else hi = mid - 1;
  }
  const double tol = 0x1p-40;
  bool near = false;
  if (lo > 0) {
    const double p = Ed[lo - 1] * n2;
    near = Dd - p <= tol * Dd;
  }
  if (lo < m) {
    const double p = Ed[lo] * n2;
    near = near || p - Dd <= tol * p;
  }
  if (near) lo = bin_zvar_exact(D, (u128)n * (u128)n, m, E);
  return 1 + lo;
}

// Value of the joint feature (MI_FEAT_JOINT) of an occupied voxel from its
// count bin bc (>= 1) and z-variance bin bz (>= 1) under nbz z-variance bins.
__device__ __forceinline__ int joint_value(int bc, int bz, int nbz) {
  return 1 + (bc - 1) * (nbz - 1) + (bz - 1);
}

// Bin of a voxel with n points and height sums s1, s2 under a feature kind;
// nbc / ce and nbz / ze are the grid's count and z-variance bins and edges.
__device__ __forceinline__ int feature_bin_dev(uint32_t kind, uint32_t n, uint64_t s1, uint64_t s2,
                                               int nbc, const uint32_t *ce, int nbz,
                                               const uint64_t *ze) {
  if (kind == MI_FEAT_COUNT) return bin_count_dev(n, nbc, ce);
  if (kind == MI_FEAT_ZVAR) return bin_zvar_dev(n, s1, s2, nbz, ze);
  if (n == 0) return 0;
  return joint_value(bin_count_dev(n, nbc, ce), bin_zvar_dev(n, s1, s2, nbz, ze), nbz);
}

// Entropy term -p ln p for a count c out of N (0 ln 0 = 0), Eqs. 3-5.
__device__ __forceinline__ double plogp_term(uint64_t c, double N) {
  if (c == 0) return 0.0;
  const double p = (double)c / N;
  return -p * log(p);
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Voxels of the table's bin in the box [x0, x1] x [y0, y1] x [z0, z1] of a
// table with (nx+1)(ny+1)(nz+1) entries of w bytes: the inclusion-exclusion of
// 8 entries, modulo 2^(8 w) like the entries (exact: the count lies in
// [0, 2^(8 w))).  Each entry is read as the aligned dword that holds it (an
// entry never straddles one, and the dword of the last entry lies within the
// table's 256-byte rounding) and shifted down; the bits above it drop out in
// the final mask, because the low 8 w bits of a sum or difference depend only
// on the operands' low 8 w bits.  The 8 loads are issued before any is used.
__device__ __forceinline__ uint32_t sat_box(const uint8_t *S, int w, int nx, int ny, int x0, int y0,
                                            int z0, int x1, int y1, int z1) {
  const int64_t sy = nx + 1, sz = (int64_t)(nx + 1) * (ny + 1);
  const int64_t X0 = x0, X1 = x1 + 1, Y0 = y0 * sy, Y1 = (y1 + 1) * sy, Z0 = z0 * sz,
                Z1 = (z1 + 1) * sz;
  // corners: + (X1 Y1 Z1), - (X0 Y1 Z1), - (X1 Y0 Z1), - (X1 Y1 Z0),
  //          + (X0 Y0 Z1), + (X0 Y1 Z0), + (X1 Y0 Z0), - (X0 Y0 Z0)
  const int64_t idx[8] = {X1 + Y1 + Z1, X0 + Y1 + Z1, X1 + Y0 + Z1, X1 + Y1 + Z0,
                          X0 + Y0 + Z1, X0 + Y1 + Z0, X1 + Y0 + Z0, X0 + Y0 + Z0};
  uint32_t e[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) e[k] = ldg((const uint32_t *)(S + ((idx[k] * w) & ~(int64_t)3)));
#pragma unroll
  for (int k = 0; k < 8; ++k) e[k] >>= 8 * (int)((idx[k] * w) & 3);
  const uint32_t v = e[0] - e[1] - e[2] - e[3] + e[4] + e[5] + e[6] - e[7];
  return w == 4 ? v : v & ((1u << (8 * w)) - 1u);
}

}  // namespace mi
