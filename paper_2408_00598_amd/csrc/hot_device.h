// Device helpers shared by the HIP kernels of libhot (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

namespace hot {

template <typename T>
struct VecT;
template <>
struct VecT<float> {
  static constexpr int W = 4;
  typedef float4 type;
  typedef float native __attribute__((ext_vector_type(4)));
};
template <>
struct VecT<double> {
  static constexpr int W = 2;
  typedef double2 type;
  typedef double native __attribute__((ext_vector_type(2)));
};

// Non-temporal 16-byte vector load: a pass reads each state element once
// (with several loads in flight per lane, plain loads left the slab pass at
// 5.25 TB/s on the 256-pair batch, non-temporal ones reach 5.47)
template <typename T>
__device__ inline typename VecT<T>::type vload_nt(const T* p) {
  const typename VecT<T>::native v =
      __builtin_nontemporal_load(reinterpret_cast<const typename VecT<T>::native*>(p));
  return __builtin_bit_cast(typename VecT<T>::type, v);
}

__device__ inline float vget(const float4& v, int e) {
  return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}
__device__ inline double vget(const double2& v, int e) { return e == 0 ? v.x : v.y; }
__device__ inline void vset(float4& v, int e, float x) {
  if (e == 0) v.x = x; else if (e == 1) v.y = x; else if (e == 2) v.z = x; else v.w = x;
}
__device__ inline void vset(double2& v, int e, double x) {
  if (e == 0) v.x = x; else v.y = x;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 256 threads of a block, fixed order; every thread gets it.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T>
__device__ inline T* pick(T* b0, T* b1, T* b2, int i) {
  return i == 0 ? b0 : (i == 1 ? b1 : b2);
}

}  // namespace hot
