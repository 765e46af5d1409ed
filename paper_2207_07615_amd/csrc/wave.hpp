// Wave64 helpers shared by the striped and single-workgroup kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace plss {

// 2- and 3-word vectors at 4-byte alignment (entry records of the striped
// stores)
typedef unsigned u32x2 __attribute__((ext_vector_type(2), aligned(4)));
typedef unsigned u32x3 __attribute__((ext_vector_type(3), aligned(4)));

// DPP controls of GFX9-family wave64 cross-lane moves
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143, kWaveShl1 = 0x130, kWaveShr1 = 0x138;

// v from another lane per the DPP control; lanes without a source (or outside
// row_mask) read 0
template <int CTRL, int RM, bool BC>
__device__ __forceinline__ int dpp32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, RM, 0xF, BC);
}
template <int CTRL, int RM, bool BC>
__device__ __forceinline__ float dppv(float v) {
  return __builtin_bit_cast(float, dpp32<CTRL, RM, BC>(__builtin_bit_cast(int, v)));
}
template <int CTRL, int RM, bool BC>
__device__ __forceinline__ double dppv(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp32<CTRL, RM, BC>((int)(b & 0xFFFFFFFFLL));
  const int hi = dpp32<CTRL, RM, BC>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane63(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ double lane63(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFLL), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes in a fixed order (inclusive scan by DPP shifts and
// row broadcasts, total taken from lane 63); the result is uniform.
template <class T>
__device__ __forceinline__ T wave_sum_dpp(T v) {
  v += dppv<kRowShr1, 0xF, true>(v);
  v += dppv<kRowShr2, 0xF, true>(v);
  v += dppv<kRowShr4, 0xF, true>(v);
  v += dppv<kRowShr8, 0xF, true>(v);
  v += dppv<kRowBcast15, 0xA, false>(v);
  v += dppv<kRowBcast31, 0xC, false>(v);
  return lane63(v);
}

// Loads through global-address-space pointers.  Arrays reached through a
// descriptor are generic pointers to the compiler, which would otherwise emit
// flat loads; those also count against the LDS wait counter.
template <class T>
__device__ __forceinline__ T gload(const T* p) {
  using GP = const __attribute__((address_space(1))) T*;
  return *(GP)p;
}
template <class T>
__device__ __forceinline__ T gload_nt(const T* p) {
  using GP = const __attribute__((address_space(1))) T*;
  return __builtin_nontemporal_load((GP)p);
}
__device__ __forceinline__ u32x2 gload_nt2(const unsigned* p) {
  using GP = const __attribute__((address_space(1))) u32x2*;
  return __builtin_nontemporal_load((GP)p);
}
__device__ __forceinline__ u32x3 gload_nt3(const unsigned* p) {
  using GP = const __attribute__((address_space(1))) u32x3*;
  return __builtin_nontemporal_load((GP)p);
}
// E consecutive elements of type T in one load (16 bytes at most; the
// address needs only T's alignment)
template <class T, int E> struct VecOf;
template <> struct VecOf<double, 1> { typedef double type; };
template <> struct VecOf<double, 2> { typedef double type __attribute__((ext_vector_type(2), aligned(8))); };
template <> struct VecOf<float, 1> { typedef float type; };
template <> struct VecOf<float, 2> { typedef float type __attribute__((ext_vector_type(2), aligned(4))); };
template <> struct VecOf<float, 4> { typedef float type __attribute__((ext_vector_type(4), aligned(4))); };
template <class T, int E>
__device__ __forceinline__ typename VecOf<T, E>::type gload_vec(const T* p) {
  using V = typename VecOf<T, E>::type;
  using GP = const __attribute__((address_space(1))) V*;
  return *(GP)p;
}
__device__ __forceinline__ double vec_elem(typename VecOf<double, 2>::type v, int i) { return v[i]; }
__device__ __forceinline__ float vec_elem(typename VecOf<float, 2>::type v, int i) { return v[i]; }
__device__ __forceinline__ float vec_elem(typename VecOf<float, 4>::type v, int i) { return v[i]; }
__device__ __forceinline__ double vec_elem(double v, int) { return v; }
__device__ __forceinline__ float vec_elem(float v, int) { return v; }
template <class T>
__device__ __forceinline__ void gstore(T* p, T v) {
  using GP = __attribute__((address_space(1))) T*;
  *(GP)p = v;
}

}  // namespace plss
