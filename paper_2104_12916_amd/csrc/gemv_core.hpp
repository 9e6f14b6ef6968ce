// Device-side building blocks of the streaming matrix-vector kernels: wave and
// workgroup reductions, 16-byte row dot products against an LDS-staged vector,
// and the per-workgroup partial of a column sweep.
#pragma once
#include "common.hpp"

namespace qpg {

// ---------------------------------------------------------------------------
// wave-level helpers
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = v2d_t;
  static constexpr int n = 2;
};
template <>
struct Vec16<float> {
  using type = v4f_t;
  static constexpr int n = 4;
};

template <typename V, typename T>
__device__ __forceinline__ T dot16(const V& a, const T* x);
template <>
__device__ __forceinline__ double dot16<v2d_t, double>(const v2d_t& a, const double* x) {
  return a.x * x[0] + a.y * x[1];
}
template <>
__device__ __forceinline__ float dot16<v4f_t, float>(const v4f_t& a, const float* x) {
  return a.x * x[0] + a.y * x[1] + a.z * x[2] + a.w * x[3];
}

template <typename V, bool NT>
__device__ __forceinline__ V ld16(const V* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// Dot product of one matrix row (len elements, already rounded to whole
// 64-lane x 16-byte chunks, zeros past the true length) with x staged in LDS.
// Returns the full sum in every lane.
// NT: non-temporal matrix loads (streamed past the caches) or plain loads.
template <typename T, int U = 4, bool NT = true>
__device__ __forceinline__ T row_dot(const T* __restrict__ a, const T* xs, int lenR, int lane) {
  using V = typename Vec16<T>::type;
  constexpr int VE = Vec16<T>::n;
  constexpr int CH = kWave * VE;  // elements per wave-wide 16 B load
  T acc[4] = {0, 0, 0, 0};
  int j = lane * VE;
  const V* av = reinterpret_cast<const V*>(a);
  for (; j + (U - 1) * CH < lenR; j += U * CH) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = ld16<V, NT>(av + (j + u * CH) / VE);
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u % 4] += dot16<V, T>(v[u], xs + j + u * CH);
  }
  for (; j < lenR; j += CH) {
    V v0 = ld16<V, NT>(av + j / VE);
    acc[0] += dot16<V, T>(v0, xs + j);
  }
  return wave_sum<T>((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// Same dot product with x read from global memory (through the caches) as
// 16-byte vectors; elements of x at or past xlen read as zero.
template <typename T, int U = 4, bool NT = true>
__device__ __forceinline__ T row_dot_gx(const T* __restrict__ a, const T* __restrict__ x, int lenR, int xlen,
                                        int lane) {
  using V = typename Vec16<T>::type;
  constexpr int VE = Vec16<T>::n;
  constexpr int CH = kWave * VE;
  T acc[4] = {0, 0, 0, 0};
  int j = lane * VE;
  const V* av = reinterpret_cast<const V*>(a);
  auto xload = [&](int jj, T* t) {
    if (jj + VE <= xlen) {
      const V w = *reinterpret_cast<const V*>(x + jj);
      __builtin_memcpy(t, &w, sizeof(V));
    } else {
#pragma unroll
      for (int e = 0; e < VE; ++e) t[e] = (jj + e < xlen) ? x[jj + e] : T(0);
    }
  };
  for (; j + (U - 1) * CH < lenR; j += U * CH) {
    V v[U];
    T t[U][VE];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = ld16<V, NT>(av + (j + u * CH) / VE);
      xload(j + u * CH, t[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u % 4] += dot16<V, T>(v[u], t[u]);
  }
  for (; j < lenR; j += CH) {
    V v0 = ld16<V, NT>(av + j / VE);
    T t[VE];
    xload(j, t);
    acc[0] += dot16<V, T>(v0, t);
  }
  return wave_sum<T>((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// Two dot products of one matrix row with x1 and x2 (both read through the caches
// as 16-byte vectors, zero at or past xlen): the row is loaded once.  Full sums
// in every lane.
template <typename T, int U = 4, bool NT = true>
__device__ __forceinline__ void row_dot2_gx(const T* __restrict__ a, const T* __restrict__ x1,
                                            const T* __restrict__ x2, int lenR, int xlen, int lane, T& d1, T& d2) {
  using V = typename Vec16<T>::type;
  constexpr int VE = Vec16<T>::n;
  constexpr int CH = kWave * VE;
  T acc1[2] = {0, 0}, acc2[2] = {0, 0};
  int j = lane * VE;
  const V* av = reinterpret_cast<const V*>(a);
  auto xload = [&](const T* __restrict__ x, int jj, T* t) {
    if (jj + VE <= xlen) {
      const V w = *reinterpret_cast<const V*>(x + jj);
      __builtin_memcpy(t, &w, sizeof(V));
    } else {
#pragma unroll
      for (int e = 0; e < VE; ++e) t[e] = (jj + e < xlen) ? x[jj + e] : T(0);
    }
  };
  for (; j + (U - 1) * CH < lenR; j += U * CH) {
    V v[U];
    T t1[U][VE], t2[U][VE];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = ld16<V, NT>(av + (j + u * CH) / VE);
      xload(x1, j + u * CH, t1[u]);
      xload(x2, j + u * CH, t2[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc1[u % 2] += dot16<V, T>(v[u], t1[u]);
      acc2[u % 2] += dot16<V, T>(v[u], t2[u]);
    }
  }
  for (; j < lenR; j += CH) {
    V v0 = ld16<V, NT>(av + j / VE);
    T t1[VE], t2[VE];
    xload(x1, j, t1);
    xload(x2, j, t2);
    acc1[0] += dot16<V, T>(v0, t1);
    acc2[0] += dot16<V, T>(v0, t2);
  }
  d1 = wave_sum<T>(acc1[0] + acc1[1]);
  d2 = wave_sum<T>(acc2[0] + acc2[1]);
}

template <typename T>
__device__ __forceinline__ int round_chunk(int len, int ld) {
  constexpr int CH = kWave * Vec16<T>::n;
  int r = (len + CH - 1) / CH * CH;
  return r < ld ? r : ld;
}

// Stage x[0..len) into LDS, zero-filled up to lenR.
template <typename T>
__device__ __forceinline__ void stage_x(T* xs, const T* __restrict__ x, int len, int lenR) {
  for (int j = threadIdx.x; j < lenR; j += blockDim.x) xs[j] = (j < len) ? x[j] : T(0);
  __syncthreads();
}

// Per-workgroup partial of y_j = sum_i A_ij x_i over rows [r0, r1) for the
// column tile starting at c0 (64 lanes x 16 B).  The four waves of the block
// split the rows; the result for column c0 + jj is returned through LDS `red`.
// Shape kLower skips rows that lie entirely above the diagonal of the tile.
template <typename T, int U = 4>
__device__ __forceinline__ void cols_block_partial(const T* __restrict__ A, int lda, int r0, int r1, int c0, int shape,
                                                   const T* __restrict__ x, T (*red)[kWave * Vec16<T>::n]) {
  using V = typename Vec16<T>::type;
  constexpr int VE = Vec16<T>::n;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  T acc[VE];
#pragma unroll
  for (int e = 0; e < VE; ++e) acc[e] = 0;
  const int j = c0 + lane * VE;
  const int step = 4 * U;
  int i = r0 + wave * U;
  if (shape == kLower && r0 < c0) i += (c0 - r0) / step * step;
  for (; i < r1; i += step) {
    V a[U];
    T xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int ii = i + u;
      if (ii < r1) {
        a[u] = __builtin_nontemporal_load(reinterpret_cast<const V*>(A + (size_t)ii * lda + j));
        xv[u] = x[ii];
      } else {
        xv[u] = 0;
#pragma unroll
        for (int e = 0; e < VE; ++e) reinterpret_cast<T*>(&a[u])[e] = 0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int e = 0; e < VE; ++e) acc[e] += reinterpret_cast<const T*>(&a[u])[e] * xv[u];
    }
  }
#pragma unroll
  for (int e = 0; e < VE; ++e) red[wave][lane * VE + e] = acc[e];
  __syncthreads();
}

// Block-wide sum (and max) helpers for 256-thread blocks.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh /* >= 4 */) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum<T>(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  T s = 0;
  for (int w = 0; w < nw; ++w) s += sh[w];
  __syncthreads();
  return s;
}

// Two sums and a max over the block with one barrier pair; each value follows
// the same order as block_sum / block_max (wave butterfly, then waves in order).
__device__ __forceinline__ void block_sum2_max1(double& a, double& b, double& m, double (*sh)[16]) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  a = wave_sum<double>(a);
  b = wave_sum<double>(b);
  m = wave_max<double>(m);
  __syncthreads();
  if (lane == 0) {
    sh[0][wave] = a;
    sh[1][wave] = b;
    sh[2][wave] = m;
  }
  __syncthreads();
  double sa = 0, sb = 0, sm = sh[2][0];
  for (int w = 0; w < nw; ++w) {
    sa += sh[0][w];
    sb += sh[1][w];
  }
  for (int w = 1; w < nw; ++w) sm = fmax(sm, sh[2][w]);
  a = sa;
  b = sb;
  m = sm;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T* sh) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  v = wave_max<T>(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  T s = sh[0];
  for (int w = 1; w < nw; ++w) s = fmax(s, sh[w]);
  __syncthreads();
  return s;
}

}  // namespace qpg
