// Device helpers shared by the kernel sources: wavefront and workgroup
// reductions into the deterministic partial-sum layout, and the XCD-aware
// tile order of the marching kernels.
#ifndef RH_DEVICE_H
#define RH_DEVICE_H

#include <hip/hip_runtime.h>

#include "rh_internal.h"

namespace rh {

__device__ inline void cell_ijk(long long idx, int ny, int nz, int& i, int& j, int& k) {
  long long jk = idx % ((long long)ny * nz);
  i = (int)(idx / ((long long)ny * nz));
  j = (int)(jk / nz);
  k = (int)(jk % nz);
}

__device__ inline long long cell_index(int i, int j, int k, int ny, int nz) {
  return ((long long)i * ny + j) * nz + k;
}

// Block reductions over 256 threads (4 wavefronts of 64).
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
template <int NV, int NTH = kBlock>
__device__ inline void block_reduce_store(double (&vals)[NV], const int (&is_max)[NV],
                                          const int (&slot)[NV], double* part) {
  __shared__ double sh[NV][NTH / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double v = is_max[q] ? wave_max(vals[q]) : wave_sum(vals[q]);
    if (lane == 0) sh[q][wid] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double v = sh[q][0];
      for (int w = 1; w < NTH / 64; ++w) v = is_max[q] ? fmax(v, sh[q][w]) : v + sh[q][w];
      part[(long long)slot[q] * kPartCap + blockIdx.x] = v;
      if (blockIdx.x == 0) part[(long long)RS_COUNT * kPartCap + slot[q]] = (double)gridDim.x;
    }
  }
}

inline int red_grid(long long N) {
  long long g = (N + kBlock - 1) / kBlock;
  return (int)(g < kRedBlocks ? (g < 1 ? 1 : g) : kRedBlocks);
}

__device__ inline int pmod(int a, int m) { return ((a % m) + m) % m; }

// Neighbour q of cell c along axis d on side s (+1 / -1): false across a
// non-periodic wall, wrapped across a periodic one.
__device__ inline bool neighbour(const int (&c)[3], const int (&n)[3], const int* per, int d,
                                 int s, int (&q)[3]) {
  q[0] = c[0]; q[1] = c[1]; q[2] = c[2];
  int v = c[d] + s;
  if (v < 0) {
    if (!per[d]) return false;
    v += n[d];
  } else if (v >= n[d]) {
    if (!per[d]) return false;
    v -= n[d];
  }
  q[d] = v;
  return true;
}

// Level operators: the + face coefficient of cell i along axis d, and the
// diagonal of cell c (index i); FP32 levels form it from the packed record
// with op_diag, the same sum the marching kernels form from staged values.
__device__ inline double face_of(const LevelK<double>& l, int d, long long i) {
  return l.cf[d][i];
}
__device__ inline float face_of(const LevelK<float>& l, int d, long long i) {
  return bf16_value(l.op[i].f[d]);
}
__device__ inline double diag_of(const LevelK<double>& l, const int (&)[3], long long i) {
  return l.diag[i];
}
__device__ inline float diag_of(const LevelK<float>& l, const int (&c)[3], long long i) {
  const int n[3] = {l.nx, l.ny, l.nz};
  float f[6];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int q[3];
    f[2 * d] = neighbour(c, n, l.per, d, +1, q) ? face_of(l, d, i) : 0.0f;
    f[2 * d + 1] = neighbour(c, n, l.per, d, -1, q)
                       ? face_of(l, d, ((long long)q[0] * l.ny + q[1]) * l.nz + q[2])
                       : 0.0f;
  }
  return op_diag(bf16_value(l.op[i].s), f[0], f[1], f[2], f[3], f[4], f[5]);
}
// One row of a level's operator at cell c (index i): the off-diagonal sum
// sum_faces f x_neighbour in the order +x, -x, +y, -y, +z, -z (when want_off)
// and the diagonal.  FP32 levels read the cell's record once (one 8-byte
// load) and each - face once, for both.
__device__ inline void row_terms(const LevelK<double>& l, const int (&c)[3], long long i,
                                 bool want_off, double& off, double& diag) {
  const int n[3] = {l.nx, l.ny, l.nz};
  double s = 0.0;
  if (want_off) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int q[3];
      if (neighbour(c, n, l.per, d, +1, q))
        s += l.cf[d][i] * l.x[((long long)q[0] * l.ny + q[1]) * l.nz + q[2]];
      if (neighbour(c, n, l.per, d, -1, q)) {
        const long long Q = ((long long)q[0] * l.ny + q[1]) * l.nz + q[2];
        s += l.cf[d][Q] * l.x[Q];
      }
    }
  }
  off = s;
  diag = l.diag[i];
}
__device__ inline void row_terms(const LevelK<float>& l, const int (&c)[3], long long i,
                                 bool want_off, float& off, float& diag) {
  const int n[3] = {l.nx, l.ny, l.nz};
  const uint2 rec = reinterpret_cast<const uint2*>(l.op)[i];
  const float fp[3] = {__uint_as_float(rec.x << 16), __uint_as_float(rec.x & 0xFFFF0000u),
                       __uint_as_float(rec.y << 16)};
  float fm[3];
  float s = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int q[3];
    if (want_off && neighbour(c, n, l.per, d, +1, q))
      s += fp[d] * l.x[((long long)q[0] * l.ny + q[1]) * l.nz + q[2]];
    fm[d] = 0.0f;
    if (neighbour(c, n, l.per, d, -1, q)) {
      const long long Q = ((long long)q[0] * l.ny + q[1]) * l.nz + q[2];
      fm[d] = face_of(l, d, Q);
      if (want_off) s += fm[d] * l.x[Q];
    }
  }
  off = s;
  // a + face towards a non-periodic wall is stored as 0
  diag = op_diag(__uint_as_float(rec.y & 0xFFFF0000u), fp[0], fm[0], fp[1], fm[1], fp[2], fm[2]);
}
__device__ inline void put_face(const LevelK<double>& l, int d, long long i, double v) {
  l.cf[d][i] = v;
}
__device__ inline void put_face(const LevelK<float>& l, int d, long long i, double v) {
  l.op[i].f[d] = bf16_round((float)v);
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Give each XCD a contiguous range of tile indices, so tiles that share
// halo cache lines (neighbours along z come next in tile order) run on the
// same XCD at about the same time.  A bijection of [0, nb).
constexpr int kXcds = 8;
__device__ inline int xcd_tile(int bid, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int xcd = bid % kXcds, k = bid / kXcds;
  return xcd * q + min(xcd, r) + k;
}

}  // namespace rh

#endif  // RH_DEVICE_H
