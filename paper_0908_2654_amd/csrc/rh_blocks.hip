// Source-centred block relaxation for the multigrid smoother.
//
// Around a point source the flux limiter makes the diffusion operator
// strongly anisotropic: faces across which E^n hardly changes (tangential
// to the source) take R = R_min and the largest coefficient D = c/R_min,
// faces along the steep radial fall-off take D ~ c r.  Shells of cells
// around each source are then tightly coupled among themselves and loosely
// to everything else; their near-constant modes are smooth for a point
// smoother but straddle the 2x2x2 cells of the coarse grids, so trilinear
// interpolation cannot carry them either.  Solving the Schur operator
// exactly on a small box around each source cell (block Gauss-Seidel on
// those boxes, in addition to the red-black sweeps) removes these modes.
//
// A level's boxes have one extent e_a = min(2R+1, n_a) per axis and never
// wrap: a box near a wall or a periodic seam is shifted inwards.  Boxes
// are coloured so that boxes of one colour neither overlap nor touch; one
// launch per colour updates all its boxes at once (each reads only x
// outside the other boxes of its colour).
#include <hip/hip_runtime.h>

#include "rh_device.h"
#include "rh_internal.h"

namespace rh {

// ---------------------------------------------------------------------------
// source cells, in cell order (two passes, no atomics: deterministic)
// ---------------------------------------------------------------------------
// Workgroup g scans cells [g chunk, (g+1) chunk) and stores its count.
__global__ void __launch_bounds__(kBlock)
k_src_count(long long N, long long chunk, const double* __restrict__ src, int* __restrict__ count) {
  const long long a = blockIdx.x * chunk;
  const long long b = a + chunk < N ? a + chunk : N;
  int c = 0;
  for (long long i = a + threadIdx.x; i < b; i += kBlock) c += src[i] > 0.0 ? 1 : 0;
  __shared__ int sh[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
    count[blockIdx.x] = t;
  }
}

// The same ranges again: each source cell goes to list[offset[g] + its rank
// among the sources of the range] (ranks by ballot within a wavefront and
// running totals across the workgroup's wavefronts).
__global__ void __launch_bounds__(kBlock)
k_src_list(long long N, long long chunk, const double* __restrict__ src,
           const int* __restrict__ offset, int* __restrict__ list) {
  const long long a = blockIdx.x * chunk;
  const long long b = a + chunk < N ? a + chunk : N;
  __shared__ int wc[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int base = offset[blockIdx.x];
  for (long long i0 = a; i0 < b; i0 += kBlock) {
    const long long i = i0 + threadIdx.x;
    const bool f = i < b && src[i] > 0.0;
    const unsigned long long m = __ballot(f);
    if (lane == 0) wc[wid] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      before += w < wid ? wc[w] : 0;
      total += wc[w];
    }
    if (f) list[base + before + __popcll(m & ((1ull << lane) - 1ull))] = (int)i;
    base += total;
    __syncthreads();
  }
}

void launch_src_count(hipStream_t s, long long N, long long chunk, int groups, const double* src,
                      int* count) {
  hipLaunchKernelGGL(k_src_count, dim3(groups), dim3(kBlock), 0, s, N, chunk, src, count);
}

void launch_src_list(hipStream_t s, long long N, long long chunk, int groups, const double* src,
                     const int* offset, int* list) {
  hipLaunchKernelGGL(k_src_list, dim3(groups), dim3(kBlock), 0, s, N, chunk, src, offset, list);
}

// ---------------------------------------------------------------------------
// box inverses (Gauss-Jordan in LDS, FP64; the box matrix is a principal
// submatrix of the symmetric positive definite Schur operator, so no
// pivoting is needed)
// ---------------------------------------------------------------------------
constexpr int kBlockThreads = 256;
static_assert(kBlockMaxCells <= 128, "one column per thread of a 128-wide row");

template <class T>
__global__ void __launch_bounds__(kBlockThreads)
k_block_inverse(LevelK<T> l, BlockSet<T> bs) {
  __shared__ double A[kBlockMaxCells * kBlockMaxCells];
  __shared__ double col[kBlockMaxCells], rowk[kBlockMaxCells];
  const int m = bs.m;
  const int blk = blockIdx.x;
  const int s0 = bs.start[3 * blk], s1 = bs.start[3 * blk + 1], s2 = bs.start[3 * blk + 2];
  for (int t = threadIdx.x; t < m * m; t += kBlockThreads) A[t] = 0.0;
  __syncthreads();
  // row of local cell p: diagonal and the couplings to the other box cells
  for (int p = threadIdx.x; p < m; p += kBlockThreads) {
    const int lx = p / (bs.ey * bs.ez), ly = (p / bs.ez) % bs.ey, lz = p % bs.ez;
    const int c[3] = {s0 + lx, s1 + ly, s2 + lz};
    const long long P = cell_index(c[0], c[1], c[2], l.ny, l.nz);
    A[p * m + p] = (double)l.diag[P];
    if (lx + 1 < bs.ex) A[p * m + p + bs.ey * bs.ez] = -(double)l.cf[0][P];
    if (lx > 0) A[p * m + p - bs.ey * bs.ez] = -(double)l.cf[0][P - (long long)l.ny * l.nz];
    if (ly + 1 < bs.ey) A[p * m + p + bs.ez] = -(double)l.cf[1][P];
    if (ly > 0) A[p * m + p - bs.ez] = -(double)l.cf[1][P - l.nz];
    if (lz + 1 < bs.ez) A[p * m + p + 1] = -(double)l.cf[2][P];
    if (lz > 0) A[p * m + p - 1] = -(double)l.cf[2][P - 1];
  }
  __syncthreads();
  // in-place Gauss-Jordan: step k divides row k by the pivot, puts 1/pivot
  // in its place and eliminates column k from the other rows (which take
  // -a_ik / pivot in column k); column k and row k are staged first, so
  // every update reads values of the previous step
  for (int k = 0; k < m; ++k) {
    for (int i = threadIdx.x; i < m; i += kBlockThreads) {
      col[i] = A[i * m + k];
      rowk[i] = i == k ? 1.0 : A[k * m + i];
    }
    __syncthreads();
    const double inv_piv = 1.0 / col[k];
    // thread: column j = tid mod 128, rows tid / 128, + 2, + 4, ... (a
    // wavefront shares its row: col[i] is a broadcast, rowk[j] contiguous)
    const int j = threadIdx.x & 127;
    if (j < m) {
      const double rj = rowk[j] * inv_piv;
      for (int i = threadIdx.x >> 7; i < m; i += kBlockThreads / 128) {
        double* a = &A[i * m + j];
        if (i == k)
          *a = rj;
        else
          *a = (j == k ? 0.0 : *a) - col[i] * rj;
      }
    }
    __syncthreads();
  }
  T* out = bs.inv + (long long)blk * m * m;
  for (int t = threadIdx.x; t < m * m; t += kBlockThreads) out[t] = (T)A[t];
}

template <class T>
void launch_block_inverse(hipStream_t s, const LevelK<T>& l, const BlockSet<T>& bs) {
  if (bs.n == 0) return;
  hipLaunchKernelGGL((k_block_inverse<T>), dim3(bs.n), dim3(kBlockThreads), 0, s, l, bs);
}

// ---------------------------------------------------------------------------
// relaxation on the boxes [b0, b0 + nb) (one colour): x_box += A_box^-1 r_box
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(128) k_block_relax(LevelK<T> l, BlockSet<T> bs, int b0) {
  __shared__ T r[kBlockMaxCells];
  const int m = bs.m;
  const int blk = b0 + blockIdx.x;
  const int s0 = bs.start[3 * blk], s1 = bs.start[3 * blk + 1], s2 = bs.start[3 * blk + 2];
  const int n[3] = {l.nx, l.ny, l.nz};
  const int p = threadIdx.x;
  long long P = -1;
  if (p < m) {
    const int c[3] = {s0 + p / (bs.ey * bs.ez), s1 + (p / bs.ez) % bs.ey, s2 + p % bs.ez};
    P = cell_index(c[0], c[1], c[2], l.ny, l.nz);
    T off = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int q[3];
      if (neighbour(c, n, l.per, d, +1, q))
        off += l.cf[d][P] * l.x[cell_index(q[0], q[1], q[2], l.ny, l.nz)];
      if (neighbour(c, n, l.per, d, -1, q)) {
        const long long Q = cell_index(q[0], q[1], q[2], l.ny, l.nz);
        off += l.cf[d][Q] * l.x[Q];
      }
    }
    r[p] = l.b[P] - (l.diag[P] * l.x[P] - off);
  }
  __syncthreads();
  if (p < m) {
    // the inverse is symmetric: column j is contiguous, read across threads
    const T* inv = bs.inv + (long long)blk * m * m;
    T dx = 0;
    for (int j = 0; j < m; ++j) dx += inv[(long long)j * m + p] * r[j];
    l.x[P] += dx;
  }
}

template <class T>
void launch_block_relax(hipStream_t s, const LevelK<T>& l, const BlockSet<T>& bs, int b0, int nb) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_block_relax<T>), dim3(nb), dim3(128), 0, s, l, bs, b0);
}

template void launch_block_inverse<float>(hipStream_t, const LevelK<float>&, const BlockSet<float>&);
template void launch_block_inverse<double>(hipStream_t, const LevelK<double>&,
                                           const BlockSet<double>&);
template void launch_block_relax<float>(hipStream_t, const LevelK<float>&, const BlockSet<float>&,
                                        int, int);
template void launch_block_relax<double>(hipStream_t, const LevelK<double>&,
                                         const BlockSet<double>&, int, int);

}  // namespace rh
