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
// box inverses (Gauss-Jordan in FP64; the box matrix is a principal
// submatrix of the symmetric positive definite Schur operator, so no
// pivoting is needed)
// ---------------------------------------------------------------------------
// The 128 x 128 padded matrix is spread over a 16 x 16 grid of threads:
// thread (r, c) keeps the 64 entries (r + 16 a, c + 16 b), a, b < 8, in
// registers; a pivot step exchanges only row k and column k through LDS.
constexpr int kBlockThreads = 256;
constexpr int kInvTile = 16;                    // thread grid side
constexpr int kInvPer = 128 / kInvTile;         // rows (columns) per thread
static_assert(kBlockMaxCells <= 128, "boxes fit the 128 x 128 register tile");
static_assert(kInvTile * kInvTile == kBlockThreads, "one thread per tile position");

template <class T>
__global__ void __launch_bounds__(kBlockThreads)
k_block_inverse(LevelK<T> l, BlockSet<T> bs) {
  // the box's 7-point rows: diagonal and the six couplings (0 outside the box)
  __shared__ double coef[kBlockMaxCells][7];
  __shared__ double rowk[128], colk[128];
  const int m = bs.m;
  const int blk = blockIdx.x;
  const int s0 = bs.start[3 * blk], s1 = bs.start[3 * blk + 1], s2 = bs.start[3 * blk + 2];
  const int exy = bs.ey * bs.ez;
  for (int p = threadIdx.x; p < m; p += kBlockThreads) {
    const int lx = p / exy, ly = (p / bs.ez) % bs.ey, lz = p % bs.ez;
    const int cc[3] = {s0 + lx, s1 + ly, s2 + lz};
    const long long P = cell_index(cc[0], cc[1], cc[2], l.ny, l.nz);
    coef[p][0] = (double)diag_of(l, cc, P);
    coef[p][1] = lx + 1 < bs.ex ? -(double)face_of(l, 0, P) : 0.0;
    coef[p][2] = lx > 0 ? -(double)face_of(l, 0, P - (long long)l.ny * l.nz) : 0.0;
    coef[p][3] = ly + 1 < bs.ey ? -(double)face_of(l, 1, P) : 0.0;
    coef[p][4] = ly > 0 ? -(double)face_of(l, 1, P - l.nz) : 0.0;
    coef[p][5] = lz + 1 < bs.ez ? -(double)face_of(l, 2, P) : 0.0;
    coef[p][6] = lz > 0 ? -(double)face_of(l, 2, P - 1) : 0.0;
  }
  __syncthreads();
  const int r = threadIdx.x / kInvTile, c = threadIdx.x % kInvTile;
  // entries; rows and columns past m form an identity block (never coupled)
  double A[kInvPer][kInvPer];
#pragma unroll
  for (int a = 0; a < kInvPer; ++a) {
    const int i = r + kInvTile * a;
#pragma unroll
    for (int b = 0; b < kInvPer; ++b) {
      const int j = c + kInvTile * b;
      double v = 0.0;
      if (i >= m || j >= m) {
        v = i == j ? 1.0 : 0.0;
      } else {
        const int d = j - i;
        if (d == 0) v = coef[i][0];
        else if (d == exy) v = coef[i][1];
        else if (d == -exy) v = coef[i][2];
        else if (d == bs.ez) v = coef[i][3];
        else if (d == -bs.ez) v = coef[i][4];
        else if (d == 1) v = coef[i][5];
        else if (d == -1) v = coef[i][6];
      }
      A[a][b] = v;
    }
  }
  // in-place Gauss-Jordan: step k divides row k by the pivot, puts 1/pivot
  // in its place and eliminates column k from the other rows (which take
  // -a_ik / pivot in column k); row k and column k of the previous step are
  // staged in LDS first
  for (int k = 0; k < m; ++k) {
    const int kr = k % kInvTile, ka = k / kInvTile;
    // row k and column k to LDS (register indices stay compile-time constants)
#pragma unroll
    for (int a = 0; a < kInvPer; ++a)
      if (a == ka && r == kr) {
#pragma unroll
        for (int b = 0; b < kInvPer; ++b) rowk[c + kInvTile * b] = A[a][b];
      }
#pragma unroll
    for (int b = 0; b < kInvPer; ++b)
      if (b == ka && c == kr) {
#pragma unroll
        for (int a = 0; a < kInvPer; ++a) colk[r + kInvTile * a] = A[a][b];
      }
    __syncthreads();
    const double inv_piv = 1.0 / colk[k];
    double ci[kInvPer], rj[kInvPer];
#pragma unroll
    for (int a = 0; a < kInvPer; ++a) ci[a] = colk[r + kInvTile * a];
#pragma unroll
    for (int b = 0; b < kInvPer; ++b) rj[b] = rowk[c + kInvTile * b] * inv_piv;
#pragma unroll
    for (int a = 0; a < kInvPer; ++a) {
      const bool rowk_here = r == kr && a == ka;
#pragma unroll
      for (int b = 0; b < kInvPer; ++b) {
        const bool colk_here = c == kr && b == ka;
        double v;
        if (rowk_here)
          v = colk_here ? inv_piv : rj[b];
        else
          v = (colk_here ? 0.0 : A[a][b]) - ci[a] * (colk_here ? inv_piv : rj[b]);
        A[a][b] = v;
      }
    }
    __syncthreads();
  }
  T* out = bs.inv + (long long)blk * m * m;
#pragma unroll
  for (int a = 0; a < kInvPer; ++a) {
    const int i = r + kInvTile * a;
#pragma unroll
    for (int b = 0; b < kInvPer; ++b) {
      const int j = c + kInvTile * b;
      if (i < m && j < m) out[i * m + j] = (T)A[a][b];
    }
  }
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
  const int p = threadIdx.x;
  long long P = -1;
  if (p < m) {
    const int c[3] = {s0 + p / (bs.ey * bs.ez), s1 + (p / bs.ez) % bs.ey, s2 + p % bs.ez};
    P = cell_index(c[0], c[1], c[2], l.ny, l.nz);
    T off, dg;
    row_terms(l, c, P, true, off, dg);
    r[p] = l.b[P] - (dg * l.x[P] - off);
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
