// Advection of the implicit step's fields by a prescribed velocity field:
// the part of the operator split's hydrodynamic step that moves the number
// densities and the radiation energy (Algorithm section, step (iv);
// equations enzo-chemical_ionization and enzo-cons_radiation,
// d_t q + (1/a) div(q v) = 0), before the implicit step starts from the
// advected values.
//
// Conserved per cell: n_H, E, n_HI and n_H e (e is energy per unit mass, so
// the gas energy density is m_H n_H e); e is recovered as (n_H e) / n_H.
// Velocities are cell-centred (proper peculiar, cm/s); a face takes the mean
// of its two cells, 0 at a zero-flux wall, and the boundary cell's own value
// at an outflow wall, where the ghost cell repeats the boundary cell.
// First-order donor-cell fluxes, unsplit: through a face with Courant number
// u the flux is u q_lower for u > 0 and u q_upper otherwise, and a cell
// changes by (flux in) - (flux out), axis by axis (x, y, z), each axis as
// q -= F_upper - F_lower.  One launch is one substep; the host picks the
// substep count from the largest outgoing Courant number.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rh_device.h"
#include "rh_internal.h"

namespace rh {

namespace {

__device__ inline int adv_wrap(int g, int n, int per) {
  if (g >= 0 && g < n) return g;
  if (!per) return -1;
  return g < 0 ? g + n : g - n;
}

// Courant numbers of a cell's lower and upper face along one axis.
// vP: the cell's velocity; vD, vU: the lower / upper neighbour's (used only
// when that neighbour exists); bcD, bcU: the wall types.
__device__ inline void face_courant(double vP, double vD, double vU, bool hasD, bool hasU,
                                    int bcD, int bcU, double scale, double& ud, double& uu) {
  ud = hasD ? (0.5 * (vD + vP)) * scale : (bcD == RH_BC_OUTFLOW ? vP * scale : 0.0);
  uu = hasU ? (0.5 * (vP + vU)) * scale : (bcU == RH_BC_OUTFLOW ? vP * scale : 0.0);
}

// q -= F_upper - F_lower for one axis (donor-cell fluxes; a missing
// neighbour's values are the cell's own).
template <int NQ>
__device__ inline void donor_axis(double (&out)[NQ], const double (&qP)[NQ],
                                  const double (&qD)[NQ], const double (&qU)[NQ], double ud,
                                  double uu) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double Fu = uu > 0.0 ? uu * qP[q] : uu * qU[q];
    const double Fd = ud > 0.0 ? ud * qD[q] : ud * qP[q];
    out[q] -= Fu - Fd;
  }
}

template <int NQ>
__device__ inline void load_q(const AdvK& a, long long P, double (&q)[NQ]) {
  q[0] = a.qi[0][P];
  q[1] = a.qi[1][P];
  q[2] = a.qi[2][P];
  if constexpr (NQ == 4) q[3] = q[0] * a.qi[3][P];
}

template <int NQ>
__device__ inline void store_q(const AdvK& a, long long P, const double (&q)[NQ]) {
  a.qo[0][P] = q[0];
  a.qo[1][P] = q[1];
  a.qo[2][P] = q[2];
  if constexpr (NQ == 4) a.qo[3][P] = q[3] / q[0];
}

}  // namespace

// Largest outgoing Courant number of a cell (sum over its six faces of the
// parts of u pointing out of it), and a flag for non-finite velocities.
__global__ void __launch_bounds__(kBlock) k_advect_courant(AdvK a, double* __restrict__ part) {
  const int per[3] = {a.bc[0] == RH_BC_PERIODIC, a.bc[2] == RH_BC_PERIODIC,
                      a.bc[4] == RH_BC_PERIODIC};
  const int n[3] = {a.nx, a.ny, a.nz};
  double cmax = 0.0, bad = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < a.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, a.ny, a.nz, c[0], c[1], c[2]);
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double vP = a.v[d][idx];
      if (!isfinite(vP)) bad = 1.0;
      const int gd = adv_wrap(c[d] - 1, n[d], per[d]), gu = adv_wrap(c[d] + 1, n[d], per[d]);
      int cd[3] = {c[0], c[1], c[2]}, cu[3] = {c[0], c[1], c[2]};
      cd[d] = gd;
      cu[d] = gu;
      const double vD = gd >= 0 ? a.v[d][cell_index(cd[0], cd[1], cd[2], a.ny, a.nz)] : 0.0;
      const double vU = gu >= 0 ? a.v[d][cell_index(cu[0], cu[1], cu[2], a.ny, a.nz)] : 0.0;
      double ud, uu;
      face_courant(vP, vD, vU, gd >= 0, gu >= 0, a.bc[2 * d], a.bc[2 * d + 1], a.scale, ud, uu);
      s += fmax(uu, 0.0) + fmax(-ud, 0.0);
    }
    cmax = fmax(cmax, s);
  }
  double v[2] = {cmax, bad};
  const int im[2] = {1, 1};
  const int sl[2] = {RS_COURANT, RS_NONFINITE};
  block_reduce_store<2>(v, im, sl, part);
}

// The same reduction marching along x in the tiles of k_advect_march: each
// velocity is read once per block (plus the tile's ring), the y and z
// components of the current plane from LDS.
constexpr int kCouTY = 8, kCouTZ = 64, kCouXC = 32;

__global__ void __launch_bounds__(kBlock) k_advect_courant_march(AdvK a, int xc,
                                                                double* __restrict__ part) {
  constexpr int TY = kCouTY, TZ = kCouTZ, HZ = TZ + 2, PL = (TY + 2) * HZ;
  constexpr int NR = TY / (kBlock / 64);
  constexpr int NRING = 2 * TZ + 2 * TY;
  static_assert(TZ == 64 && NRING <= kBlock, "one wave per row, one ring cell per thread");
  __shared__ double svy[2][PL], svz[2][PL];
  const int per[3] = {a.bc[0] == RH_BC_PERIODIC, a.bc[2] == RH_BC_PERIODIC,
                      a.bc[4] == RH_BC_PERIODIC};
  const int ntz = (a.nz + TZ - 1) / TZ, nty = (a.ny + TY - 1) / TY;
  int bid = xcd_tile(blockIdx.x, gridDim.x);
  const int tz = bid % ntz;
  bid /= ntz;
  const int ty = bid % nty;
  const int cx = bid / nty;
  const int ya = ty * TY, za = tz * TZ;
  const int xa = cx * xc, xb = min(xa + xc, a.nx);
  const long long plane = (long long)a.ny * a.nz;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  auto off2 = [&](int gy, int gz) -> int {
    const int wy = adv_wrap(gy, a.ny, per[1]), wz = adv_wrap(gz, a.nz, per[2]);
    return (wy >= 0 && wz >= 0) ? wy * a.nz + wz : -1;
  };
  int own[NR], li[NR];
  bool real[NR], hym[NR], hyp[NR], hzm[NR], hzp[NR];
#pragma unroll
  for (int m = 0; m < NR; ++m) {
    const int ly = wid + (kBlock / 64) * m, gy = ya + ly, gz = za + lane;
    real[m] = gy < a.ny && gz < a.nz;
    own[m] = off2(gy, gz);
    hym[m] = off2(gy - 1, gz) >= 0;
    hyp[m] = off2(gy + 1, gz) >= 0;
    hzm[m] = off2(gy, gz - 1) >= 0;
    hzp[m] = off2(gy, gz + 1) >= 0;
    li[m] = (ly + 1) * HZ + lane + 1;
  }
  int r_off = -1, r_li = -1, r_axis = 1;
  if (threadIdx.x < NRING) {
    const int e = threadIdx.x;
    int ly, lz;
    if (e < 2 * TZ) {
      ly = e < TZ ? 0 : TY + 1;
      lz = e % TZ + 1;
    } else {
      const int f = e - 2 * TZ;
      ly = f % TY + 1;
      lz = f < TY ? 0 : TZ + 1;
      r_axis = 2;
    }
    r_li = ly * HZ + lz;
    r_off = off2(ya + ly - 1, za + lz - 1);
  }
  auto fetch = [&](int p, int off, int d) -> double {
    const int gx = adv_wrap(p, a.nx, per[0]);
    return (gx >= 0 && off >= 0) ? a.v[d][gx * plane + off] : 0.0;
  };
  double vxm[NR], vxc[NR], vxn[NR], vyn[NR], vzn[NR], vxo[NR], vyo[NR], vzo[NR];
  double ring1 = 0.0, ring2 = 0.0;
  {
    const int b0 = xa & 1;
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      vxm[m] = fetch(xa - 1, own[m], 0);
      vxc[m] = fetch(xa, own[m], 0);
      svy[b0][li[m]] = fetch(xa, own[m], 1);
      svz[b0][li[m]] = fetch(xa, own[m], 2);
      vxn[m] = fetch(xa + 1, own[m], 0);
      vyn[m] = fetch(xa + 1, own[m], 1);
      vzn[m] = fetch(xa + 1, own[m], 2);
    }
    if (r_li >= 0) {
      const double v0 = fetch(xa, r_off, r_axis);
      if (r_axis == 1) svy[b0][r_li] = v0; else svz[b0][r_li] = v0;
      ring1 = fetch(xa + 1, r_off, r_axis);
    }
  }
  __syncthreads();
  double cmax = 0.0, bad = 0.0;
  for (int x = xa; x < xb; ++x) {
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      if (x + 2 <= xb) {
        vxo[m] = fetch(x + 2, own[m], 0);
        vyo[m] = fetch(x + 2, own[m], 1);
        vzo[m] = fetch(x + 2, own[m], 2);
      }
    }
    if (r_li >= 0 && x + 2 < xb) ring2 = fetch(x + 2, r_off, r_axis);
    const int b = x & 1;
    const bool hxm = adv_wrap(x - 1, a.nx, per[0]) >= 0;
    const bool hxp = adv_wrap(x + 1, a.nx, per[0]) >= 0;
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      if (!real[m]) continue;
      const int t = li[m];
      const double vy = svy[b][t], vz = svz[b][t];
      if (!isfinite(vxc[m]) || !isfinite(vy) || !isfinite(vz)) bad = 1.0;
      double ud, uu, sc = 0.0;
      face_courant(vxc[m], vxm[m], vxn[m], hxm, hxp, a.bc[0], a.bc[1], a.scale, ud, uu);
      sc += fmax(uu, 0.0) + fmax(-ud, 0.0);
      face_courant(vy, svy[b][t - HZ], svy[b][t + HZ], hym[m], hyp[m], a.bc[2], a.bc[3],
                   a.scale, ud, uu);
      sc += fmax(uu, 0.0) + fmax(-ud, 0.0);
      face_courant(vz, svz[b][t - 1], svz[b][t + 1], hzm[m], hzp[m], a.bc[4], a.bc[5], a.scale,
                   ud, uu);
      sc += fmax(uu, 0.0) + fmax(-ud, 0.0);
      cmax = fmax(cmax, sc);
    }
    if (x + 1 < xb) {
      const int b1 = b ^ 1;
#pragma unroll
      for (int m = 0; m < NR; ++m) {
        svy[b1][li[m]] = vyn[m];
        svz[b1][li[m]] = vzn[m];
      }
      if (r_li >= 0) {
        if (r_axis == 1) svy[b1][r_li] = ring1; else svz[b1][r_li] = ring1;
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      vxm[m] = vxc[m];
      vxc[m] = vxn[m];
      if (x + 2 <= xb) {
        vxn[m] = vxo[m];
        vyn[m] = vyo[m];
        vzn[m] = vzo[m];
      }
    }
    ring1 = ring2;
  }
  double v[2] = {cmax, bad};
  const int im[2] = {1, 1};
  const int sl[2] = {RS_COURANT, RS_NONFINITE};
  block_reduce_store<2>(v, im, sl, part);
}

void launch_advect_courant(hipStream_t s, const AdvK& a, double* part) {
  const int nty = (a.ny + kCouTY - 1) / kCouTY, ntz = (a.nz + kCouTZ - 1) / kCouTZ;
  const long long tiles = (long long)nty * ntz;
  if (a.nz >= kCouTZ && a.ny >= kCouTY && a.nx >= 2) {
    int ncx = (a.nx + kCouXC - 1) / kCouXC;
    const int xc = (a.nx + ncx - 1) / ncx;
    ncx = (a.nx + xc - 1) / xc;
    if (tiles * ncx <= kPartCap) {
      hipLaunchKernelGGL(k_advect_courant_march, dim3((unsigned)(tiles * ncx)), dim3(kBlock), 0,
                         s, a, xc, part);
      return;
    }
  }
  hipLaunchKernelGGL(k_advect_courant, dim3(red_grid(a.N)), dim3(kBlock), 0, s, a, part);
}

// One substep, one thread per cell (any grid shape).
template <int NQ>
__global__ void __launch_bounds__(kBlock) k_advect(AdvK a) {
  const int per[3] = {a.bc[0] == RH_BC_PERIODIC, a.bc[2] == RH_BC_PERIODIC,
                      a.bc[4] == RH_BC_PERIODIC};
  const int n[3] = {a.nx, a.ny, a.nz};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < a.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, a.ny, a.nz, c[0], c[1], c[2]);
    double qP[NQ], out[NQ];
    load_q<NQ>(a, idx, qP);
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = qP[q];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int gd = adv_wrap(c[d] - 1, n[d], per[d]), gu = adv_wrap(c[d] + 1, n[d], per[d]);
      int cd[3] = {c[0], c[1], c[2]}, cu[3] = {c[0], c[1], c[2]};
      cd[d] = gd;
      cu[d] = gu;
      const long long D = gd >= 0 ? cell_index(cd[0], cd[1], cd[2], a.ny, a.nz) : idx;
      const long long U = gu >= 0 ? cell_index(cu[0], cu[1], cu[2], a.ny, a.nz) : idx;
      double qD[NQ], qU[NQ];
      load_q<NQ>(a, D, qD);
      load_q<NQ>(a, U, qU);
      double ud, uu;
      face_courant(a.v[d][idx], a.v[d][D], a.v[d][U], gd >= 0, gu >= 0, a.bc[2 * d],
                   a.bc[2 * d + 1], a.scale, ud, uu);
      donor_axis<NQ>(out, qP, qD, qU, ud, uu);
    }
    store_q<NQ>(a, idx, out);
  }
}

// The same substep marching along x (the slowest index): a block owns a
// TY x TZ tile of the (y, z) plane over xc consecutive planes.  The current
// plane's conserved values and y / z velocities (tile plus a one-cell ring)
// are staged in LDS (two buffers, one barrier per plane); each thread keeps
// the values and x velocity of its own cells on the planes before and after
// in registers, and issues the global loads of plane x + 2 while it computes
// plane x.  Same arithmetic, in the same order, as k_advect.
constexpr int kAdvTY = 8, kAdvTZ = 64, kAdvXC = 32;

template <int NQ>
__global__ void __launch_bounds__(kBlock) k_advect_march(AdvK a, int xc) {
  constexpr int TY = kAdvTY, TZ = kAdvTZ, HZ = TZ + 2, PL = (TY + 2) * HZ;
  constexpr int NR = TY / (kBlock / 64);  // own rows per thread
  constexpr int NRING = 2 * TZ + 2 * TY;  // ring cells of a plane (no corners)
  static_assert(TZ == 64 && NRING <= kBlock, "one wave per row, one ring cell per thread");
  __shared__ double sq[2][NQ][PL];
  __shared__ double svy[2][PL], svz[2][PL];
  const int per[3] = {a.bc[0] == RH_BC_PERIODIC, a.bc[2] == RH_BC_PERIODIC,
                      a.bc[4] == RH_BC_PERIODIC};
  const int ntz = (a.nz + TZ - 1) / TZ, nty = (a.ny + TY - 1) / TY;
  int bid = xcd_tile(blockIdx.x, gridDim.x);
  const int tz = bid % ntz;
  bid /= ntz;
  const int ty = bid % nty;
  const int cx = bid / nty;
  const int ya = ty * TY, za = tz * TZ;  // tile cell (0, 0) = LDS (1, 1)
  const int xa = cx * xc, xb = min(xa + xc, a.nx);
  const long long plane = (long long)a.ny * a.nz;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  auto off2 = [&](int gy, int gz) -> int {
    const int wy = adv_wrap(gy, a.ny, per[1]), wz = adv_wrap(gz, a.nz, per[2]);
    return (wy >= 0 && wz >= 0) ? wy * a.nz + wz : -1;
  };
  // own cells (rows wid + 4m, column lane); overhang cells of a ragged tile
  // stand for their wrapped cell (or outside) and are not written
  int own[NR], li[NR];
  bool real[NR], hym[NR], hyp[NR], hzm[NR], hzp[NR];
#pragma unroll
  for (int m = 0; m < NR; ++m) {
    const int ly = wid + (kBlock / 64) * m, gy = ya + ly, gz = za + lane;
    real[m] = gy < a.ny && gz < a.nz;
    own[m] = off2(gy, gz);
    hym[m] = off2(gy - 1, gz) >= 0;
    hyp[m] = off2(gy + 1, gz) >= 0;
    hzm[m] = off2(gy, gz - 1) >= 0;
    hzp[m] = off2(gy, gz + 1) >= 0;
    li[m] = (ly + 1) * HZ + lane + 1;
  }
  // this thread's ring cell: rows 0 and TY + 1 need v_y, columns 0 and TZ + 1 v_z
  int r_off = -1, r_li = -1, r_axis = 1;
  if (threadIdx.x < NRING) {
    const int e = threadIdx.x;
    int ly, lz;
    if (e < 2 * TZ) {
      ly = e < TZ ? 0 : TY + 1;
      lz = e % TZ + 1;
    } else {
      const int f = e - 2 * TZ;
      ly = f % TY + 1;
      lz = f < TY ? 0 : TZ + 1;
      r_axis = 2;
    }
    r_li = ly * HZ + lz;
    r_off = off2(ya + ly - 1, za + lz - 1);
  }
  // raw loads (e not yet multiplied by n_H); zeros outside the grid
  struct Raw {
    double q[NQ];
    double v[3];
  };
  auto fetch = [&](int p, int off, int vmask, Raw& R) {
    const int gx = adv_wrap(p, a.nx, per[0]);
    const bool ok = gx >= 0 && off >= 0;
    const long long P = ok ? gx * plane + off : 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) R.q[q] = ok ? a.qi[q][P] : 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) R.v[d] = (ok && ((vmask >> d) & 1)) ? a.v[d][P] : 0.0;
  };
  auto conserved = [&](const Raw& R, double (&q)[NQ]) {
    q[0] = R.q[0];
    q[1] = R.q[1];
    q[2] = R.q[2];
    if constexpr (NQ == 4) q[3] = R.q[0] * R.q[3];
  };
  const int rmask = 1 << r_axis;
  double qm[NR][NQ], qc[NR][NQ], qn[NR][NQ];
  double vxm[NR], vxc[NR], vxn[NR], vyn[NR], vzn[NR];
  Raw own_o[NR], ring1, ring2;
  {
    const int b0 = xa & 1;
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      Raw R;
      fetch(xa - 1, own[m], 1, R);
      conserved(R, qm[m]);
      vxm[m] = R.v[0];
      fetch(xa, own[m], 7, R);
      conserved(R, qc[m]);
      vxc[m] = R.v[0];
#pragma unroll
      for (int q = 0; q < NQ; ++q) sq[b0][q][li[m]] = qc[m][q];
      svy[b0][li[m]] = R.v[1];
      svz[b0][li[m]] = R.v[2];
      fetch(xa + 1, own[m], 7, R);
      conserved(R, qn[m]);
      vxn[m] = R.v[0];
      vyn[m] = R.v[1];
      vzn[m] = R.v[2];
    }
    if (r_li >= 0) {
      Raw R;
      double q[NQ];
      fetch(xa, r_off, rmask, R);
      conserved(R, q);
#pragma unroll
      for (int k = 0; k < NQ; ++k) sq[b0][k][r_li] = q[k];
      svy[b0][r_li] = R.v[1];
      svz[b0][r_li] = R.v[2];
      fetch(xa + 1, r_off, rmask, ring1);
    }
  }
  __syncthreads();
  for (int x = xa; x < xb; ++x) {
    // loads of plane x + 2, in flight while plane x is computed
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      if (x + 2 <= xb) fetch(x + 2, own[m], 7, own_o[m]);
    }
    if (r_li >= 0 && x + 2 < xb) fetch(x + 2, r_off, rmask, ring2);
    const int b = x & 1;
    const bool hxm = adv_wrap(x - 1, a.nx, per[0]) >= 0;
    const bool hxp = adv_wrap(x + 1, a.nx, per[0]) >= 0;
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      if (!real[m]) continue;
      const int t = li[m];
      double out[NQ], qD[NQ], qU[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) out[q] = qc[m][q];
      double ud, uu;
      // x
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        qD[q] = hxm ? qm[m][q] : qc[m][q];
        qU[q] = hxp ? qn[m][q] : qc[m][q];
      }
      face_courant(vxc[m], vxm[m], vxn[m], hxm, hxp, a.bc[0], a.bc[1], a.scale, ud, uu);
      donor_axis<NQ>(out, qc[m], qD, qU, ud, uu);
      // y
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        qD[q] = hym[m] ? sq[b][q][t - HZ] : qc[m][q];
        qU[q] = hyp[m] ? sq[b][q][t + HZ] : qc[m][q];
      }
      face_courant(svy[b][t], svy[b][t - HZ], svy[b][t + HZ], hym[m], hyp[m], a.bc[2], a.bc[3],
                   a.scale, ud, uu);
      donor_axis<NQ>(out, qc[m], qD, qU, ud, uu);
      // z
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        qD[q] = hzm[m] ? sq[b][q][t - 1] : qc[m][q];
        qU[q] = hzp[m] ? sq[b][q][t + 1] : qc[m][q];
      }
      face_courant(svz[b][t], svz[b][t - 1], svz[b][t + 1], hzm[m], hzp[m], a.bc[4], a.bc[5],
                   a.scale, ud, uu);
      donor_axis<NQ>(out, qc[m], qD, qU, ud, uu);
      store_q<NQ>(a, x * plane + own[m], out);
    }
    // plane x + 1 into the other buffer (its readers finished before the
    // last barrier)
    if (x + 1 < xb) {
      const int b1 = b ^ 1;
#pragma unroll
      for (int m = 0; m < NR; ++m) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) sq[b1][q][li[m]] = qn[m][q];
        svy[b1][li[m]] = vyn[m];
        svz[b1][li[m]] = vzn[m];
      }
      if (r_li >= 0) {
        double q[NQ];
        conserved(ring1, q);
#pragma unroll
        for (int k = 0; k < NQ; ++k) sq[b1][k][r_li] = q[k];
        svy[b1][r_li] = ring1.v[1];
        svz[b1][r_li] = ring1.v[2];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NR; ++m) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        qm[m][q] = qc[m][q];
        qc[m][q] = qn[m][q];
      }
      vxm[m] = vxc[m];
      vxc[m] = vxn[m];
      if (x + 2 <= xb) {
        conserved(own_o[m], qn[m]);
        vxn[m] = own_o[m].v[0];
        vyn[m] = own_o[m].v[1];
        vzn[m] = own_o[m].v[2];
      }
    }
    ring1 = ring2;
  }
}

void launch_advect(hipStream_t s, const AdvK& a) {
  const int nty = (a.ny + kAdvTY - 1) / kAdvTY, ntz = (a.nz + kAdvTZ - 1) / kAdvTZ;
  const long long tiles = (long long)nty * ntz;
  if (a.nz >= kAdvTZ && a.ny >= kAdvTY && a.nx >= 2) {
    int ncx = (a.nx + kAdvXC - 1) / kAdvXC;
    const int xc = (a.nx + ncx - 1) / ncx;
    ncx = (a.nx + xc - 1) / xc;
    if (a.iso)
      hipLaunchKernelGGL((k_advect_march<3>), dim3((unsigned)(tiles * ncx)), dim3(kBlock), 0, s,
                         a, xc);
    else
      hipLaunchKernelGGL((k_advect_march<4>), dim3((unsigned)(tiles * ncx)), dim3(kBlock), 0, s,
                         a, xc);
    return;
  }
  const long long g = (a.N + kBlock - 1) / kBlock;
  const unsigned grid = (unsigned)(g < 65536 ? g : 65536);
  if (a.iso)
    hipLaunchKernelGGL((k_advect<3>), dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_advect<4>), dim3(grid), dim3(kBlock), 0, s, a);
}

}  // namespace rh
