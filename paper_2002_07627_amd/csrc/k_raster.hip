// Rasterization of oriented tools (the Rotate step of Algorithm 1, Sec. 2.1.5).
// Voxel-model tools are re-sampled: a grid offset o takes the label of the
// tool-frame voxel nearest to R^T o.
//
// The paper rotates and re-samples a voxel tool; here the axisymmetric tool
// (cutter K of radius r over axial [0, L), holder H of radius rh over axial
// [L, L + Lh)) is rasterized analytically at voxel centres for every
// orientation.  With a = o.d (axial coordinate) and q^2 = |o - a d|^2:
//   flat cutter  0 <= a < L and q^2 <= r^2
//   ball cutter  |o - r d|^2 <= r^2, or r <= a < L and q^2 <= r^2
//   holder       L <= a < L + Lh and q^2 <= rh^2
// Lattice directions v use exact integer forms of the same tests.  Float64
// directions evaluate a = (x dx + y dy) + z dz, p = o - a d, q^2 = (px^2 + py^2)
// + pz^2 in that order; this file is compiled without FP contraction.
//
// Output per orientation: a flag byte per bounding-box voxel (bit 0 tool T,
// bit 1 cutter K, bit 2 sharp point S), extents by atomics, then runs.
#include "imf_internal.h"

#pragma clang fp contract(off)

__device__ __forceinline__ int raster_member(const imf_raster_desc& c, long long ox, long long oy,
                                             long long oz) {
  int cut = 0, hold = 0;
  if (c.kind == 3) {
    // voxel model: inverse nearest-neighbour re-sampling, the tool-frame point
    // R^T o rounded (halves to even) to a label voxel
    const double x = (double)ox, y = (double)oy, z = (double)oz;
    long long idx[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const double u = (c.R[a] * x + c.R[3 + a] * y) + c.R[6 + a] * z;
      idx[a] = (long long)rint(u) + c.vorg[a];
      if (idx[a] < 0 || idx[a] >= c.vdim[a]) return 0;
    }
    const uint8_t lab = c.vox[(idx[2] * c.vdim[1] + idx[1]) * c.vdim[0] + idx[0]];
    cut = lab == 2;
    hold = lab == 1;
    return (cut || hold) | (cut << 1);
  }
  if (c.lattice) {
    long long dot, o2;
    if (c.ndim == 3) {
      dot = ox * c.v[0] + oy * c.v[1] + oz * c.v[2];
      o2 = ox * ox + oy * oy + oz * oz;
    } else {
      dot = ox * c.v[0] + oy * c.v[1];
      o2 = ox * ox + oy * oy;
    }
    const long long n = c.vn;
    const long long perp4 = 4 * (o2 * n - dot * dot);
    const long long dot4 = 4 * dot * dot;
    const bool in_r = perp4 <= c.r2 * c.r2 * n;
    const bool a_ge0 = dot >= 0;
    const bool a_ltL = a_ge0 && dot4 < c.L2 * c.L2 * n;
    if (c.kind == 1) {
      const bool in_ball = a_ge0 && o2 * o2 * n <= c.r2 * c.r2 * dot * dot;
      const bool a_ger = a_ge0 && dot4 >= c.r2 * c.r2 * n;
      cut = in_ball || (a_ger && a_ltL && in_r);
    } else {
      cut = a_ltL && in_r;
    }
    hold = a_ge0 && dot4 >= c.L2 * c.L2 * n && dot4 < c.LH2 * c.LH2 * n &&
           perp4 <= c.rh2 * c.rh2 * n;
  } else {
    const double dx = c.d[0], dy = c.d[1], dz = c.d[2];
    const double x = (double)ox, y = (double)oy, z = (double)oz;
    double a, q2;
    if (c.ndim == 3) {
      a = (x * dx + y * dy) + z * dz;
      const double px = x - a * dx, py = y - a * dy, pz = z - a * dz;
      q2 = (px * px + py * py) + pz * pz;
    } else {
      a = x * dx + y * dy;
      const double px = x - a * dx, py = y - a * dy;
      q2 = px * px + py * py;
    }
    const double r = c.r, L = c.L;
    const bool in_cyl = a < L && q2 <= r * r;
    if (c.kind == 1) {
      const double bx = x - r * dx, by = y - r * dy;
      double b2;
      if (c.ndim == 3) {
        const double bz = z - r * dz;
        b2 = (bx * bx + by * by) + bz * bz;
      } else {
        b2 = bx * bx + by * by;
      }
      cut = b2 <= r * r || (a >= r && in_cyl);
    } else {
      cut = a >= 0 && in_cyl;
    }
    hold = a >= L && a < c.LH && q2 <= c.rh * c.rh;
  }
  return (cut || hold) | (cut << 1);
}

// wave-wide min / max of an int (wave64)
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ void __launch_bounds__(IMF_WG) k_raster(const imf_raster_desc* __restrict__ descs,
                                                   uint8_t* __restrict__ flags,
                                                   int* __restrict__ ext_all) {
  const int q = blockIdx.y;
  const imf_raster_desc c = descs[q];
  const long long vol = (long long)c.dim[0] * c.dim[1] * c.dim[2];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int m = 0, x = 0, y = 0, z = 0;
  if (i < vol) {
    x = (int)(i % c.dim[0]);
    y = (int)((i / c.dim[0]) % c.dim[1]);
    z = (int)(i / ((long long)c.dim[0] * c.dim[1]));
    x += c.lo[0];
    y += c.lo[1];
    z += c.lo[2];
    m = raster_member(c, x, y, z);
    flags[c.flags_off + i] = (uint8_t)m;
  }
  // tool extents: ext[0..5] min/max, ext[12] count
  int* ext = ext_all + (size_t)q * IMF_EXT_INTS;
  {
    const int BIG = 1 << 29;
    const bool in = (m & 1) != 0;
    int mn[3] = {in ? x : BIG, in ? y : BIG, in ? z : BIG};
    int mx[3] = {in ? x : -BIG, in ? y : -BIG, in ? z : -BIG};
    int cnt = in ? 1 : 0;
    for (int a = 0; a < 3; a++) {
      mn[a] = wave_min(mn[a]);
      mx[a] = wave_max(mx[a]);
    }
    cnt = wave_sum(cnt);
    if ((threadIdx.x & 63) == 0 && cnt > 0) {
      for (int a = 0; a < 3; a++) {
        atomicMin(&ext[a], mn[a]);
        atomicMax(&ext[3 + a], mx[a]);
      }
      atomicAdd(&ext[12], cnt);
    }
  }
}

// Select the sharp points S among the cutter voxels (bit 2) and reduce the
// extents of S.  Mode 0: all cutter voxels (Algorithm 1 loops over the whole
// support of the cutter).  Mode 1: cutter voxels with an axis neighbour outside
// the cutter (boundary sampling).  Mode 2: the tip (origin) voxel only.
__global__ void __launch_bounds__(IMF_WG) k_sharp(const imf_raster_desc* __restrict__ descs,
                                                  uint8_t* __restrict__ flags,
                                                  int* __restrict__ ext_all) {
  const int q = blockIdx.y;
  const imf_raster_desc& c = descs[q];
  const int d0 = c.dim[0], d1 = c.dim[1], d2 = c.dim[2];
  const long long vol = (long long)d0 * d1 * d2;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool in = false;
  int x = 0, y = 0, z = 0;
  if (i < vol) {
    x = (int)(i % d0);
    y = (int)((i / d0) % d1);
    z = (int)(i / ((long long)d0 * d1));
    uint8_t* fl = flags + c.flags_off;
    const int m = fl[i];
    if (c.sharp == 2) {
      // the tip alone: the origin (a ball cutter's raster may miss it by
      // rounding, since it lies exactly on the sphere)
      in = (x + c.lo[0] == 0) && (y + c.lo[1] == 0) && (z + c.lo[2] == 0);
    } else if (m & 2) {
      if (c.sharp == 0) {
        in = true;
      } else {
        // the bounding box has a margin of at least one empty voxel
        const int p[3] = {x, y, z};
        for (int a = 0; a < c.ndim && !in; a++)
          for (int sgn = -1; sgn <= 1 && !in; sgn += 2) {
            int nb[3] = {p[0], p[1], p[2]};
            nb[a] += sgn;
            bool cutn = false;
            if (nb[a] >= 0 && nb[a] < c.dim[a])
              cutn = (fl[((long long)nb[2] * d1 + nb[1]) * d0 + nb[0]] & 2) != 0;
            if (!cutn) in = true;
          }
      }
    }
    // bit 2 is written by this kernel only; neighbours read bit 1
    if (in) atomicOr((unsigned int*)(fl + (i & ~3LL)), 4u << (8 * (i & 3)));
  }
  int* ext = ext_all + (size_t)q * IMF_EXT_INTS;
  const int BIG = 1 << 29;
  int mn[3] = {in ? x + c.lo[0] : BIG, in ? y + c.lo[1] : BIG, in ? z + c.lo[2] : BIG};
  int mx[3] = {in ? x + c.lo[0] : -BIG, in ? y + c.lo[1] : -BIG, in ? z + c.lo[2] : -BIG};
  int cnt = in ? 1 : 0;
  for (int a = 0; a < 3; a++) {
    mn[a] = wave_min(mn[a]);
    mx[a] = wave_max(mx[a]);
  }
  cnt = wave_sum(cnt);
  if ((threadIdx.x & 63) == 0 && cnt > 0) {
    for (int a = 0; a < 3; a++) {
      atomicMin(&ext[6 + a], mn[a]);
      atomicMax(&ext[9 + a], mx[a]);
    }
    atomicAdd(&ext[13], cnt);
  }
}

// One thread per row of the bounding box: emit the runs of bit `bit` along
// axis `ax` into the row's slots.  kind 0: T along x, 1: S along s_axis,
// 2: S along x.
__global__ void __launch_bounds__(IMF_WG) k_runs(const imf_raster_desc* __restrict__ descs,
                                                 const uint8_t* __restrict__ flags,
                                                 imf_run* __restrict__ slots,
                                                 int* __restrict__ cnt, int* __restrict__ ext_all,
                                                 int max_rows) {
  const int q = blockIdx.y;
  const int kind = blockIdx.z;
  const imf_raster_desc& c = descs[q];
  const int ax = kind == 1 ? c.s_axis : 0;
  const int bit = kind == 0 ? 1 : 4;
  const int u = (ax + 1) % 3, w = (ax + 2) % 3;
  const int rows = c.dim[u] * c.dim[w];
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  int nr = 0;
  if (row < rows) {
    const int iu = row % c.dim[u], iw = row / c.dim[u];
    const long long str[3] = {1, c.dim[0], (long long)c.dim[0] * c.dim[1]};
    const uint8_t* fl = flags + c.flags_off + iu * str[u] + iw * str[w];
    imf_run* out = slots + ((size_t)(c.rows_off + row) * 3 + kind) * IMF_MAX_RUNS_PER_ROW;
    int start = -1;
    bool overflow = false;
    for (int j = 0; j <= c.dim[ax]; j++) {
      const bool on = j < c.dim[ax] && (fl[j * str[ax]] & bit);
      if (on && start < 0) start = j;
      if (!on && start >= 0) {
        if (nr < IMF_MAX_RUNS_PER_ROW) {
          int p[3];
          p[ax] = start + c.lo[ax];
          p[u] = iu + c.lo[u];
          p[w] = iw + c.lo[w];
          out[nr] = imf_run{p[0], p[1], p[2], j - start};
        } else {
          overflow = true;
        }
        nr++;
        start = -1;
      }
    }
    cnt[(size_t)(c.rows_off + row) * 3 + kind] = nr < IMF_MAX_RUNS_PER_ROW ? nr
                                                                             : IMF_MAX_RUNS_PER_ROW;
    if (overflow) atomicOr(&ext_all[(size_t)q * IMF_EXT_INTS + 14], 1);
  }
  (void)max_rows;
  const int tot = wave_sum(nr < IMF_MAX_RUNS_PER_ROW ? nr : IMF_MAX_RUNS_PER_ROW);
  if ((threadIdx.x & 63) == 0 && tot > 0)
    atomicAdd(&ext_all[(size_t)q * IMF_EXT_INTS + 15 + kind], tot);
}

// One workgroup per (orientation, kind): ordered compaction of the row slots.
__global__ void __launch_bounds__(IMF_WG) k_compact(const imf_raster_desc* __restrict__ descs,
                                                    const imf_run* __restrict__ slots,
                                                    const int* __restrict__ cnt,
                                                    const long long* __restrict__ out_base,
                                                    imf_run* __restrict__ out) {
  const int q = blockIdx.x;
  const int kind = blockIdx.y;
  const imf_raster_desc& c = descs[q];
  const int ax = kind == 1 ? c.s_axis : 0;
  const int u = (ax + 1) % 3, w = (ax + 2) % 3;
  const int rows = c.dim[u] * c.dim[w];
  __shared__ int sc[IMF_WG];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  imf_run* dst = out + out_base[(size_t)q * 3 + kind];
  for (int r0 = 0; r0 < rows; r0 += IMF_WG) {
    const int row = r0 + threadIdx.x;
    const int n = row < rows ? cnt[(size_t)(c.rows_off + row) * 3 + kind] : 0;
    sc[threadIdx.x] = n;
    __syncthreads();
    // inclusive scan (Hillis-Steele)
    for (int o = 1; o < IMF_WG; o <<= 1) {
      const int v = threadIdx.x >= o ? sc[threadIdx.x - o] : 0;
      __syncthreads();
      sc[threadIdx.x] += v;
      __syncthreads();
    }
    const int excl = sc[threadIdx.x] - n + base;
    const imf_run* src = slots + (size_t)((c.rows_off + row) * 3 + kind) * IMF_MAX_RUNS_PER_ROW;
    for (int k = 0; k < n; k++) dst[excl + k] = src[k];
    __syncthreads();
    if (threadIdx.x == IMF_WG - 1) base += sc[IMF_WG - 1];
    __syncthreads();
  }
}

hipError_t imf_launch_raster(const imf_raster_desc* d_desc, int n_orient, int max_vol,
                             uint8_t* flags, int* ext, hipStream_t s) {
  dim3 grid((max_vol + IMF_WG - 1) / IMF_WG, n_orient);
  hipLaunchKernelGGL(k_raster, grid, dim3(IMF_WG), 0, s, d_desc, flags, ext);
  return hipGetLastError();
}

hipError_t imf_launch_sharp_subset(const imf_raster_desc* d_desc, int n_orient, int max_vol,
                                   uint8_t* flags, int* ext, hipStream_t s) {
  dim3 grid((max_vol + IMF_WG - 1) / IMF_WG, n_orient);
  hipLaunchKernelGGL(k_sharp, grid, dim3(IMF_WG), 0, s, d_desc, flags, ext);
  return hipGetLastError();
}

hipError_t imf_launch_runs(const imf_raster_desc* d_desc, int n_orient, int max_rows,
                           const uint8_t* flags, imf_run* slots, int* cnt, int* ext,
                           hipStream_t s) {
  dim3 grid((max_rows + IMF_WG - 1) / IMF_WG, n_orient, 3);
  hipLaunchKernelGGL(k_runs, grid, dim3(IMF_WG), 0, s, d_desc, flags, slots, cnt, ext, max_rows);
  return hipGetLastError();
}

hipError_t imf_launch_compact(const imf_raster_desc* d_desc, int n_orient, int max_rows,
                              const imf_run* slots, const int* cnt, const long long* out_base,
                              imf_run* out, hipStream_t s) {
  (void)max_rows;
  dim3 grid(n_orient, 3);
  hipLaunchKernelGGL(k_compact, grid, dim3(IMF_WG), 0, s, d_desc, slots, cnt, out_base, out);
  return hipGetLastError();
}
