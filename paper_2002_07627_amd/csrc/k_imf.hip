// Exact overlaps (direct correlation, guard-band recheck), the sharp-point
// minimum filter with the running minimum over orientations, the accessible
// masks, and the final normalization / classification of Algorithm 1.
#include "imf_internal.h"

#define Q24 16777216.0

__device__ __forceinline__ float wave_max_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// order-preserving map of float to unsigned int (for atomic max)
__device__ __forceinline__ unsigned int f2ord(float f) {
  const unsigned int b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord2f(unsigned int u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// ---------------------------------------------------------------------------
// prefix sums of rho_O = max(design, fixture) along x, fixed point:
// ps[z][y][x'] = sum_{x < x'} rho_O(x, y, z), x' in [0, nx]   (one wave per row)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(IMF_WG) k_prefix_x(const void* __restrict__ design, int density,
                                                     const uint8_t* __restrict__ fixture, int nx,
                                                     long long rows, long long* __restrict__ ps) {
  const long long row = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  long long carry = 0;
  long long* out = ps + row * (nx + 1);
  if (lane == 0) out[0] = 0;
  for (int x0 = 0; x0 < nx; x0 += 64) {
    const int x = x0 + lane;
    long long v = 0;
    if (x < nx) {
      const long long idx = row * nx + x;
      if (fixture && fixture[idx]) {
        v = density ? (long long)Q24 : 1;
      } else if (density) {
        v = (long long)((double)((const float*)design)[idx] * Q24);
      } else {
        v = ((const uint8_t*)design)[idx];
      }
    }
    // inclusive wave scan
    for (int o = 1; o < 64; o <<= 1) {
      const long long u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    if (x < nx) out[x + 1] = carry + v;
    carry += __shfl(v, 63);
  }
}

hipError_t imf_launch_prefix_x(const void* design, int density, const uint8_t* fixture, int nx,
                               int ny, int nz, long long* ps, hipStream_t s) {
  const long long rows = (long long)ny * nz;
  const int per = IMF_WG / 64;
  hipLaunchKernelGGL(k_prefix_x, dim3((unsigned)((rows + per - 1) / per)), dim3(IMF_WG), 0, s,
                     design, density, fixture, nx, rows, ps);
  return hipGetLastError();
}

// exact overlap at translation t: sum over x-runs of T of row sums (Eq. ident)
__device__ __forceinline__ long long exact_overlap(const imf_orient_desc& d,
                                                   const long long* __restrict__ ps, int nx,
                                                   int ny, int nz, int tx, int ty, int tz) {
  const imf_run* rl = d.truns;
  long long s = 0;
  for (int r = 0; r < d.n_truns; r++) {
    const imf_run u = rl[r];
    const int y = ty + u.y, z = tz + u.z;
    if (y < 0 || y >= ny || z < 0 || z >= nz) continue;
    int x0 = tx + u.x, x1 = x0 + u.len;
    x0 = max(x0, 0);
    x1 = min(x1, nx);
    if (x1 <= x0) continue;
    const long long* row = ps + ((long long)z * ny + y) * (nx + 1);
    s += row[x1] - row[x0];
  }
  return s;
}

// ---------------------------------------------------------------------------
// direct correlation over the query box (exact)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(IMF_WG) k_direct(const imf_orient_desc* __restrict__ desc,
                                                   const long long* __restrict__ ps, int nx,
                                                   int ny, int nz, int density,
                                                   float* __restrict__ g, long long g_stride) {
  const int q = blockIdx.y;
  const imf_orient_desc& d = desc[q];
  const long long vol = (long long)d.box_dim[0] * d.box_dim[1] * d.box_dim[2];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vol) return;
  const int bx = (int)(i % d.box_dim[0]);
  const int by = (int)((i / d.box_dim[0]) % d.box_dim[1]);
  const int bz = (int)(i / ((long long)d.box_dim[0] * d.box_dim[1]));
  const long long s = exact_overlap(d, ps, nx, ny, nz, bx + d.box_lo[0],
                                    by + d.box_lo[1], bz + d.box_lo[2]);
  g[q * g_stride + i] = density ? (float)((double)s * (1.0 / Q24)) : (float)s;
}

hipError_t imf_launch_direct(const imf_orient_desc* desc, int nq, const long long* ps, int nx, int ny, int nz, int density, float* g,
                             long long g_stride, int max_vol, hipStream_t s) {
  dim3 grid((max_vol + IMF_WG - 1) / IMF_WG, nq);
  hipLaunchKernelGGL(k_direct, grid, dim3(IMF_WG), 0, s, desc, ps, nx, ny, nz, density, g,
                     g_stride);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// guard-band recheck: recompute flagged overlaps exactly.  Binary: the exact
// count.  Density with a known threshold: the exact value, rounded to float so
// that the decision g <= theta taken on the float equals the exact decision.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(IMF_WG) k_recheck(const imf_orient_desc* __restrict__ desc,
                                                    const long long* __restrict__ ps, int nx,
                                                    int ny, int nz, int density,
                                                    const int* __restrict__ flag_cnt,
                                                    const int2* __restrict__ flags, int flag_cap,
                                                    int theta_known, double theta,
                                                    float* __restrict__ g, long long g_stride) {
  const int n = min(*flag_cnt, flag_cap);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int2 f = flags[k];
    const imf_orient_desc& d = desc[f.x];
    const long long i = f.y;
    const int bx = (int)(i % d.box_dim[0]);
    const int by = (int)((i / d.box_dim[0]) % d.box_dim[1]);
    const int bz = (int)(i / ((long long)d.box_dim[0] * d.box_dim[1]));
    const long long s = exact_overlap(d, ps, nx, ny, nz, bx + d.box_lo[0],
                                      by + d.box_lo[1], bz + d.box_lo[2]);
    float v;
    if (!density) {
      v = (float)s;
    } else {
      const double e = (double)s * (1.0 / Q24);
      v = (float)e;
      if (theta_known) {
        const bool free_ = e <= theta;
        for (int it = 0; it < 4; it++) {
          if (free_ && (double)v > theta) v = nextafterf(v, -INFINITY);
          else if (!free_ && (double)v <= theta) v = nextafterf(v, INFINITY);
          else break;
        }
      }
    }
    g[(long long)f.x * g_stride + i] = v;
  }
}

hipError_t imf_launch_recheck(const imf_orient_desc* desc, const long long* ps, int nx, int ny, int nz, int density,
                              const int* flag_cnt, const int2* flags, int flag_cap,
                              int theta_known, double theta, float* g, long long g_stride,
                              hipStream_t s) {
  const int blocks = flag_cap < 256 * 1024 ? (flag_cap + IMF_WG - 1) / IMF_WG : 1024;
  hipLaunchKernelGGL(k_recheck, dim3(blocks > 0 ? blocks : 1), dim3(IMF_WG), 0, s, desc, ps,
                     nx, ny, nz, density, flag_cnt, flags, flag_cap, theta_known, theta, g,
                     g_stride);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sharp-point minimum (Eq. imf_2): gamma(x) = min over runs of S of the window
// minimum of g along the run axis.  Level s of the sparse table holds
// min g[p, p + 2^s) along the axis; a run of length l reads two level-s
// windows, s = floor(log2 l).
// ---------------------------------------------------------------------------
// All sparse-table levels of one orientation in one pass: lines along the run
// axis are staged in LDS (ping-pong), each level is formed there and written
// out.  A workgroup holds LT lines of length m = box extent along the axis;
// for the x axis the lines are rows, otherwise LT consecutive x columns.
#define LVL_LT 16
__global__ void __launch_bounds__(IMF_WG) k_levels(const imf_orient_desc* __restrict__ desc,
                                                   const float* __restrict__ g,
                                                   long long g_stride, float* __restrict__ lvl,
                                                   long long lvl_stride, int nlvl) {
  extern __shared__ float lds[];
  const int q = blockIdx.z;
  const imf_orient_desc& d = desc[q];
  const int ax = d.s_axis;
  const int mx = d.box_dim[0], my = d.box_dim[1], mz = d.box_dim[2];
  const int m = d.box_dim[ax];
  const long long sa = ax == 0 ? 1 : (ax == 1 ? (long long)mx : (long long)mx * my);
  // lines: for ax == 0, rows (y, z); else groups of LVL_LT consecutive x at a
  // fixed coordinate of the third axis
  long long nlines;
  if (ax == 0) nlines = (long long)my * mz;
  else nlines = (long long)((mx + LVL_LT - 1) / LVL_LT) * (ax == 1 ? mz : my);
  const long long gid = blockIdx.x;
  const int lines_per_wg = ax == 0 ? 4 : 1;
  if (gid * lines_per_wg >= nlines) return;
  float* A = lds;
  float* B = lds + LVL_LT * m;
  const float* src = g + q * g_stride;
  float* dstb = lvl + q * lvl_stride;
  // element (line l, position i) -> box index
  auto index_of = [&](int l, int i, bool& ok) -> long long {
    ok = true;
    if (ax == 0) {
      const long long row = gid * 4 + l;
      if (row >= nlines) { ok = false; return 0; }
      return row * mx + i;
    }
    const long long grp = gid;
    const int nxg = (mx + LVL_LT - 1) / LVL_LT;
    const int x = (int)(grp % nxg) * LVL_LT + l;
    const int o = (int)(grp / nxg);
    if (x >= mx) { ok = false; return 0; }
    return ax == 1 ? ((long long)o * my * mx + x + (long long)i * sa)
                   : ((long long)o * mx + x + (long long)i * sa);
  };
  const int nl = ax == 0 ? 4 : LVL_LT;
  // load: for ax != 0 consecutive threads take consecutive x (coalesced)
  for (int t = threadIdx.x; t < nl * m; t += IMF_WG) {
    int l, i;
    if (ax == 0) { l = t / m; i = t - l * m; }
    else { i = t / nl; l = t - i * nl; }
    bool ok;
    const long long gi = index_of(l, i, ok);
    A[l * m + i] = ok ? src[gi] : INFINITY;
  }
  __syncthreads();
  const int nl_q = d.nlvl < nlvl ? d.nlvl : nlvl;
  for (int s = 1; s <= nl_q; s++) {
    const int h = 1 << (s - 1);
    float* dst = dstb + (long long)(s - 1) * g_stride;
    for (int t = threadIdx.x; t < nl * m; t += IMF_WG) {
      int l, i;
      if (ax == 0) { l = t / m; i = t - l * m; }
      else { i = t / nl; l = t - i * nl; }
      float v = A[l * m + i];
      if (i + h < m) v = fminf(v, A[l * m + i + h]);
      B[l * m + i] = v;
      bool ok;
      const long long gi = index_of(l, i, ok);
      if (ok) dst[gi] = v;
    }
    __syncthreads();
    float* tmp = A;
    A = B;
    B = tmp;
  }
}

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

// Sharp-point minimum of ONE orientation (Eq. imf_2): one wave per 64
// consecutive x of a row; f is updated in place (one orientation per launch,
// so every voxel has a single writer).  The runs are turned into box-index
// offsets in LDS once per workgroup, and the run loop is unrolled so that 16
// independent gathers are in flight per wave.
#define MF_LDS_RUNS 1024
#define MF_BY 16
#define MF_BZ 16
// Wave -> output mapping.  The hardware hands workgroups to the 8 XCDs round
// robin, so workgroup b runs on XCD b % 8.  Each XCD is given a contiguous range
// of bricks (one 64-wide x chunk by MF_BY rows by MF_BZ planes, y fastest), so
// the waves resident on one XCD cover a compact region and share its L2.
__device__ __forceinline__ bool mf_map(int nx, int ny, int nz, int& w, int& y, int& z) {
  const int words = (nx + 63) >> 6;
  const int nby = (ny + MF_BY - 1) / MF_BY, nbz = (nz + MF_BZ - 1) / MF_BZ;
  const long long nbricks = (long long)words * nby * nbz;
  const int wg_per_brick = MF_BY * MF_BZ / (IMF_WG / 64);
  const long long nwg = nbricks * wg_per_brick;
  const long long per_xcd = (nwg + 7) / 8;
  const long long b = blockIdx.x;
  const long long lg = (b % 8) * per_xcd + b / 8;
  if (lg >= nwg) return false;
  const long long brick = lg / wg_per_brick;
  const int wib = (int)(lg % wg_per_brick) * (IMF_WG / 64) + (threadIdx.x >> 6);
  const int yb = (int)(brick % nby);
  const long long r = brick / nby;
  const int zb = (int)(r % nbz);
  w = (int)(r / nbz);
  y = yb * MF_BY + wib % MF_BY;
  z = zb * MF_BZ + wib / MF_BY;
  return y < ny && z < nz;
}

__global__ void __launch_bounds__(IMF_WG) k_minfilter(imf_min_args a, int qi) {
  __shared__ int4 rr[MF_LDS_RUNS];
  const imf_orient_desc& d = a.desc[qi];
  const int nr = d.n_sruns;
  const int ax = d.s_axis;
  const long long sx = 1, sy = d.box_dim[0], sz = (long long)d.box_dim[0] * d.box_dim[1];
  const long long sa = ax == 0 ? sx : (ax == 1 ? sy : sz);
  for (int r = threadIdx.x; r < nr && r < MF_LDS_RUNS; r += IMF_WG) {
    const imf_run u = d.sruns[r];
    const int sl = ilog2(u.len);
    rr[r] = make_int4((int)(-(u.x * sx + u.y * sy + u.z * sz) - (long long)(u.len - 1) * sa), sl,
                      (int)((long long)(u.len - (1 << sl)) * sa), 0);
  }
  __syncthreads();
  const int words = (a.nx + 63) >> 6;
  const int lane = threadIdx.x & 63;
  int w, y, z;
  if (!mf_map(a.nx, a.ny, a.nz, w, y, z)) return;
  const int x = w * 64 + lane;
  const bool valid = x < a.nx;
  const long long vi = ((long long)z * a.ny + y) * a.nx + x;
  const float* g = a.g + qi * a.g_stride;
  const float* lv = a.lvl + qi * a.lvl_stride - a.g_stride;  // level s at lv + s * g_stride
  float gam = INFINITY;
  // translation t = x - k; box index of t for k = 0 (invalid lanes read a
  // clamped in-box position and are discarded)
  const int xc = valid ? x : a.nx - 1;
  const long long base = (long long)(xc - d.box_lo[0]) + (long long)(y - d.box_lo[1]) * sy +
                         (long long)(z - d.box_lo[2]) * sz;
  const int nl = nr < MF_LDS_RUNS ? nr : MF_LDS_RUNS;
  int r = 0;
  for (; r + 8 <= nl; r += 8) {
    float v[16];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int4 u = rr[r + j];
      const float* L = u.y == 0 ? g : lv + (long long)u.y * a.g_stride;
      const long long p = base + u.x;
      v[2 * j] = L[p];
      v[2 * j + 1] = L[p + u.z];
    }
#pragma unroll
    for (int j = 0; j < 8; j++) gam = fminf(gam, fminf(v[2 * j], v[2 * j + 1]));
  }
  for (; r < nl; r++) {
    const int4 u = rr[r];
    const float* L = u.y == 0 ? g : lv + (long long)u.y * a.g_stride;
    const long long p = base + u.x;
    gam = fminf(gam, fminf(L[p], L[p + u.z]));
  }
  for (r = MF_LDS_RUNS; r < nr; r++) {  // beyond the LDS capacity: read the runs directly
    const imf_run u = d.sruns[r];
    const int sl = ilog2(u.len);
    const float* L = sl == 0 ? g : lv + (long long)sl * a.g_stride;
    const long long p = base - (u.x * sx + u.y * sy + u.z * sz) - (long long)(u.len - 1) * sa;
    gam = fminf(gam, fminf(L[p], L[p + (long long)(u.len - (1 << sl)) * sa]));
  }
  if (valid) {
    const float fo = a.f[vi];
    if (gam < fo) a.f[vi] = gam;
    if (a.gamma_stack)
      a.gamma_stack[(long long)(a.gamma_q0 + qi) * a.nx * a.ny * a.nz + vi] = gam;
  }
  if (a.masks_on) {
    const bool om = valid && a.omega0[vi];
    const unsigned long long bits = __ballot(om && (double)gam <= a.theta);
    if (lane == 0)
      a.masks[((long long)(a.mask_q0 + qi) * a.nz + z) * a.ny * words + (long long)y * words + w] =
          bits;
  }
}

hipError_t imf_launch_minfilter(const imf_min_args& a, hipStream_t s, int stage) {
  hipError_t e;
  if ((stage < 0 || stage == 0) && a.nlvl > 0) {
    // one launch for all orientations of the batch; the grid covers the
    // largest line count (rows for x runs, x groups otherwise)
    const size_t sm = (size_t)2 * LVL_LT * a.max_m * sizeof(float);
    if (sm > 64 * 1024)
      if ((e = hipFuncSetAttribute((const void*)k_levels,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm)) !=
          hipSuccess)
        return e;
    hipLaunchKernelGGL(k_levels, dim3((unsigned)a.max_lines, 1, a.nq), dim3(IMF_WG), sm, s, a.desc, a.g, a.g_stride, a.lvl, a.lvl_stride, a.nlvl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (stage == 0) return hipSuccess;
  const int words = (a.nx + 63) >> 6;
  const long long nbricks = (long long)words * ((a.ny + MF_BY - 1) / MF_BY) *
                            ((a.nz + MF_BZ - 1) / MF_BZ);
  const long long nwg = nbricks * (MF_BY * MF_BZ / (IMF_WG / 64));
  const long long grid = (nwg + 7) / 8 * 8;
  for (int q = 0; q < a.nq; q++) {
    hipLaunchKernelGGL(k_minfilter, dim3((unsigned)grid), dim3(IMF_WG), 0, s, a, q);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// sweep route for the masks: A = Omega_0 and (D^c dilated by S), D^c = {t :
// g(t) <= theta}, as bit rows along x (Eqs. sweep, A and conv_A).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(IMF_WG) k_dc_bits(const imf_orient_desc* __restrict__ desc,
                                                    const float* __restrict__ g,
                                                    long long g_stride, double theta,
                                                    uint64_t* __restrict__ dc,
                                                    long long dc_stride) {
  const int q = blockIdx.y;
  const imf_orient_desc& d = desc[q];
  const int mx = d.box_dim[0];
  const int words = (mx + 63) >> 6;
  const long long rows = (long long)d.box_dim[1] * d.box_dim[2];
  const long long wave = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wave >= rows * words) return;
  const long long row = wave / words;
  const int w = (int)(wave % words);
  const int x = w * 64 + lane;
  bool fr = false;
  if (x < mx) fr = (double)g[q * g_stride + row * mx + x] <= theta;
  const unsigned long long b = __ballot(fr);
  if (lane == 0) dc[q * dc_stride + row * words + w] = b;
}

// bit i of the 64-bit window starting at bit position `pos` of a bit row
__device__ __forceinline__ uint64_t row_window(const uint64_t* row, int nwords, long long pos) {
  // bits [pos, pos + 64) ; positions outside [0, 64*nwords) read as 0
  const long long wi = pos >> 6;  // arithmetic shift (floor)
  const int sh = (int)(pos & 63);
  const uint64_t lo = (wi >= 0 && wi < nwords) ? row[wi] : 0ull;
  const uint64_t hi = (wi + 1 >= 0 && wi + 1 < nwords) ? row[wi + 1] : 0ull;
  return sh == 0 ? lo : ((lo >> sh) | (hi << (64 - sh)));
}

__global__ void __launch_bounds__(IMF_WG) k_sweep(imf_sweep_args a) {
  const int q = blockIdx.y;
  const imf_orient_desc& d = a.desc[q];
  const int words = (a.nx + 63) >> 6;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)words * a.ny * a.nz) return;
  const int w = (int)(idx % words);
  const long long yz = idx / words;
  const int y = (int)(yz % a.ny), z = (int)(yz / a.ny);
  const int mx = d.box_dim[0];
  const int bw = (mx + 63) >> 6;
  const uint64_t* dc = a.dc + q * a.dc_stride;
  uint64_t acc = 0;
  const imf_run* rl = d.sruns;  // x-runs of S for this route
  for (int r = 0; r < d.n_sruns; r++) {
    const imf_run u = rl[r];
    const int ty = y - u.y - d.box_lo[1], tz = z - u.z - d.box_lo[2];
    if (ty < 0 || ty >= d.box_dim[1] || tz < 0 || tz >= d.box_dim[2]) continue;
    const uint64_t* row = dc + ((long long)tz * d.box_dim[1] + ty) * bw;
    // x is swept iff some j in [0, len) has D^c at t_x = x - u.x - j; in box
    // coordinates b = x - u.x - j - box_lo_x.  For the word's 64 x values
    // OR the windows starting at b0 - j.
    const long long b0 = (long long)w * 64 - u.x - d.box_lo[0];
    uint64_t m = 0;
    for (int j = 0; j < u.len; j++) m |= row_window(row, bw, b0 - j);
    acc |= m;
  }
  // Omega_0 bits and the grid tail
  uint64_t om = 0;
  const long long vrow = ((long long)z * a.ny + y) * a.nx;
  for (int b = 0; b < 64; b++) {
    const int x = w * 64 + b;
    if (x < a.nx && a.omega0[vrow + x]) om |= 1ull << b;
  }
  a.masks[((long long)(a.mask_q0 + q) * a.nz + z) * a.ny * words + (long long)y * words + w] =
      acc & om;
}

hipError_t imf_launch_sweep(const imf_sweep_args& a, hipStream_t s) {
  hipError_t e;
  // D^c bits over the largest box
  {
    const long long waves = a.dc_stride;  // >= rows * words of every box
    const int per = IMF_WG / 64;
    hipLaunchKernelGGL(k_dc_bits, dim3((unsigned)((waves + per - 1) / per), a.nq), dim3(IMF_WG),
                       0, s, a.desc, a.g, a.g_stride, a.theta, a.dc, a.dc_stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int words = (a.nx + 63) >> 6;
  const long long n = (long long)words * a.ny * a.nz;
  hipLaunchKernelGGL(k_sweep, dim3((unsigned)((n + IMF_WG - 1) / IMF_WG), a.nq), dim3(IMF_WG), 0,
                     s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// finalize
// ---------------------------------------------------------------------------
__global__ void k_fill(float* f, long long n, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = v;
}
hipError_t imf_launch_fill_f(float* f, long long n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f, n, v);
  return hipGetLastError();
}

__global__ void k_omega0(const uint8_t* fixture, const uint8_t* domain, uint8_t* om, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  om[i] = domain ? (domain[i] != 0) : (fixture ? (fixture[i] == 0) : 1);
}
hipError_t imf_launch_omega0(const uint8_t* fixture, const uint8_t* domain, uint8_t* omega0,
                             long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_omega0, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fixture,
                     domain, omega0, n);
  return hipGetLastError();
}

// F_max = max of f over Omega_0 (0 if Omega_0 is empty); stored order-mapped
__global__ void __launch_bounds__(IMF_WG) k_fmax(const float* __restrict__ f,
                                                 const uint8_t* __restrict__ om, long long n,
                                                 unsigned int* out) {
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    if (om[i]) m = fmaxf(m, f[i]);
  m = wave_max_f(m);
  if ((threadIdx.x & 63) == 0) atomicMax(out, f2ord(m));
}
hipError_t imf_launch_fmax(const float* f, const uint8_t* omega0, long long n,
                           unsigned int* fmax_bits, hipStream_t s) {
  long long blocks = (n + IMF_WG - 1) / IMF_WG;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fmax, dim3((unsigned)blocks), dim3(IMF_WG), 0, s, f, omega0, n, fmax_bits);
  return hipGetLastError();
}

// B = Omega_0 and f > lambda F_max; fbar = f / F_max on B, 0 elsewhere;
// Gamma = B and not Omega, Omega = [rho_Omega > tau]   (Algorithm 1, Eq. gamma)
__global__ void __launch_bounds__(IMF_WG) k_finalize(const float* __restrict__ f,
                                                     const uint8_t* __restrict__ om,
                                                     const void* __restrict__ design, int density,
                                                     long long n,
                                                     const unsigned int* __restrict__ fmax_bits,
                                                     double lambda, double tau,
                                                     float* __restrict__ imf_out,
                                                     float* __restrict__ imf_norm,
                                                     uint8_t* __restrict__ secluded) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double fmax = (double)ord2f(*fmax_bits);
  const float v = f[i];
  const bool inB = om[i] && (double)v > lambda * fmax;
  if (imf_out) imf_out[i] = v;
  if (imf_norm) imf_norm[i] = inB ? (float)((double)v / fmax) : 0.0f;
  if (secluded) {
    const double rho = density ? (double)((const float*)design)[i]
                               : (double)((const uint8_t*)design)[i];
    secluded[i] = (uint8_t)(inB && !(rho > tau));
  }
}
hipError_t imf_launch_finalize(const float* f, const uint8_t* omega0, const void* design,
                               int density, long long n, const unsigned int* fmax_bits,
                               double lambda, double tau, float* imf_out, float* imf_norm,
                               uint8_t* secluded, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n + IMF_WG - 1) / IMF_WG)), dim3(IMF_WG), 0, s,
                     f, omega0, design, density, n, fmax_bits, lambda, tau, imf_out, imf_norm,
                     secluded);
  return hipGetLastError();
}

// masks from stored gamma once theta = lambda F_max is known
__global__ void __launch_bounds__(IMF_WG) k_masks_gamma(const float* __restrict__ gs, int nq,
                                                        const uint8_t* __restrict__ om, int nx,
                                                        int ny, int nz,
                                                        const unsigned int* __restrict__ fmax_bits,
                                                        double lambda, uint64_t* __restrict__ masks) {
  const int words = (nx + 63) >> 6;
  const long long wave = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const long long per_q = (long long)words * ny * nz;
  if (wave >= per_q * nq) return;
  const int q = (int)(wave / per_q);
  const long long r = wave % per_q;
  const int w = (int)(r % words);
  const long long yz = r / words;
  const int x = w * 64 + lane;
  const double theta = lambda * (double)ord2f(*fmax_bits);
  bool b = false;
  if (x < nx) {
    const long long vi = yz * nx + x;
    b = om[vi] && (double)gs[(long long)q * nx * ny * nz + vi] <= theta;
  }
  const unsigned long long bits = __ballot(b);
  if (lane == 0) masks[(long long)q * per_q + yz * words + w] = bits;
}
hipError_t imf_launch_masks_from_gamma(const float* gamma_stack, int nq, const uint8_t* omega0,
                                       int nx, int ny, int nz, const unsigned int* fmax_bits,
                                       double lambda, uint64_t* masks, hipStream_t s) {
  const int words = (nx + 63) >> 6;
  const long long waves = (long long)words * ny * nz * nq;
  const int per = IMF_WG / 64;
  hipLaunchKernelGGL(k_masks_gamma, dim3((unsigned)((waves + per - 1) / per)), dim3(IMF_WG), 0, s,
                     gamma_stack, nq, omega0, nx, ny, nz, fmax_bits, lambda, masks);
  return hipGetLastError();
}
