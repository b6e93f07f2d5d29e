// Exact overlaps (direct correlation, guard-band recheck), the sharp-point
// minimum filter with the running minimum over orientations, the accessible
// masks, and the final normalization / classification of Algorithm 1.
#include "imf_internal.h"

#define Q24 16777216.0



// ---------------------------------------------------------------------------
// prefix sums of rho_O = max(design, fixture) along x, fixed point:
// ps[z][y][x'] = sum_{x < x'} rho_O(x, y, z), x' in [0, nx]   (one wave per row)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(IMF_WG) k_prefix_x(const void* __restrict__ design, int density,
                                                     const uint8_t* __restrict__ fixture, int nx,
                                                     long long rows, long long* __restrict__ ps,
                                                     unsigned int* __restrict__ bad) {
  const long long row = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  long long carry = 0;
  long long* out = ps + row * (nx + 1);
  if (lane == 0) out[0] = 0;
  for (int x0 = 0; x0 < nx; x0 += 64) {
    const int x = x0 + lane;
    long long v = 0;
    bool ok = true;
    if (x < nx) {
      const long long idx = row * nx + x;
      // the design must lie in the value set the fixed-point arithmetic
      // represents exactly: {0, 1} for binary designs, multiples of 2^-24 in
      // [0, 1] for densities (fixture voxels included)
      if (density) {
        const float d = ((const float*)design)[idx];
        const float sc = d * 16777216.0f;  // exact: a power-of-two scaling
        ok = d >= 0.f && d <= 1.f && rintf(sc) == sc;
        v = ok ? (long long)sc : 0;
      } else {
        v = ((const uint8_t*)design)[idx];
        ok = v <= 1;
      }
      if (fixture && fixture[idx]) v = density ? (long long)Q24 : 1;
    }
    if (bad) {
      const unsigned long long m = __ballot(!ok);
      if (lane == 0 && m) atomicAdd(bad, (unsigned)__popcll(m));
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
                               int ny, int nz, long long* ps, unsigned int* bad, hipStream_t s) {
  const long long rows = (long long)ny * nz;
  const int per = IMF_WG / 64;
  hipLaunchKernelGGL(k_prefix_x, dim3((unsigned)((rows + per - 1) / per)), dim3(IMF_WG), 0, s,
                     design, density, fixture, nx, rows, ps, bad);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// direct correlation over the query box (exact)
// ---------------------------------------------------------------------------
// float32 value of an exact overlap e (voxel units): rounded, then moved by
// ulps so that the decision v <= th is the exact one for each known threshold
__device__ __forceinline__ float decided_float(double e, int nth, double th0, double th1) {
  float v = (float)e;
  for (int it = 0; it < 4; it++) {
    bool moved = false;
    for (int k = 0; k < nth; k++) {
      const double th = k ? th1 : th0;
      if (e <= th && (double)v > th) {
        v = nextafterf(v, -INFINITY);
        moved = true;
      } else if (e > th && (double)v <= th) {
        v = nextafterf(v, INFINITY);
        moved = true;
      }
    }
    if (!moved) break;
  }
  return v;
}

__global__ void __launch_bounds__(IMF_WG) k_direct(const imf_orient_desc* __restrict__ desc,
                                                   const long long* __restrict__ ps, int nx,
                                                   int ny, int nz, int density,
                                                   float* __restrict__ g, long long g_stride,
                                                   int nth, double th0, double th1) {
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
  g[q * g_stride + i] =
      density ? decided_float((double)s * (1.0 / Q24), nth, th0, th1) : (float)s;
}

hipError_t imf_launch_direct(const imf_orient_desc* desc, int nq, const long long* ps, int nx,
                             int ny, int nz, int density, float* g, long long g_stride,
                             int max_vol, int nth, double th0, double th1, hipStream_t s) {
  dim3 grid((max_vol + IMF_WG - 1) / IMF_WG, nq);
  hipLaunchKernelGGL(k_direct, grid, dim3(IMF_WG), 0, s, desc, ps, nx, ny, nz, density, g,
                     g_stride, nth, th0, th1);
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
                                                    int nth, double th0, double th1,
                                                    float* __restrict__ g, long long g_stride,
                                                    unsigned int* __restrict__ cellmin,
                                                    long long cell_stride, int cwx, int cwy,
                                                    int cwz, unsigned int* __restrict__ err_bits) {
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
      if (err_bits) {  // the float32 transform's error at this overlap
        const float er = (float)fabs((double)g[(long long)f.x * g_stride + i] - e);
        if (__float_as_uint(er) > __atomic_load_n(err_bits, __ATOMIC_RELAXED))
          atomicMax(err_bits, __float_as_uint(er));
      }
      v = decided_float(e, nth, th0, th1);
    }
    g[(long long)f.x * g_stride + i] = v;
    if (cellmin) {  // the corrected value may lie below its cell's minimum
      const int cdx = (d.box_dim[0] + cwx - 1) / cwx + 1;
      const int cdy = (d.box_dim[1] + cwy - 1) / cwy + 1;
      atomicMin(&cellmin[(long long)f.x * cell_stride +
                         ((long long)(bz / cwz) * cdy + by / cwy) * cdx + bx / cwx],
                f2ord(v));
    }
  }
}

hipError_t imf_launch_recheck(const imf_orient_desc* desc, const long long* ps, int nx, int ny, int nz, int density,
                              const int* flag_cnt, const int2* flags, int flag_cap,
                              int nth, double th0, double th1, float* g, long long g_stride,
                              unsigned int* cellmin, long long cell_stride, int cwx, int cwy,
                              int cwz, unsigned int* err_bits, hipStream_t s) {
  const int blocks = flag_cap < 256 * 1024 ? (flag_cap + IMF_WG - 1) / IMF_WG : 1024;
  hipLaunchKernelGGL(k_recheck, dim3(blocks > 0 ? blocks : 1), dim3(IMF_WG), 0, s, desc, ps,
                     nx, ny, nz, density, flag_cnt, flags, flag_cap, nth, th0, th1, g,
                     g_stride, cellmin, cell_stride, cwx, cwy, cwz, err_bits);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sharp-point minimum (Eq. imf_2): gamma(x) = min over runs of S of the window
// minimum of g along the run axis.  Level s of the sparse table holds
// min g[p, p + 2^s) along the axis; a run of length l reads two level-s
// windows, s = floor(log2 l).  Levels between 1 and the highest are formed
// for the recurrence but stored only where some run of the orientation reads
// them (lvl_used of the descriptor).
// ---------------------------------------------------------------------------
// All sparse-table levels of one orientation in one pass: lines along the run
// axis are staged in LDS (ping-pong), each level is formed there and written
// out.  A workgroup holds LT lines of length m = box extent along the axis;
// for the x axis the lines are rows, otherwise LT consecutive x columns.
#define LVL_LT 16
#define LS_MAXL 6  // levels handled by the register forms
__global__ void __launch_bounds__(IMF_WG) k_levels(const imf_orient_desc* __restrict__ desc,
                                                   const float* __restrict__ g,
                                                   long long g_stride, float* __restrict__ lvl,
                                                   long long lvl_stride, int nlvl) {
  extern __shared__ float lds[];
  const int q = blockIdx.z;
  const imf_orient_desc& d = desc[q];
  const int ax = d.s_axis;
  if (ax > 2) return;  // runs along a lattice vector: k_levels_vstream
  const int mx = d.box_dim[0], my = d.box_dim[1], mz = d.box_dim[2];
  const int m = d.box_dim[ax];
  const long long sa = ax == 0 ? 1 : (ax == 1 ? (long long)mx : (long long)mx * my);
  {
    const int nl_q = d.nlvl < nlvl ? d.nlvl : nlvl;
    if (nl_q >= 1 && nl_q <= LS_MAXL) return;  // k_levels_stream / k_levels_x
  }
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
      if (ok && ((d.lvl_used >> (s - 1)) & 1u)) dst[gi] = v;
    }
    __syncthreads();
    float* tmp = A;
    A = B;
    B = tmp;
  }
}

// Sparse-table levels along y or z lines, streamed: one wave per 64
// consecutive x of a line, walking the line from its end (coalesced 256-byte
// loads and stores, no LDS).  Level s at position i is
// min(L_{s-1}(i), L_{s-1}(i + 2^(s-1))), with +inf past the line's end (the
// same values as k_levels), so each level needs the previous level's value
// 2^(s-1) steps back: delay lines in registers, with the loop unrolled by the
// longest delay so that every slot index is a compile-time constant.  The
// four waves of a workgroup (neighbouring 64-x chunks) walk in step, a
// barrier per unrolled group of steps, so that their loads and stores of one
// step reach memory together: the level pass of 256^3 x 130 takes 15.7 ms
// instead of 16.6 with the waves drifting apart (two waves in step: 16.0;
// eight, a workgroup per CU at these registers: 19.0).
template <int NL>
__device__ __forceinline__ void levels_stream_line(const float* __restrict__ src,
                                                   float* __restrict__ dst, long long g_stride,
                                                   int m, long long sa, long long base, bool ok,
                                                   unsigned used) {
  // steps per group (a multiple of every delay 2^(s-1)): twice the longest
  // delay below six levels, so more loads are in flight per barrier without
  // raising the registers the six-level form sets (256^3 x 130: level pass
  // 15.7 -> 14.9 ms; 32 steps for every level count: 14.9 as well)
  constexpr int U = NL < 6 ? 1 << NL : 1 << (NL - 1);
  float D[(1 << NL) - 1];  // level s - 1 delays at [2^(s-1) - 1, 2^s - 1)
#pragma unroll
  for (int k = 0; k < (1 << NL) - 1; k++) D[k] = INFINITY;
  const int nb = (m + U - 1) / U;
  for (int b = nb - 1; b >= 0; b--) {
    __syncthreads();  // the workgroup's lines in step: neighbouring stores at once
    float gv[U];
#pragma unroll
    for (int j = 0; j < U; j++) {
      const int i = b * U + (U - 1 - j);
      gv[j] = (ok && i < m) ? src[base + (long long)i * sa] : INFINITY;
    }
#pragma unroll
    for (int j = 0; j < U; j++) {
      const int i = b * U + (U - 1 - j);
      float v = gv[j];
#pragma unroll
      for (int s = 1; s <= NL; s++) {
        const int slot = ((1 << (s - 1)) - 1) + (j & ((1 << (s - 1)) - 1));
        const float prev = D[slot];
        D[slot] = v;
        v = fminf(v, prev);
        if (((used >> (s - 1)) & 1u) && ok && i < m)
          dst[(long long)(s - 1) * g_stride + base + (long long)i * sa] = v;
      }
    }
  }
}

__global__ void __launch_bounds__(IMF_WG) k_levels_stream(const imf_orient_desc* __restrict__ desc,
                                                          const float* __restrict__ g,
                                                          long long g_stride,
                                                          float* __restrict__ lvl,
                                                          long long lvl_stride, int nlvl) {
  const int q = blockIdx.y;
  const imf_orient_desc& d = desc[q];
  const int ax = d.s_axis;
  const int nl_q = d.nlvl < nlvl ? d.nlvl : nlvl;
  if (ax == 0 || ax > 2 || nl_q < 1 || nl_q > LS_MAXL) return;  // left to the other forms
  const int mx = d.box_dim[0], my = d.box_dim[1], mz = d.box_dim[2];
  const int nxw = (mx + 63) / 64;
  const long long w = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  long long o = w / nxw;
  const bool wave_in = o < (ax == 1 ? mz : my);
  if (!wave_in) o = 0;  // walks with its workgroup, storing nothing
  const int x = (int)(w % nxw) * 64 + (threadIdx.x & 63);
  const bool ok = wave_in && x < mx;
  const long long base = ax == 1 ? o * my * mx + x : o * mx + x;
  const long long sa = ax == 1 ? (long long)mx : (long long)mx * my;
  const int m = d.box_dim[ax];
  const float* src = g + q * g_stride;
  float* dst = lvl + q * lvl_stride;
  const unsigned used = d.lvl_used;
  switch (nl_q) {
    case 1: levels_stream_line<1>(src, dst, g_stride, m, sa, base, ok, used); break;
    case 2: levels_stream_line<2>(src, dst, g_stride, m, sa, base, ok, used); break;
    case 3: levels_stream_line<3>(src, dst, g_stride, m, sa, base, ok, used); break;
    case 4: levels_stream_line<4>(src, dst, g_stride, m, sa, base, ok, used); break;
    case 5: levels_stream_line<5>(src, dst, g_stride, m, sa, base, ok, used); break;
    default: levels_stream_line<6>(src, dst, g_stride, m, sa, base, ok, used); break;
  }
}

// Levels along x lines (rows, contiguous): one wave per row, 64 positions per
// step, two chunks in registers (a = positions c..c+63, b = the next 64).
// Level s of a needs level s-1 at lane + 2^(s-1), from a or (past lane 63)
// from b; b's level s-1 is needed only at lanes < 2^(s-1), which stay inside
// b for s <= 6.  Coalesced 256-byte loads and stores, no LDS.
__global__ void __launch_bounds__(IMF_WG) k_levels_x(const imf_orient_desc* __restrict__ desc,
                                                     const float* __restrict__ g,
                                                     long long g_stride, float* __restrict__ lvl,
                                                     long long lvl_stride, int nlvl) {
  const int q = blockIdx.y;
  const imf_orient_desc& d = desc[q];
  const int nl_q = d.nlvl < nlvl ? d.nlvl : nlvl;
  if (d.s_axis != 0 || nl_q < 1 || nl_q > LS_MAXL) return;  // left to the other forms
  const int mx = d.box_dim[0];
  const long long rows = (long long)d.box_dim[1] * d.box_dim[2];
  const long long row = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int lane = threadIdx.x & 63;
  const float* src = g + q * g_stride + row * mx;
  float* dst = lvl + q * lvl_stride + row * mx;
  float b = lane < mx ? src[lane] : INFINITY;
  for (int c = 0; c < mx; c += 64) {
    float a = b;
    b = c + 64 + lane < mx ? src[c + 64 + lane] : INFINITY;
    float bb = b;
    for (int s = 1; s <= nl_q; s++) {
      const int h = 1 << (s - 1);
      const int src_lane = (lane + h) & 63;
      const float xa = __shfl(a, src_lane);
      const float xb = __shfl(bb, src_lane);
      a = fminf(a, lane + h < 64 ? xa : xb);
      bb = fminf(bb, lane + h < 64 ? xb : INFINITY);  // valid where it is used
      if (((d.lvl_used >> (s - 1)) & 1u) && c + lane < mx)
        dst[(long long)(s - 1) * g_stride + c + lane] = a;
    }
  }
}

// Levels along the lines of a lattice vector v (runs of S along v, Sec. 2.1.3
// computes the minimum over S, any exact cover of S by runs gives it): level
// s at t is min_{j < 2^s} g(t + j v), +inf outside the box.  One wave per 64
// seeds of consecutive x (imf_vlines), each lane walking its line from the far
// end with the register delay lines of levels_stream_line; steps past a
// lane's part of the box load +inf and store nothing.  Loads and stores at
// one step are 64 consecutive x: coalesced.  The workgroup's waves walk the
// union of their step ranges in step (as in levels_stream_line).
__device__ __forceinline__ void vline_range(int c0, int dv, int m, int S, int& lo, int& hi) {
  // steps s in [0, S) with 0 <= c0 + s dv < m
  if (dv == 0) {
    lo = 0;
    hi = (c0 >= 0 && c0 < m) ? S : 0;
  } else if (dv > 0) {
    lo = max(0, imf_ceil_div(-c0, dv));
    hi = min(S, imf_floor_div(m - 1 - c0, dv) + 1);
  } else {
    lo = max(0, imf_floor_div(c0 - m, -dv) + 1);
    hi = min(S, imf_floor_div(c0, -dv) + 1);
  }
}

template <int NL>
__device__ __forceinline__ void levels_vstream_line(const float* __restrict__ src,
                                                    float* __restrict__ dst, long long g_stride,
                                                    long long idx0, long long step, int wlo,
                                                    int whi, int llo, int lhi, unsigned used) {
  // steps per group (a multiple of every delay 2^(s-1)): twice the longest
  // delay below six levels, so more loads are in flight per barrier without
  // raising the registers the six-level form sets (256^3 x 130: level pass
  // 15.7 -> 14.9 ms; 32 steps for every level count: 14.9 as well)
  constexpr int U = NL < 6 ? 1 << NL : 1 << (NL - 1);
  float D[(1 << NL) - 1];
#pragma unroll
  for (int k = 0; k < (1 << NL) - 1; k++) D[k] = INFINITY;
  const int nb = (whi - wlo + U - 1) / U;
  for (int b = nb - 1; b >= 0; b--) {
    __syncthreads();  // the workgroup's lines in step: neighbouring stores at once
    float gv[U];
#pragma unroll
    for (int j = 0; j < U; j++) {
      const int i = wlo + b * U + (U - 1 - j);
      gv[j] = (i >= llo && i < lhi) ? src[idx0 + (long long)i * step] : INFINITY;
    }
#pragma unroll
    for (int j = 0; j < U; j++) {
      const int i = wlo + b * U + (U - 1 - j);
      const bool ok = i >= llo && i < lhi;
      float v = gv[j];
#pragma unroll
      for (int s = 1; s <= NL; s++) {
        const int slot = ((1 << (s - 1)) - 1) + (j & ((1 << (s - 1)) - 1));
        const float prev = D[slot];
        D[slot] = v;
        v = fminf(v, prev);
        if (((used >> (s - 1)) & 1u) && ok)
          dst[(long long)(s - 1) * g_stride + idx0 + (long long)i * step] = v;
      }
    }
  }
}

__global__ void __launch_bounds__(IMF_WG) k_levels_vstream(const imf_orient_desc* __restrict__ desc,
                                                           const float* __restrict__ g,
                                                           long long g_stride,
                                                           float* __restrict__ lvl,
                                                           long long lvl_stride, int nlvl) {
  const int q = blockIdx.y;
  const imf_orient_desc& d = desc[q];
  const int nl_q = d.nlvl < nlvl ? d.nlvl : nlvl;
  if (d.s_axis != 3 || nl_q < 1 || nl_q > LS_MAXL) return;
  const int v[3] = {d.sv[0], d.sv[1], d.sv[2]};
  const int dim[3] = {d.box_dim[0], d.box_dim[1], d.box_dim[2]};
  const imf_vlines L = imf_vlines_of(v, dim);
  long long w = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  const bool wave_in = w < L.waves;
  if (!wave_in) w = 0;  // walks with its workgroup, storing nothing
  const int lane = threadIdx.x & 63;
  const int xc = (int)(w % L.nxc);
  const long long rest = w / L.nxc;
  const int b0 = L.lob + (int)(rest % L.nb0);
  const int r = (int)(rest / L.nb0);
  const int a0 = v[L.a] > 0 ? r : dim[L.a] - 1 - r;
  const int xs = L.lox + xc * 64 + lane;
  int lo, hi, l2, h2;
  vline_range(xs, v[0], dim[0], L.S, lo, hi);
  vline_range(a0, v[L.a], dim[L.a], L.S, l2, h2);
  lo = max(lo, l2);
  hi = min(hi, h2);
  vline_range(b0, v[L.b], dim[L.b], L.S, l2, h2);
  lo = max(lo, l2);
  hi = min(hi, h2);
  if (!wave_in) hi = lo;
  // the wave's steps: the union of its lanes' (contiguous) ranges
  int wlo = lo < hi ? lo : 0x7fffffff, whi = lo < hi ? hi : -1;
  for (int o = 32; o > 0; o >>= 1) {
    wlo = min(wlo, __shfl_xor(wlo, o));
    whi = max(whi, __shfl_xor(whi, o));
  }
  {  // the workgroup's waves walk the union of their ranges in step
    __shared__ int rlo[IMF_WG / 64], rhi[IMF_WG / 64];
    if (lane == 0) {
      rlo[threadIdx.x >> 6] = wlo;
      rhi[threadIdx.x >> 6] = whi;
    }
    __syncthreads();
    for (int k = 0; k < IMF_WG / 64; k++) {
      wlo = min(wlo, rlo[k]);
      whi = max(whi, rhi[k]);
    }
  }
  if (wlo >= whi) return;  // uniform over the workgroup
  int c[3];
  c[0] = xs;
  c[L.a] = a0;
  c[L.b] = b0;
  const long long idx0 = c[0] + (long long)dim[0] * (c[1] + (long long)dim[1] * c[2]);
  const long long step = v[0] + (long long)dim[0] * (v[1] + (long long)dim[1] * v[2]);
  const float* src = g + q * g_stride;
  float* dst = lvl + q * lvl_stride;
  const unsigned used = d.lvl_used;
  switch (nl_q) {
    case 1: levels_vstream_line<1>(src, dst, g_stride, idx0, step, wlo, whi, lo, hi, used); break;
    case 2: levels_vstream_line<2>(src, dst, g_stride, idx0, step, wlo, whi, lo, hi, used); break;
    case 3: levels_vstream_line<3>(src, dst, g_stride, idx0, step, wlo, whi, lo, hi, used); break;
    case 4: levels_vstream_line<4>(src, dst, g_stride, idx0, step, wlo, whi, lo, hi, used); break;
    case 5: levels_vstream_line<5>(src, dst, g_stride, idx0, step, wlo, whi, lo, hi, used); break;
    default: levels_vstream_line<6>(src, dst, g_stride, idx0, step, wlo, whi, lo, hi, used); break;
  }
}

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

void imf_block_dims(int shape, int& wx, int& wy, int& wz) {
  switch (shape) {
    case 1: wx = 32; wy = 2; wz = 1; break;
    case 2: wx = 16; wy = 2; wz = 2; break;
    case 3: wx = 16; wy = 4; wz = 1; break;
    case 4: wx = 8; wy = 4; wz = 2; break;
    default: wx = 64; wy = 1; wz = 1; break;
  }
}

__device__ __forceinline__ float wave_min_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}

// ---------------------------------------------------------------------------
// branch and bound, part 1: footprints and cell minima
// ---------------------------------------------------------------------------
// Footprint of one orientation: the offsets (in cells of the block shape) of
// every cell that meets block - S, the same for every block because blocks and
// cells are aligned (t - box_lo = W b + i + e with e = kmax - k >= 0, so the
// cell is b + floor((i + e) / W), i in [0, W)).  One workgroup per orientation.
#define FP_BITS 65536
__global__ void __launch_bounds__(IMF_WG) k_footprint(const imf_orient_desc* __restrict__ desc,
                                                      int nx, int ny, int nz, int WX, int WY,
                                                      int WZ, int* __restrict__ fp, int fp_cap) {
  __shared__ unsigned int bm[FP_BITS / 32];
  __shared__ int cnt;
  const int q = blockIdx.x;
  const imf_orient_desc& d = desc[q];
  int* out = fp + (long long)q * (fp_cap + 1);
  const int n[3] = {nx, ny, nz};
  const int W[3] = {WX, WY, WZ};
  int kmax[3], fd[3], cd[3];
  for (int a = 0; a < 3; a++) {
    kmax[a] = -d.box_lo[a];
    const int E = d.box_dim[a] - n[a] + 1;  // extent of S
    fd[a] = (E - 1 + W[a] - 1) / W[a] + 1;
    cd[a] = (d.box_dim[a] + W[a] - 1) / W[a] + 1;  // one spare cell: padded blocks
  }
  const long long nbits = (long long)fd[0] * fd[1] * fd[2];
  if (nbits > FP_BITS) {  // no bound for this orientation: nothing is skipped
    if (threadIdx.x == 0) out[0] = -1;
    return;
  }
  for (int i = threadIdx.x; i < FP_BITS / 32; i += IMF_WG) bm[i] = 0;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < d.n_sruns; r += IMF_WG) {
    const imf_run u = d.sruns[r];
    for (int j = 0; j < u.len; j++) {
      const int k[3] = {u.x + j * d.sv[0], u.y + j * d.sv[1], u.z + j * d.sv[2]};
      int lo[3], hi[3];
      for (int a = 0; a < 3; a++) {
        const int e = kmax[a] - k[a];
        lo[a] = e / W[a];
        hi[a] = (e + W[a] - 1) / W[a];
      }
      for (int dz = lo[2]; dz <= hi[2]; dz++)
        for (int dy = lo[1]; dy <= hi[1]; dy++)
          for (int dx = lo[0]; dx <= hi[0]; dx++) {
            const int b = (dz * fd[1] + dy) * fd[0] + dx;
            atomicOr(&bm[b >> 5], 1u << (b & 31));
          }
    }
  }
  __syncthreads();
  for (int wi = threadIdx.x; wi < (int)((nbits + 31) / 32); wi += IMF_WG) {
    unsigned int m = bm[wi];
    while (m) {
      const int bit = __ffs(m) - 1;
      m &= m - 1;
      const int b = wi * 32 + bit;
      const int dx = b % fd[0], dy = (b / fd[0]) % fd[1], dz = b / (fd[0] * fd[1]);
      const int slot = atomicAdd(&cnt, 1);
      if (slot < fp_cap) out[1 + slot] = (dz * cd[1] + dy) * cd[0] + dx;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) out[0] = cnt <= fp_cap ? cnt : -1;
}

// minimum of g over each cell of the block shape (cells aligned to the box).
// One wave per (64-x segment, cell row cy, CM_CZ cell planes): lanes read
// consecutive x, reduce in groups of WX lanes and combine the WY x WZ rows of a
// cell.
#define CM_CZ 8
__global__ void __launch_bounds__(IMF_WG) k_cellmin(const imf_orient_desc* __restrict__ desc,
                                                    const float* __restrict__ g,
                                                    long long g_stride, int WX, int WY, int WZ,
                                                    unsigned int* __restrict__ cellmin,
                                                    long long cell_stride) {
  const int q = blockIdx.y;
  const imf_orient_desc& d = desc[q];
  const int mx = d.box_dim[0], my = d.box_dim[1], mz = d.box_dim[2];
  // one spare cell per axis (all +inf) for blocks that pad past the grid
  const int cdx = (mx + WX - 1) / WX + 1, cdy = (my + WY - 1) / WY + 1;
  const int cdz = (mz + WZ - 1) / WZ + 1;
  const int lane = threadIdx.x & 63;
  const int segs = (cdx * WX + 63) / 64;
  const int czc = (cdz + CM_CZ - 1) / CM_CZ;
  const long long wave = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  if (wave >= (long long)segs * cdy * czc) return;
  const int sg = (int)(wave % segs);
  const long long rc = wave / segs;
  const int cy = (int)(rc % cdy), cz0 = (int)(rc / cdy) * CM_CZ;
  const int x = sg * 64 + lane;
  const int cx = x / WX;
  const float* gq = g + q * g_stride;
  unsigned int* out = cellmin + q * cell_stride;
  const int y0 = cy * WY;
  // the rows of a cell (WY * WZ <= 8 for every block shape) four at a time,
  // those of the CM_CZ cell planes together, so the loads are in flight
  // together
  float mm[CM_CZ];
#pragma unroll
  for (int c = 0; c < CM_CZ; c++) mm[c] = INFINITY;
  for (int r0 = 0; r0 < WY * WZ; r0 += 4) {
    float v[CM_CZ][4];
#pragma unroll
    for (int c = 0; c < CM_CZ; c++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int rr = r0 + r;
        const int cz = cz0 + c, z = cz * WZ + rr / WY, y = y0 + rr % WY;
        const bool ok = rr < WY * WZ && cz < cdz && z < mz && y < my && x < mx;
        v[c][r] = ok ? gq[((long long)z * my + y) * mx + x] : INFINITY;
      }
#pragma unroll
    for (int c = 0; c < CM_CZ; c++)
      mm[c] = fminf(mm[c], fminf(fminf(v[c][0], v[c][1]), fminf(v[c][2], v[c][3])));
  }
#pragma unroll
  for (int c = 0; c < CM_CZ; c++) {
    const int cz = cz0 + c;
    float m = mm[c];
    for (int o = 1; o < WX; o <<= 1) m = fminf(m, __shfl_xor(m, o));
    if ((lane % WX) == 0 && cx < cdx && cz < cdz)
      out[((long long)cz * cdy + cy) * cdx + cx] = f2ord(m);
  }
}

__global__ void k_fill(float* f, long long n, float v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    f[i] = v;
}
__global__ void k_fill_u32(unsigned int* p, long long n, unsigned int v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
// ---------------------------------------------------------------------------
// Sharp-point minimum of ONE orientation (Eq. imf_2).  The output is cut into
// blocks of WX x WY x WZ voxels, one wave per block; f is updated in place (one
// orientation per launch, so every voxel has a single writer).
//
// Logical block order: bricks of 128 x 16 x 16 voxels (x chunk slowest, then z,
// y fastest), blocks inside a brick x, y, z.  Consecutive logical indices are
// close in space, so the waves one XCD runs at a time read overlapping windows
// of g and its levels from that XCD's L2.
// ---------------------------------------------------------------------------
#define MF_LDS_RUNS IMF_MF_LDS_RUNS
#ifndef MF_GRP
// runs per group of the gather loop (a barrier per group when the waves go in
// step), i.e. 8 gathers: two windows per run, or 2 * MF_GRP runs of
// power-of-two length (the host splits runs into such windows).  Eight
// 16 x 2 x 2 blocks making 8 gathers touch ~160 lines, within the 256 lines of
// the L1, so the later waves of a group still find them there
#define MF_GRP 4
#endif
struct mf_run {
  long long off;   // element offset from g of the first window (level and far end folded in)
  long long off2;  // the second (overlapping) window
};

template <int WX>
__device__ __forceinline__ void mf_store_chunk(uint64_t* row_words, int bx, uint64_t chunk) {
  if (WX == 64) row_words[bx] = chunk;
  else if (WX == 32) ((uint32_t*)row_words)[bx] = (uint32_t)chunk;
  else if (WX == 16) ((uint16_t*)row_words)[bx] = (uint16_t)chunk;
  else ((uint8_t*)row_words)[bx] = (uint8_t)chunk;
}

// max over the block maxima of f (an upper bound of F_max: the threshold
// lambda F_max of two-phase masks is at most lambda times this)
__global__ void __launch_bounds__(IMF_WG) k_blockmax(const float* __restrict__ fb, long long n,
                                                     unsigned int* __restrict__ out) {
  __shared__ float red[IMF_WG / 64];
  float m = -INFINITY;
  for (long long i = (long long)blockIdx.x * IMF_WG + threadIdx.x; i < n;
       i += (long long)gridDim.x * IMF_WG)
    m = fmaxf(m, fb[i]);
  m = wave_max_f(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < IMF_WG / 64; i++) m = fmaxf(m, red[i]);
    atomicMax(out, f2ord(m));
  }
}

// Branch and bound, part 2: lower bound of gamma over every block of one
// orientation (the minimum of the cell minima over the footprint), the skip
// decision and the compacted list of the blocks left to compute.  One thread
// per logical block; the footprint offsets are the same for every block and
// are staged in LDS, so neighbouring lanes read neighbouring cells.  A block is
// skipped when its bound is >= its maximum of f (f cannot decrease) and, when
// masks are produced, above the bound on the mask threshold (no mask bit).
#define BND_CHUNK 2048
template <int WX, int WY, int WZ>
__global__ void __launch_bounds__(IMF_WG) k_bound(imf_min_args a, int qi) {
  __shared__ int fpl[BND_CHUNK];
  const mf_geom G(WX, WY, WZ, a.nx, a.ny, a.nz);
  const imf_orient_desc& d = a.desc[qi];
  const int* fpg = a.fp + (long long)qi * (a.fp_cap + 1);
  const int nfp = fpg[0];
  const long long lg = (long long)blockIdx.x * IMF_WG + threadIdx.x;
  int bx = 0, by = 0, bz = 0;
  const bool live = lg < G.nlog && G.block(lg, bx, by, bz);
  const int cdx = (d.box_dim[0] + WX - 1) / WX + 1, cdy = (d.box_dim[1] + WY - 1) / WY + 1;
  const long long cb = ((long long)bz * cdy + by) * cdx + bx;
  const unsigned int* cm = a.cellmin + qi * a.cell_stride;
  // minimum in the order-preserving integer map of the cell minima
  unsigned int lbo = nfp < 0 ? 0u : IMF_ORD_INF;  // no footprint: no bound
  for (int c0 = 0; c0 < nfp; c0 += BND_CHUNK) {
    const int n = min(BND_CHUNK, nfp - c0);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += IMF_WG) fpl[i] = fpg[1 + c0 + i];
    __syncthreads();
    if (live) {
      // 32-bit cell indices (an orientation's cell grid is far below 2^32)
      // off the uniform base: one register per load, 16 loads in flight
      const unsigned cbu = (unsigned)cb;
#pragma unroll 16
      for (int i = 0; i < n; i++) lbo = min(lbo, cm[cbu + (unsigned)fpl[i]]);
    }
  }
  const float lb = nfp < 0 ? -INFINITY : ord2f(lbo);
  const long long blk = ((long long)bz * G.nby + by) * G.nbx + bx;
  const float fb = live ? a.fblock[blk] : -INFINITY;
  // f: no voxel's running minimum can fall (by more than fmargin below it:
  // the candidates of an exact F_max need every gamma within 2E of f)
  bool sk = live && (a.fmargin > 0 ? (double)lb > (double)fb + a.fmargin : lb >= fb);
  // masks at a known threshold (exact after the recheck): no bit
  if (a.masks_on) sk = sk && (double)lb > a.theta;
  // masks or B at lambda F_max: F_max is at most the current maximum of f
  // (plus E), so above that bound (plus E) no bit is set and no overlap of the
  // band reaches the block
  if (a.gamma_stack) {
    double thu = a.theta_lambda * ((double)ord2f(*a.fmax_up) + a.e_theta) + a.e_theta;
    if (a.e_theta > 0) thu *= 1.0 + 1e-12;
    sk = sk && (double)lb > thu;
  }
  const unsigned long long mw = __ballot(live && !sk);
  if ((threadIdx.x & 63) == 0 && lg < G.nlog) {
    a.wmask[(long long)qi * a.wstride + (lg >> 6)] = mw;
    if (a.keepbits) a.keepbits[(long long)d.out_q * a.wstride + (lg >> 6)] = mw;
  }
}

// Branch and bound, part 3: order-preserving compaction of the blocks left to
// compute.  One workgroup scans the per-wave counts of the bound pass
// (exclusive offsets and the total); the scatter pass then writes each kept
// block at its offset, so the list keeps the logical (spatially coherent)
// order that the minimum pass relies on for L2 reuse.
__global__ void __launch_bounds__(1024) k_scan_masks(imf_min_args a, int qi, int nw) {
  __shared__ int wsum[16];
  __shared__ int carry;
  const unsigned long long* m = a.wmask + (long long)qi * a.wstride;
  int* off = a.woff + (long long)qi * a.wstride;
  // the offsets again per request orientation, for the compact gamma stack
  int* koff = a.koff ? a.koff + (long long)a.desc[qi].out_q * a.wstride : nullptr;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nw; c0 += 4096) {
    int v[4], t = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int i = c0 + threadIdx.x * 4 + j;
      v[j] = i < nw ? __popcll(m[i]) : 0;
      t += v[j];
    }
    int x = t;  // inclusive scan over the wave
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    if (wv == 0) {
      int w = lane < 16 ? wsum[lane] : 0;
      for (int o = 1; o < 16; o <<= 1) {
        const int y = __shfl_up(w, o);
        if (lane >= o) w += y;
      }
      if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    int ex = carry + (wv > 0 ? wsum[wv - 1] : 0) + x - t;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int i = c0 + threadIdx.x * 4 + j;
      if (i < nw) {
        off[i] = ex;
        if (koff) koff[i] = ex;
      }
      ex += v[j];
    }
    __syncthreads();
    if (threadIdx.x == 1023) carry = ex;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.count[qi] = carry;
    if (a.kept) a.kept[a.q0 + qi] = carry;
    if (a.gbase) {  // this orientation's slots in the compact gamma stack
      const unsigned long long need = 64ull * (unsigned long long)carry;
      const unsigned long long base = atomicAdd(a.gused, need);
      const bool over = base + need > (unsigned long long)a.gcap;
      a.gbase[a.desc[qi].out_q] = over ? -1LL : (long long)base;
      if (over) atomicOr(a.gover, 1u);
    }
  }
}

template <int WX, int WY, int WZ>
__global__ void __launch_bounds__(IMF_WG) k_scatter(imf_min_args a, int qi) {
  const mf_geom G(WX, WY, WZ, a.nx, a.ny, a.nz);
  const long long lg = (long long)blockIdx.x * IMF_WG + threadIdx.x;
  if (lg >= G.nlog) return;
  const unsigned long long m = a.wmask[(long long)qi * a.wstride + (lg >> 6)];
  const int lane = threadIdx.x & 63;
  if (!((m >> lane) & 1ull)) return;
  int bx, by, bz;
  G.block(lg, bx, by, bz);
  const int o = a.woff[(long long)qi * a.wstride + (lg >> 6)] + __popcll(m & ((1ull << lane) - 1));
  // packed block coordinates (bx < 1024, by, bz < 2048)
  a.list[(long long)qi * a.list_stride + o] =
      (int)((unsigned)bx | ((unsigned)by << 10) | ((unsigned)bz << 21));
}

// The minimum over the sharp points for one block (one wave): gathers of the
// sparse-table levels at the run offsets staged in LDS, 8 independent gathers
// in flight per wave between the barriers of the in-step walk; then the
// running minimum f, the gamma stack, the block maximum of f (branch and
// bound) and the mask chunk.
template <int WX, int WY, int WZ, bool SYNC = false>
__device__ __forceinline__ void mf_block(const imf_min_args& a, const imf_orient_desc& d,
                                         const mf_run* rr, int qi, int bx, int by, int bz,
                                         long long blk, bool act = true,
                                         long long slot = -1, long long gb = -1) {
  const int nr = d.n_sruns;
  const long long sx = 1, sy = d.box_dim[0], sz = (long long)d.box_dim[0] * d.box_dim[1];
  const long long sa = d.sv[0] * sx + d.sv[1] * sy + d.sv[2] * sz;  // box offset of sv
  const int lane = threadIdx.x & 63;
  const int lx = lane % WX, ly = (lane / WX) % WY, lz = lane / (WX * WY);
  const int x = bx * WX + lx, y = by * WY + ly, z = bz * WZ + lz;
  const bool valid = x < a.nx && y < a.ny && z < a.nz;
  const long long vi = ((long long)z * a.ny + y) * a.nx + x;
  const float* g = a.g + qi * a.g_stride;
  const float* lv = a.lvl + qi * a.lvl_stride - a.g_stride;  // level s at lv + s * g_stride
  const int nl = nr < MF_LDS_RUNS ? nr : MF_LDS_RUNS;
  // translation t = x - k; box index of t for k = 0 (invalid lanes read a
  // clamped in-box position and are discarded)
  const int xc = x < a.nx ? x : a.nx - 1, yc = y < a.ny ? y : a.ny - 1;
  const int zc = z < a.nz ? z : a.nz - 1;
  const long long base = (long long)(xc - d.box_lo[0]) + (long long)(yc - d.box_lo[1]) * sy +
                         (long long)(zc - d.box_lo[2]) * sz;
  float gam = INFINITY;
  int r = 0;
  const float* gq = a.g + qi * a.g_stride;  // run offsets are relative to g (levels included)
  // runs of power-of-two length come first: one window each
  const int n1 = d.n_sruns1 < nl ? d.n_sruns1 : nl;
  for (; r + 2 * MF_GRP <= n1; r += 2 * MF_GRP) {
    if (act) {
      float v[2 * MF_GRP];
#pragma unroll
      for (int j = 0; j < 2 * MF_GRP; j++) v[j] = gq[base + rr[r + j].off];
#pragma unroll
      for (int j = 0; j < 2 * MF_GRP; j++) gam = fminf(gam, v[j]);
    }
    if (SYNC) __syncthreads();  // the workgroup's waves gather the same runs together
  }
  if (act)
    for (; r < n1; r++) gam = fminf(gam, gq[base + rr[r].off]);
  else
    r = n1;
  for (; r + MF_GRP <= nl; r += MF_GRP) {
    if (act) {
      float v[2 * MF_GRP];
#pragma unroll
      for (int j = 0; j < MF_GRP; j++) {
        const mf_run u = rr[r + j];
        v[2 * j] = gq[base + u.off];
        v[2 * j + 1] = gq[base + u.off2];
      }
#pragma unroll
      for (int j = 0; j < MF_GRP; j++) gam = fminf(gam, fminf(v[2 * j], v[2 * j + 1]));
    }
    if (SYNC) __syncthreads();
  }
  if (!act) return;
  for (; r < nl; r++) {
    const mf_run u = rr[r];
    gam = fminf(gam, fminf(gq[base + u.off], gq[base + u.off2]));
  }
  for (r = MF_LDS_RUNS; r < nr; r++) {  // beyond the LDS capacity: read the runs directly
    const imf_run u = d.sruns[r];
    const int sl = ilog2(u.len);
    const float* L = sl == 0 ? g : lv + (long long)sl * a.g_stride;
    const long long p = base - (u.x * sx + u.y * sy + u.z * sz) - (long long)(u.len - 1) * sa;
    gam = fminf(gam, fminf(L[p], L[p + (long long)(u.len - (1 << sl)) * sa]));
  }
  float fnew = -INFINITY;
  if (valid) {
    const float fo = a.f[vi];
    fnew = fminf(fo, gam);
    if (gam < fo) a.f[vi] = gam;
    if (a.gamma_stack) {
      if (!a.gbase) {
        a.gamma_stack[(long long)d.out_q * a.nx * a.ny * a.nz + vi] = gam;
      } else if (gb >= 0 && slot >= 0) {  // compact: the block's slot is its place in
        a.gamma_stack[gb + slot * 64 + lane] = gam;  // the list, from the orientation's base
      }
    }
  }
  if (a.bnb) {
    fnew = wave_max_f(fnew);
    if (lane == 0) a.fblock[blk] = fnew;
  }
  if (a.masks_on) {
    const bool om = valid && a.omega0[vi];
    const unsigned long long bits = __ballot(om && (double)gam <= a.theta);
    if (lx == 0 && y < a.ny && z < a.nz) {
      const int words = (a.nx + 63) >> 6;
      const int row = ly + WY * lz;
      uint64_t* row_words = a.masks + ((long long)d.out_q * a.nz + z) * a.ny * words +
                            (long long)y * words;
      mf_store_chunk<WX>(row_words, bx,
                         WX == 64 ? bits : (bits >> (row * WX)) & ((1ull << WX) - 1));
    }
  }
}

// runs of S as element offsets from g of this orientation, for k = 0: off =
// the run's far end in its sparse-table level (the level arrays live in the
// same workspace as g), off2 = the second (overlapping) window
__device__ __forceinline__ void mf_stage_runs(const imf_min_args& a, const imf_orient_desc& d,
                                              int qi, mf_run* rr) {
  const int nr = d.n_sruns;
  const long long sx = 1, sy = d.box_dim[0], sz = (long long)d.box_dim[0] * d.box_dim[1];
  const long long sa = d.sv[0] * sx + d.sv[1] * sy + d.sv[2] * sz;  // box offset of sv
  // level s >= 1 of orientation qi, relative to its g
  const long long l1 = (long long)(a.lvl - a.g) + qi * (a.lvl_stride - a.g_stride);
  for (int r = threadIdx.x; r < nr && r < MF_LDS_RUNS; r += blockDim.x) {
    const imf_run u = d.sruns[r];
    const int sl = ilog2(u.len);
    mf_run m;
    m.off = (sl == 0 ? 0 : l1 + (long long)(sl - 1) * a.g_stride) -
            (u.x * sx + u.y * sy + u.z * sz) - (long long)(u.len - 1) * sa;
    m.off2 = m.off + (long long)(u.len - (1 << sl)) * sa;
    rr[r] = m;
  }
}

// All blocks (no bound): one wave per block, 4 blocks per workgroup, runs
// staged in LDS once per workgroup.  The logical blocks are cut into 8
// contiguous ranges of workgroups, one per XCD: the hardware deals workgroups
// to the XCDs round robin (workgroup b runs on XCD b % 8), so workgroup b takes
// the (b / 8)-th group of 4 of range b % 8 and the blocks in flight on one XCD
// stay a compact window that shares its L2.
template <int WX, int WY, int WZ>
__global__ void __launch_bounds__(IMF_WG) k_minfilter(imf_min_args a, int qi) {
  __shared__ mf_run rr[MF_LDS_RUNS];
  const mf_geom G(WX, WY, WZ, a.nx, a.ny, a.nz);
  const long long nwg = (G.nlog + 3) / 4;
  const long long per = (nwg + 7) / 8;
  const long long lg = (long long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lg >= nwg) return;  // uniform over the workgroup
  const imf_orient_desc& d = a.desc[qi];
  mf_stage_runs(a, d, qi, rr);
  __syncthreads();
  int bx, by, bz;
  if (!G.block(lg * 4 + (threadIdx.x >> 6), bx, by, bz)) return;
  mf_block<WX, WY, WZ>(a, d, rr, qi, bx, by, bz, ((long long)bz * G.nby + by) * G.nbx + bx);
}

// Blocks left by the bound (compacted list in logical order): a resident grid
// whose waves walk the list with a static schedule.  XCD x (workgroups x,
// x + 8, ...) takes the x-th eighth of the list; inside it, its workgroups
// take consecutive groups of NW entries, then advance by the XCD's total.
// With SYNC the NW waves of a workgroup walk the runs in step (a barrier per
// 8 runs): consecutive kept blocks are mostly x neighbours in one brick row,
// so their gathers of one run hit the same cache lines while they are in L1.
template <int WX, int WY, int WZ, bool SYNC, int NW>
__global__ void __launch_bounds__(64 * NW) k_minfilter_list(imf_min_args a, int qi) {
  __shared__ mf_run rr[MF_LDS_RUNS];
  const mf_geom G(WX, WY, WZ, a.nx, a.ny, a.nz);
  const long long M = a.count[qi];
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.skipped)
    atomicAdd(a.skipped, (unsigned long long)((long long)G.nbx * G.nby * G.nbz - M));
  const imf_orient_desc& d = a.desc[qi];
  mf_stage_runs(a, d, qi, rr);
  __syncthreads();
  const int* list = a.list + (long long)qi * a.list_stride;
  // the orientation's first slot in a compact gamma stack, read once
  const long long gb = a.gbase ? a.gbase[d.out_q] : -1;
  const long long per = (M + 7) / 8;
  const long long lo = (long long)(blockIdx.x & 7) * per;
  const long long hi = lo + per < M ? lo + per : M;
  const long long step = (long long)(gridDim.x >> 3) * NW;
  if (SYNC) {
    // groups of NW consecutive entries, one per wave, walked in step
    for (long long e0 = lo + (long long)(blockIdx.x >> 3) * NW; e0 < hi; e0 += step) {
      const long long e = e0 + (threadIdx.x >> 6);
      const bool act = e < hi;
      const unsigned int pk = act ? (unsigned int)list[e] : 0u;
      const int bx = (int)(pk & 1023u), by = (int)((pk >> 10) & 2047u), bz = (int)(pk >> 21);
      mf_block<WX, WY, WZ, true>(a, d, rr, qi, bx, by, bz,
                                 ((long long)bz * G.nby + by) * G.nbx + bx, act, e, gb);
    }
    return;
  }
  for (long long e = lo + (long long)(blockIdx.x >> 3) * NW + (threadIdx.x >> 6); e < hi;
       e += step) {
    const unsigned int pk = (unsigned int)list[e];
    const int bx = (int)(pk & 1023u), by = (int)((pk >> 10) & 2047u), bz = (int)(pk >> 21);
    mf_block<WX, WY, WZ>(a, d, rr, qi, bx, by, bz, ((long long)bz * G.nby + by) * G.nbx + bx,
                         true, e, gb);
  }
}

// part 1: bound, scan and scatter of orientation q; part 2: its minimum pass
template <int WX, int WY, int WZ>
static hipError_t launch_mf(const imf_min_args& a, hipStream_t s, int part, int q) {
  const mf_geom G(WX, WY, WZ, a.nx, a.ny, a.nz);
  hipError_t e;
  if (part == 1) {
    const unsigned gb = (unsigned)((G.nlog + IMF_WG - 1) / IMF_WG);
    hipLaunchKernelGGL((k_bound<WX, WY, WZ>), dim3(gb), dim3(IMF_WG), 0, s, a, q);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_masks, dim3(1), dim3(1024), 0, s, a, q, (int)((G.nlog + 63) / 64));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_scatter<WX, WY, WZ>), dim3(gb), dim3(IMF_WG), 0, s, a, q);
    return hipGetLastError();
  }
  const long long nwg = (G.nlog + 3) / 4;
  if (a.bnb) {
    // resident capacity (a multiple of 8 workgroups)
    long long lgrid = std::min((long long)a.n_cu * a.wg_per_cu, nwg);
    lgrid = std::max(8LL, (lgrid + 7) / 8 * 8);
    if (a.sync_waves == 2) {  // eight waves per workgroup (half as many workgroups)
      lgrid = std::max(8LL, ((long long)a.n_cu * std::max(1, a.wg_per_cu / 2) + 7) / 8 * 8);
      hipLaunchKernelGGL((k_minfilter_list<WX, WY, WZ, true, 8>), dim3((unsigned)lgrid), dim3(512),
                         0, s, a, q);
    } else if (a.sync_waves) {
      hipLaunchKernelGGL((k_minfilter_list<WX, WY, WZ, true, 4>), dim3((unsigned)lgrid),
                         dim3(IMF_WG), 0, s, a, q);
    } else {
      hipLaunchKernelGGL((k_minfilter_list<WX, WY, WZ, false, 4>), dim3((unsigned)lgrid),
                         dim3(IMF_WG), 0, s, a, q);
    }
  } else {
    const long long grid = (nwg + 7) / 8 * 8;
    hipLaunchKernelGGL((k_minfilter<WX, WY, WZ>), dim3((unsigned)grid), dim3(IMF_WG), 0, s, a, q);
  }
  return hipGetLastError();
}

long long imf_block_logical(int shape, int nx, int ny, int nz) {
  int wx, wy, wz;
  imf_block_dims(shape, wx, wy, wz);
  return mf_geom(wx, wy, wz, nx, ny, nz).nlog;
}

hipError_t imf_launch_minfilter(const imf_min_args& a, hipStream_t s, int stage, int q) {
  hipError_t e;
  int wx, wy, wz;
  imf_block_dims(a.shape, wx, wy, wz);
  if ((stage < 0 || stage == 0) && a.nlvl > 0) {
    // one launch for all orientations of the batch; the grid covers the
    // largest line count (rows for x runs, x groups otherwise)
    if (a.lds_levels) {  // orientations with more than LS_MAXL levels
      const size_t sm = (size_t)2 * LVL_LT * a.max_m * sizeof(float);
      if (sm > 64 * 1024)
        if ((e = hipFuncSetAttribute((const void*)k_levels,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm)) !=
            hipSuccess)
          return e;
      hipLaunchKernelGGL(k_levels, dim3((unsigned)a.max_lines, 1, a.nq), dim3(IMF_WG), sm, s,
                         a.desc, a.g, a.g_stride, a.lvl, a.lvl_stride, a.nlvl);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (a.x_rows > 0) {
      hipLaunchKernelGGL(k_levels_x,
                         dim3((unsigned)((a.x_rows + IMF_WG / 64 - 1) / (IMF_WG / 64)), a.nq),
                         dim3(IMF_WG), 0, s, a.desc, a.g, a.g_stride, a.lvl, a.lvl_stride, a.nlvl);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (a.vstream_waves > 0) {
      hipLaunchKernelGGL(k_levels_vstream,
                         dim3((unsigned)((a.vstream_waves + IMF_WG / 64 - 1) / (IMF_WG / 64)),
                              a.nq),
                         dim3(IMF_WG), 0, s, a.desc, a.g, a.g_stride, a.lvl, a.lvl_stride, a.nlvl);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (a.stream_waves > 0) {
      hipLaunchKernelGGL(k_levels_stream,
                         dim3((unsigned)((a.stream_waves + IMF_WG / 64 - 1) / (IMF_WG / 64)), a.nq),
                         dim3(IMF_WG), 0, s, a.desc, a.g, a.g_stride, a.lvl, a.lvl_stride, a.nlvl);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if ((stage < 0 || stage == 0) && a.bnb) {
    hipLaunchKernelGGL(k_footprint, dim3(a.nq), dim3(IMF_WG), 0, s, a.desc, a.nx, a.ny, a.nz, wx,
                       wy, wz, a.fp, a.fp_cap);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // waves: (64-x segment, cell row, CM_CZ cell planes) over the largest box
    const long long waves = a.cell_waves;
    if (!a.cellmin_fused) {
      hipLaunchKernelGGL(k_cellmin, dim3((unsigned)((waves + 3) / 4), a.nq), dim3(IMF_WG), 0, s,
                         a.desc, a.g, a.g_stride, wx, wy, wz, a.cellmin, a.cell_stride);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (a.fmax_up) {  // two-phase masks: bound of the threshold for this batch
      const long long nb = (long long)((a.nx + wx - 1) / wx) * ((a.ny + wy - 1) / wy) *
                           ((a.nz + wz - 1) / wz);
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, a.fmax_up, 1LL, 0u);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const long long wg = std::min(256LL, (nb + IMF_WG - 1) / IMF_WG);
      hipLaunchKernelGGL(k_blockmax, dim3((unsigned)wg), dim3(IMF_WG), 0, s, a.fblock, nb,
                         a.fmax_up);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (stage == 0) return hipSuccess;
  for (int qi = (stage < 0 ? 0 : q); qi < (stage < 0 ? a.nq : q + 1); qi++)
    for (int part = 1; part <= 2; part++) {
      if (part == 1 && (!a.bnb || stage == 2)) continue;
      if (part == 2 && stage == 1) continue;
      switch (a.shape) {
        case 1: e = launch_mf<32, 2, 1>(a, s, part, qi); break;
        case 2: e = launch_mf<16, 2, 2>(a, s, part, qi); break;
        case 3: e = launch_mf<16, 4, 1>(a, s, part, qi); break;
        case 4: e = launch_mf<8, 4, 2>(a, s, part, qi); break;
        default: e = launch_mf<64, 1, 1>(a, s, part, qi); break;
      }
      if (e != hipSuccess) return e;
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
  a.masks[((long long)d.out_q * a.nz + z) * a.ny * words + (long long)y * words + w] =
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
static unsigned fill_grid(long long n) {
  const long long b = (n + 255) / 256;
  return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}
hipError_t imf_launch_fill_f(float* f, long long n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(fill_grid(n)), dim3(256), 0, s, f, n, v);
  return hipGetLastError();
}
hipError_t imf_launch_fill_u32(unsigned int* p, long long n, unsigned int v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
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

// out = (a != 0) | (b != 0), a may be NULL: the fixture of one setup (the
// common fixture with that setup's set), or the union over every setup
__global__ void k_or_u8(const uint8_t* __restrict__ a, const uint8_t* __restrict__ b,
                        uint8_t* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (uint8_t)(((a ? a[i] : 0) | b[i]) != 0);
}
hipError_t imf_launch_or_u8(const uint8_t* a, const uint8_t* b, uint8_t* out, long long n,
                            hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_or_u8, dim3((unsigned)blocks), dim3(256), 0, s, a, b, out, n);
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

// masks from stored gamma once theta = lambda F_max is known.  One wave per
// 64-voxel word of a row: Omega_0 is read once and the wave walks all
// orientations (independent coalesced loads, one mask word each).
__global__ void __launch_bounds__(IMF_WG) k_masks_gamma(const float* __restrict__ gs, int nq,
                                                        const uint8_t* __restrict__ om, int nx,
                                                        int ny, int nz,
                                                        const unsigned long long* __restrict__ Fq,
                                                        double scale, double lambda, double E,
                                                        uint64_t* __restrict__ masks,
                                                        const unsigned long long* __restrict__ keep,
                                                        int WX, int WY, int WZ, long long kstride,
                                                        const long long* __restrict__ gbase,
                                                        const int* __restrict__ koff) {
  const int words = (nx + 63) >> 6;
  const long long wave = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const long long per_q = (long long)words * ny * nz;
  if (wave >= per_q) return;
  const int w = (int)(wave % words);
  const long long yz = wave / words;
  const int x = w * 64 + lane;
  // theta = lambda F_max as the definition takes it (fixed point), in voxel
  // units; a bit is set here only where it is certain (gamma + E <= theta),
  // the band around theta is decided from exact overlaps afterwards
  const double theta = lambda * (double)*Fq * scale;
  const long long N = (long long)nx * ny * nz;
  const long long vi = yz * nx + (x < nx ? x : nx - 1);
  const bool in = x < nx && om[vi];
  const float* g = gs + vi;
  // Blocks the bound skipped hold no gamma (their mask bits are 0).  The
  // blocks of one 64-voxel word are consecutive in the logical order (bricks
  // are 128 voxels wide, blocks x fastest), so one keep word per orientation,
  // the same for the whole wave, holds their bits from (lg0 & 63) on.
  long long kw = 0;
  int kb0 = 0, li = 0;
  if (keep) {
    const mf_geom G(WX, WY, WZ, nx, ny, nz);
    const int y = (int)(yz % ny), z = (int)(yz / ny);
    const long long lg0 = G.logical((w * 64) / WX, y / WY, z / WZ);
    kw = lg0 >> 6;
    kb0 = (int)(lg0 & 63);
    li = x % WX + WX * (y % WY + WY * (z % WZ));  // lane of the voxel in its block
  }
  const int kbit = kb0 + (WX < 64 ? lane / WX : 0);
  // gamma of orientation q here, +inf where its block was skipped (and where
  // a compact stack overflowed: a second pass then decides the request)
  auto gamma_at = [&](int q, unsigned long long word) -> float {
    if (!((word >> kbit) & 1)) return INFINITY;
    if (!gbase) return g[(long long)q * N];
    const long long gb = gbase[q];
    if (gb < 0) return INFINITY;
    const int slot = koff[(long long)q * kstride + kw] + __popcll(word & ((1ull << kbit) - 1));
    return gs[gb + (long long)slot * 64 + li];
  };
  // keep words of 64 orientations at a time, one per lane, then broadcast
  for (int qc = 0; qc < nq; qc += 64) {
    const int nc = nq - qc < 64 ? nq - qc : 64;
    const unsigned long long mine_w =
        keep && lane < nc ? keep[(long long)(qc + lane) * kstride + kw] : ~0ull;
    const unsigned int lo32 = (unsigned int)mine_w, hi32 = (unsigned int)(mine_w >> 32);
    auto word_of = [&](int j) {
      return ((unsigned long long)__builtin_amdgcn_readlane(hi32, j) << 32) |
             (unsigned int)__builtin_amdgcn_readlane(lo32, j);
    };
    int j = 0;
    for (; j + 4 <= nc; j += 4) {
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; i++) v[i] = gamma_at(qc + j + i, word_of(j + i));
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const unsigned long long bits = __ballot(in && (double)v[i] + E <= theta);
        if (lane == 0) masks[(long long)(qc + j + i) * per_q + wave] = bits;
      }
    }
    for (; j < nc; j++) {
      const float v = gamma_at(qc + j, word_of(j));
      const unsigned long long bits = __ballot(in && (double)v + E <= theta);
      if (lane == 0) masks[(long long)(qc + j) * per_q + wave] = bits;
    }
  }
}
hipError_t imf_launch_masks_from_gamma(const float* gamma_stack, int nq, const uint8_t* omega0,
                                       int nx, int ny, int nz, const unsigned long long* Fq,
                                       double scale, double lambda, double E, uint64_t* masks,
                                       const unsigned long long* keep, int shape,
                                       long long kstride, const long long* gbase,
                                       const int* koff, hipStream_t s) {
  const int words = (nx + 63) >> 6;
  const long long waves = (long long)words * ny * nz;
  const int per = IMF_WG / 64;
  int wx, wy, wz;
  imf_block_dims(shape, wx, wy, wz);
  hipLaunchKernelGGL(k_masks_gamma, dim3((unsigned)((waves + per - 1) / per)), dim3(IMF_WG), 0, s,
                     gamma_stack, nq, omega0, nx, ny, nz, Fq, scale, lambda, E, masks, keep, wx,
                     wy, wz, kstride, gbase, koff);
  return hipGetLastError();
}
