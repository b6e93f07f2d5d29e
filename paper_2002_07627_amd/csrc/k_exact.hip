// Exact threshold decisions of density requests whose threshold depends on
// F_max (Algorithm 1 of Sec. 2.1.5: the normalization by the maximum and the
// allowance B = [fbar > lambda]; the per-orientation masks of Eq. A at the
// threshold lambda F_max).
//
// The float32 transforms give every overlap g within E of its exact value (an
// error model that every exact recomputation checks), and the minima gamma
// and f are exact minima of those floats, so:
//   * F_max: only voxels of Omega_0 whose float32 f is within 2E of the float32
//     maximum can hold the exact maximum; their f is recomputed exactly from
//     the overlaps that can attain it (orientations whose gamma is within 2E of
//     f, translations whose g is within 2E of f);
//   * a mask bit A_R(x) is set for certain where gamma + E <= theta and clear
//     for certain where gamma - E > theta.  Otherwise only the translations
//     of the band theta - E < g <= theta + E can decide it: their overlaps are
//     recomputed exactly, and those at or below theta are swept by the cutter
//     (Eq. sweep) into the masks;
//   * B(x) is certain where f - E > theta or f + E <= theta; otherwise x is in
//     B iff no orientation's mask holds it (f <= theta iff some gamma_R <= theta).
// Exact overlaps are sums of prefix sums of rho_O (fixed point, 2^-24 units for
// density), so every decision equals the one the definition takes.
#include "imf_internal.h"

static unsigned grid_cap(long long n, long long cap) {
  const long long b = (n + IMF_WG - 1) / IMF_WG;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

// exact overlap at translation t, the tool's x-runs split over the wave's
// lanes, four runs per lane with their loads in flight together (lanes past
// the last run read the last one and add 0)
__device__ __forceinline__ long long exact_overlap_wave(const imf_orient_desc& d,
                                                        const long long* __restrict__ ps, int nx,
                                                        int ny, int nz, int tx, int ty, int tz) {
  const int lane = threadIdx.x & 63;
  const int n = d.n_truns;
  long long s = 0;
  for (int r0 = 0; r0 < n; r0 += 4 * 64) {
    long long hi[4], lo[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int r = r0 + 64 * k + lane;
      const long long* row;
      int a0, a1;
      exact_run_terms(d.truns[r < n ? r : n - 1], ps, nx, ny, nz, tx, ty, tz, row, a0, a1);
      if (r >= n) a0 = a1 = 0;
      hi[k] = row[a1];
      lo[k] = row[a0];
    }
#pragma unroll
    for (int k = 0; k < 4; k++) s += hi[k] - lo[k];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

__device__ __forceinline__ void err_max(unsigned int* bits, float e) {
  if (__float_as_uint(e) > __atomic_load_n(bits, __ATOMIC_RELAXED))
    atomicMax(bits, __float_as_uint(e));
}

// the threshold lambda F_max in fixed-point units (as the definition takes it)
// and in voxel units (an exact power-of-two scaling)
__device__ __forceinline__ void thresholds(const imf_exact_args& a, double& thq, double& thv) {
  thq = a.lambda * (double)*a.Fq;
  thv = thq * a.scale;
}

// ---------------------------------------------------------------------------
// F_max: candidates, then their exact f
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(IMF_WG) k_fmax_cand(imf_exact_args a) {
  const double lim = (double)ord2f(*a.fmax_bits) - 2.0 * a.E;
  for (long long i = (long long)blockIdx.x * IMF_WG + threadIdx.x; i < a.N;
       i += (long long)gridDim.x * IMF_WG) {
    if (!a.omega0[i] || (double)a.f[i] < lim) continue;
    const unsigned slot = atomicAdd(a.cand_cnt, 1u);
    if (slot < (unsigned)a.cand_cap) a.cand[slot] = (int)i;
  }
}

// Exact f at the candidates, spread over the whole device: a work item is a
// (candidate x, orientation R, chunk of S_R's points); items whose gamma_R(x)
// is not within 2E of f(x) end at once (blocks the bound skipped have gamma >
// f + 2E).  The item's threads take the points k of S_R (the x-runs of S,
// flattened by a prefix sum in LDS) and recompute exactly every g(x - k) whose
// float32 value is within 2E of f(x) (all of them without a stored g); the
// smallest lowers the candidate's exact f (atomic min).
#define EXF_CHUNKS 8
#define EXF_RUNS 2048
__global__ void __launch_bounds__(IMF_WG) k_exact_f(imf_exact_args a,
                                                    unsigned long long* __restrict__ cmin) {
  __shared__ int pref[EXF_RUNS + 1];
  __shared__ unsigned long long wmin[IMF_WG / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long nc = min((long long)*a.cand_cnt, (long long)a.cand_cap);
  const long long items = nc * a.nO * EXF_CHUNKS;
  const long long nxy = (long long)a.nx * a.ny;
  for (long long it = blockIdx.x; it < items; it += gridDim.x) {
    const int ch = (int)(it % EXF_CHUNKS);
    const int q = (int)((it / EXF_CHUNKS) % a.nO);
    const long long c = it / ((long long)EXF_CHUNKS * a.nO);
    const long long vi = a.cand[c];
    const int z = (int)(vi / nxy), y = (int)((vi / a.nx) % a.ny), x = (int)(vi % a.nx);
    const double lim = (double)a.f[vi] + 2.0 * a.E;
    const imf_orient_desc& d = a.desc[q];
    const imf_orient_desc& sd = a.desc[a.nO + q];  // x-runs of S
    if (a.gamma) {  // uniform over the workgroup
      long long gi = (long long)d.out_q * a.N + vi;  // where gamma is stored, or -1
      if (a.keep) {
        const mf_geom G(a.WX, a.WY, a.WZ, a.nx, a.ny, a.nz);
        const long long lg = G.logical(x / a.WX, y / a.WY, z / a.WZ);
        const unsigned long long word = a.keep[(long long)d.out_q * a.kstride + (lg >> 6)];
        if (!((word >> (lg & 63)) & 1ull)) continue;
        if (a.gbase) {  // compact stack: the block's slot, none after an overflow
          const long long gb = a.gbase[d.out_q];
          const int slot = a.koff[(long long)d.out_q * a.kstride + (lg >> 6)] +
                           __popcll(word & ((1ull << (lg & 63)) - 1));
          const int li = x % a.WX + a.WX * (y % a.WY + a.WY * (z % a.WZ));
          gi = gb < 0 ? -1 : gb + (long long)slot * 64 + li;
        }
      }
      if (gi >= 0 && (double)a.gamma[gi] > lim) continue;
    }
    const int nr = min(sd.n_sruns, EXF_RUNS);
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int r = 0; r < nr; r++) {
        pref[r] = acc;
        acc += sd.sruns[r].len;
      }
      pref[nr] = acc;
    }
    __syncthreads();
    const int npts = pref[nr];
    const long long* ps = a.ps + a.ps_stride * d.set;
    const float* gq = a.gst ? a.gst + (long long)q * a.gst_stride : nullptr;
    unsigned long long best = ~0ull;
    unsigned int evals = 0;
    float err = 0.f;
    for (int p = ch * IMF_WG + threadIdx.x; p < npts; p += EXF_CHUNKS * IMF_WG) {
      int lo = 0, hi = nr - 1;  // the run holding point p
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= p) lo = mid; else hi = mid - 1;
      }
      const imf_run u = sd.sruns[lo];
      const int tx = x - (u.x + (p - pref[lo])), ty = y - u.y, tz = z - u.z;
      float g32 = 0.f;
      if (gq) {
        g32 = gq[((long long)(tz - d.box_lo[2]) * d.box_dim[1] + (ty - d.box_lo[1])) * d.box_dim[0] +
                 (tx - d.box_lo[0])];
        if ((double)g32 > lim) continue;
      }
      const long long s = exact_overlap(d, ps, a.nx, a.ny, a.nz, tx, ty, tz);
      evals++;
      if (gq) err = fmaxf(err, (float)fabs((double)g32 - (double)s * a.scale));
      if ((unsigned long long)s < best) best = (unsigned long long)s;
    }
    // runs beyond the LDS prefix (very wide cutters): one thread per run
    for (int r = EXF_RUNS + ch * IMF_WG + threadIdx.x; r < sd.n_sruns; r += EXF_CHUNKS * IMF_WG) {
      const imf_run u = sd.sruns[r];
      for (int j = 0; j < u.len; j++) {
        const int tx = x - (u.x + j), ty = y - u.y, tz = z - u.z;
        const long long s = exact_overlap(d, ps, a.nx, a.ny, a.nz, tx, ty, tz);
        evals++;
        if ((unsigned long long)s < best) best = (unsigned long long)s;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long b2 = __shfl_xor(best, o);
      best = b2 < best ? b2 : best;
      evals += __shfl_xor(evals, o);
      err = fmaxf(err, __shfl_xor(err, o));
    }
    if (lane == 0) {
      wmin[wv] = best;
      if (evals) atomicAdd(a.n_exact, evals);
      if (err > 0.f) err_max(a.err_bits, err);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long m = wmin[0];
      for (int w = 1; w < IMF_WG / 64; w++) m = wmin[w] < m ? wmin[w] : m;
      if (m != ~0ull) atomicMin(cmin + c, m);
    }
  }
}

__global__ void k_cmin_init(unsigned long long* cmin, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    cmin[i] = ~0ull;
}

// F_max = the largest exact f among the candidates
__global__ void __launch_bounds__(IMF_WG) k_cmin_max(imf_exact_args a,
                                                     const unsigned long long* cmin) {
  const long long nc = min((long long)*a.cand_cnt, (long long)a.cand_cap);
  unsigned long long m = 0;
  for (long long c = threadIdx.x; c < nc; c += IMF_WG)
    if (cmin[c] != ~0ull && cmin[c] > m) m = cmin[c];
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long m2 = __shfl_xor(m, o);
    m = m2 > m ? m2 : m;
  }
  if ((threadIdx.x & 63) == 0 && m) atomicMax(a.Fq, m);
}

hipError_t imf_launch_exact_fmax(const imf_exact_args& a, unsigned long long* cmin,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_cmin_init, dim3(64), dim3(IMF_WG), 0, s, cmin, a.cand_cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fmax_cand, dim3(grid_cap(a.N, 4096)), dim3(IMF_WG), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_exact_f, dim3(2048), dim3(IMF_WG), 0, s, a, cmin);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cmin_max, dim3(1), dim3(IMF_WG), 0, s, a, (const unsigned long long*)cmin);
  return hipGetLastError();
}

// fixed-point F_max from the float32 maximum (binary: exact integers; density
// requests that take no exact maximum)
__global__ void k_fq_from_fmax(const unsigned int* fmax_bits, double inv_scale,
                               unsigned long long* Fq) {
  if (threadIdx.x == 0) *Fq = (unsigned long long)llrint((double)ord2f(*fmax_bits) * inv_scale);
}
hipError_t imf_launch_fq_from_fmax(const unsigned int* fmax_bits, double inv_scale,
                                   unsigned long long* Fq, hipStream_t s) {
  hipLaunchKernelGGL(k_fq_from_fmax, dim3(1), dim3(64), 0, s, fmax_bits, inv_scale, Fq);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the band around theta: stored overlaps theta - E < g <= theta + E
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(IMF_WG) k_band_scan(imf_exact_args a) {
  if (a.skip_scan && *a.skip_scan == 1u) return;
  const int q = blockIdx.y;
  const imf_orient_desc& d = a.desc[q];
  const long long vol = (long long)d.box_dim[0] * d.box_dim[1] * d.box_dim[2];
  const float* gq = a.gst + (long long)q * a.gst_stride;
  double thq, thv;
  thresholds(a, thq, thv);
  const int lane = threadIdx.x & 63;
  const long long stride = (long long)gridDim.x * IMF_WG;
  // every wave runs the same number of iterations (the ballot needs the whole wave)
  const long long base0 = (long long)blockIdx.x * IMF_WG + (threadIdx.x & ~63);
  for (long long b = base0; b < vol; b += stride) {
    const long long i = b + lane;
    float g = 0.f;
    bool in = false;
    if (i < vol) {
      g = gq[i];
      in = !((double)g + a.E <= thv) && !((double)g - a.E > thv);
    }
    const unsigned long long m = __ballot(in);
    if (!m) continue;
    unsigned base = 0;
    if (lane == 0) base = atomicAdd(a.band_cnt, (unsigned)__popcll(m));
    base = __shfl(base, 0);
    if (in) {
      const unsigned slot = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
      if (slot < (unsigned)a.band_cap) a.band[slot] = make_int4(q, (int)i, __float_as_int(g), 0);
    }
  }
}

// one workgroup: no bracket list overflowed, and the band (thv - E, thv + E]
// lies inside the listed bracket (blo, bhi]
__global__ void __launch_bounds__(1024) k_bracket_check(imf_exact_args a, double blo, double bhi,
                                                        unsigned int* ok) {
  __shared__ unsigned int over, total;
  if (threadIdx.x == 0) {
    over = 0;
    total = 0;
  }
  __syncthreads();
  const long long nsl = (long long)a.nO * IMF_BR_SLICES;
  unsigned o = 0, t = 0;
  for (long long i = threadIdx.x; i < nsl; i += blockDim.x) {
    const unsigned c = a.bcnt[i];
    o |= c > (unsigned)a.bslot;
    t += c;
  }
  if (o) atomicOr(&over, 1u);
  atomicAdd(&total, t);
  __syncthreads();
  if (threadIdx.x == 0) {
    double thq, thv;
    thresholds(a, thq, thv);
    const bool in = !over && thv - a.E >= blo && thv + a.E <= bhi;
    *ok = in ? 1u : (over ? 2u : 0u);
    *a.blisted = total;
  }
}
hipError_t imf_launch_bracket_check(const imf_exact_args& a, double blo, double bhi,
                                    unsigned int* ok, hipStream_t s) {
  hipLaunchKernelGGL(k_bracket_check, dim3(1), dim3(1024), 0, s, a, blo, bhi, ok);
  return hipGetLastError();
}

hipError_t imf_launch_band_scan(const imf_exact_args& a, long long max_vol, hipStream_t s) {
  const long long per = (max_vol + IMF_WG - 1) / IMF_WG;
  const unsigned gx = (unsigned)(per < 512 ? (per > 0 ? per : 1) : 512);
  hipLaunchKernelGGL(k_band_scan, dim3(gx, a.nO), dim3(IMF_WG), 0, s, a);
  return hipGetLastError();
}

// One band entry on one wave: the exact overlap; at or below theta, the cutter
// swept from that translation (the x-runs of S) sets the mask bits of the
// voxels of Omega_0 it covers (atomic or; these voxels have gamma within E of
// theta or below, so no bit set here is a certain zero).  Bracket entries
// outside the band are left alone.
__device__ __forceinline__ void band_entry(const imf_exact_args& a, const int4 ent, double thq,
                                           double thv, float& err, unsigned int& evals) {
  const int lane = threadIdx.x & 63;
  const int words = (a.nx + 63) >> 6;
  const long long per_q = (long long)words * a.ny * a.nz;
  {
    const double g = (double)__int_as_float(ent.z);
    if (g + a.E <= thv || g - a.E > thv) return;
  }
  {
    const int q = ent.x;
    const long long li = ent.y;
    const imf_orient_desc& d = a.desc[q];
    const int bx = (int)(li % d.box_dim[0]);
    const int by = (int)((li / d.box_dim[0]) % d.box_dim[1]);
    const int bz = (int)(li / ((long long)d.box_dim[0] * d.box_dim[1]));
    const int tx = bx + d.box_lo[0], ty = by + d.box_lo[1], tz = bz + d.box_lo[2];
    const long long s = exact_overlap_wave(d, a.ps + a.ps_stride * d.set, a.nx, a.ny, a.nz, tx,
                                           ty, tz);
    evals++;
    err = fmaxf(err, (float)fabs((double)__int_as_float(ent.z) - (double)s * a.scale));
    if (!((double)s <= thq)) return;
    const imf_orient_desc& sd = a.desc[a.nO + q];
    uint64_t* mq = a.masks + (long long)d.out_q * per_q;
    for (int r = lane; r < sd.n_sruns; r += 64) {
      const imf_run u = sd.sruns[r];
      const int y = ty + u.y, z = tz + u.z;
      if (y < 0 || y >= a.ny || z < 0 || z >= a.nz) continue;
      const int x0 = max(tx + u.x, 0), x1 = min(tx + u.x + u.len, a.nx);
      const long long rw = ((long long)z * a.ny + y) * words;
      uint64_t* row = mq + rw;
      for (int x = x0; x < x1;) {
        const int w = x >> 6;
        const int xe = min(x1, (w + 1) << 6);
        // bits x .. xe - 1 of word w, those of Omega_0
        const int b0 = x & 63, b1 = xe - (w << 6);
        const uint64_t span = (b1 == 64 ? ~0ull : (1ull << b1) - 1ull) & ~((1ull << b0) - 1ull);
        const uint64_t bits = span & a.om_bits[rw + w];
        if (bits && (row[w] & bits) != bits)
          atomicOr((unsigned long long*)(row + w), (unsigned long long)bits);
        x = xe;
      }
    }
  }
}

__global__ void __launch_bounds__(IMF_WG) k_band_exact(imf_exact_args a) {
  const int lane = threadIdx.x & 63;
  double thq, thv;
  thresholds(a, thq, thv);
  float err = 0.f;
  unsigned int evals = 0;
  const long long wave = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  const long long nwaves = (long long)gridDim.x * (IMF_WG / 64);
  // the scanned list
  const long long n = min((long long)*a.band_cnt, (long long)a.band_cap);
  for (long long e = wave; e < n; e += nwaves) band_entry(a, a.band[e], thq, thv, err, evals);
  // the bracket lists, when they hold the band (a wave per list)
  if (a.blist && *a.skip_scan == 1u) {
    const long long nsl = (long long)a.nO * IMF_BR_SLICES;
    for (long long sl = wave; sl < nsl; sl += nwaves) {
      const unsigned c = min(a.bcnt[sl], (unsigned)a.bslot);
      for (unsigned e = 0; e < c; e++)
        band_entry(a, a.blist[sl * a.bslot + e], thq, thv, err, evals);
    }
  }
  for (int o = 32; o > 0; o >>= 1) err = fmaxf(err, __shfl_xor(err, o));
  if (lane == 0) {
    if (err > 0.f) err_max(a.err_bits, err);
    if (evals) atomicAdd(a.n_exact, evals);
  }
}

// one wave per 64-voxel row word
__global__ void __launch_bounds__(IMF_WG) k_om_bits(const uint8_t* __restrict__ om, int nx,
                                                    long long rows, uint64_t* __restrict__ out) {
  const int words = (nx + 63) >> 6;
  const long long wv = (long long)blockIdx.x * (IMF_WG / 64) + (threadIdx.x >> 6);
  if (wv >= rows * words) return;  // uniform over the wave
  const long long rr = wv / words;
  const int x = (int)(wv - rr * words) * 64 + (threadIdx.x & 63);
  const unsigned long long m = __ballot(x < nx && om[rr * nx + x]);
  if ((threadIdx.x & 63) == 0) out[wv] = m;
}

hipError_t imf_launch_om_bits(const uint8_t* om, int nx, long long rows, uint64_t* out,
                              hipStream_t s) {
  const long long waves = rows * ((nx + 63) / 64);
  const long long per = IMF_WG / 64;
  hipLaunchKernelGGL(k_om_bits, dim3((unsigned)((waves + per - 1) / per)), dim3(IMF_WG), 0, s,
                     om, nx, rows, out);
  return hipGetLastError();
}

hipError_t imf_launch_band_exact(const imf_exact_args& a, hipStream_t s) {
  hipLaunchKernelGGL(k_band_exact, dim3(2048), dim3(IMF_WG), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// B = Omega_0 and f > lambda F_max; fbar = f / F_max on B, 0 elsewhere;
// Gamma = B and not Omega, Omega = [rho_Omega > tau]  (Algorithm 1, Eq. gamma)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(IMF_WG) k_finalize_exact(imf_exact_args a, const void* design,
                                                           int density, double tau, double Efin,
                                                           float* __restrict__ imf_out,
                                                           float* __restrict__ imf_norm,
                                                           uint8_t* __restrict__ secluded) {
  const long long i = (long long)blockIdx.x * IMF_WG + threadIdx.x;
  if (i >= a.N) return;
  double thq, thv;
  thresholds(a, thq, thv);
  const double Fv = (double)*a.Fq * a.scale;
  const float v = a.f[i];
  bool inB = false;
  if (a.omega0[i]) {
    if ((double)v - Efin > thv) {
      inB = true;
    } else if (!((double)v + Efin <= thv)) {
      // within the band: in B iff no orientation's (exact) mask holds x
      const int words = (a.nx + 63) >> 6;
      const long long per_q = (long long)words * a.ny * a.nz;
      const long long row = i / a.nx;
      const int x = (int)(i % a.nx);
      const long long wi = row * words + (x >> 6);
      const uint64_t bit = 1ull << (x & 63);
      inB = true;
      for (int q = 0; q < a.nO && inB; q++)
        if (a.masks[(long long)q * per_q + wi] & bit) inB = false;
    }
  }
  if (imf_out) imf_out[i] = v;
  if (imf_norm) imf_norm[i] = inB && Fv > 0 ? (float)((double)v / Fv) : 0.0f;
  if (secluded) {
    const double rho = density ? (double)((const float*)design)[i]
                               : (double)((const uint8_t*)design)[i];
    secluded[i] = (uint8_t)(inB && !(rho > tau));
  }
}

hipError_t imf_launch_finalize_exact(const imf_exact_args& a, const void* design, int density,
                                     double tau, double Efin, float* imf_out, float* imf_norm,
                                     uint8_t* secluded, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_exact, dim3((unsigned)((a.N + IMF_WG - 1) / IMF_WG)), dim3(IMF_WG),
                     0, s, a, design, density, tau, Efin, imf_out, imf_norm, secluded);
  return hipGetLastError();
}
