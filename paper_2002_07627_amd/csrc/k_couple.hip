// Steps that couple the IMF to a density-based TO loop (Sec. 2.2): the
// Heaviside projection of the design variables (Eq. Heaviside), the
// accessibility filter (Eq. accFilter) and the filtered sensitivity
// (Eq. filtered_sens).  Pointwise and HBM-bound; float64 arithmetic, compiled
// without FP contraction so that every operation rounds as written.
#include <mutex>

#include "imf_internal.h"

#define Q24 16777216.0

static unsigned grid_of(long long n) {
  const long long b = (n + 255) / 256;
  return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

// rho = 1 - exp(-beta xi) + xi exp(-beta), xi clamped to [0, 1], rounded to
// the nearest multiple of 2^-24 (halves up) and clamped to [0, 1]
__global__ void k_heaviside(const float* __restrict__ xi, long long n, double beta,
                            float* __restrict__ rho) {
  const double eb = exp(-beta);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double x = (double)xi[i];
    x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
    const double r = (1.0 - exp(-beta * x)) + x * eb;
    double q = floor(r * Q24 + 0.5) / Q24;
    q = q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
    rho[i] = (float)q;
  }
}

hipError_t imf_launch_heaviside(const float* xi, long long n, double beta, float* rho,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_heaviside, dim3(grid_of(n)), dim3(256), 0, s, xi, n, beta, rho);
  return hipGetLastError();
}

__global__ void k_fill_u32_couple(unsigned int* p) {
  if (threadIdx.x == 0) *p = 0u;
}

__device__ __forceinline__ bool in_omega0(const uint8_t* fixture, const uint8_t* domain,
                                          long long i) {
  return domain ? domain[i] != 0 : (fixture ? fixture[i] == 0 : true);
}

// Sbar_IMF: fbar on Omega = [rho > tau], 1 on Gamma, 0 elsewhere; and the
// largest |S_phi| over Omega_0 (non-negative floats order as their bits)
__global__ void k_access_filter(const void* __restrict__ design, int density,
                                const float* __restrict__ imf_norm,
                                const uint8_t* __restrict__ secluded, double tau, long long n,
                                float* __restrict__ filt, const float* __restrict__ sens,
                                const uint8_t* __restrict__ fixture,
                                const uint8_t* __restrict__ domain,
                                unsigned int* __restrict__ smax) {
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double rho = density ? (double)((const float*)design)[i]
                               : (double)((const uint8_t*)design)[i];
    float v = secluded[i] ? 1.f : 0.f;
    if (rho > tau) v = imf_norm[i];
    filt[i] = v;
    if (sens && in_omega0(fixture, domain, i)) m = fmaxf(m, fabsf(sens[i]));
  }
  if (sens) {  // one atomic per workgroup (the grid is capped at 2048 workgroups)
    __shared__ float red[4];
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
      atomicMax(smax, __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
  }
}

// S = (1 - w) S_phi / max|S_phi| + w Sbar_IMF
__global__ void k_filtered_sens(const float* __restrict__ sens, const float* __restrict__ filt,
                                long long n, double w, const unsigned int* __restrict__ smax,
                                float* __restrict__ out) {
  const double m = (double)__uint_as_float(*smax);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double sb = m > 0.0 ? (double)sens[i] / m : 0.0;
    out[i] = (float)((1.0 - w) * sb + w * (double)filt[i]);
  }
}

hipError_t imf_launch_access_filter(const imf_couple_args& a, hipStream_t s) {
  hipError_t e;
  if (a.sens) {
    hipLaunchKernelGGL(k_fill_u32_couple, dim3(1), dim3(64), 0, s, a.smax);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const unsigned gf = grid_of(a.n) < 2048 ? grid_of(a.n) : 2048;
  hipLaunchKernelGGL(k_access_filter, dim3(gf), dim3(256), 0, s, a.design, a.density,
                     a.imf_norm, a.secluded, a.tau, a.n, a.filt, a.sens, a.fixture, a.domain,
                     a.smax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.sens && a.sens_out) {
    hipLaunchKernelGGL(k_filtered_sens, dim3(grid_of(a.n)), dim3(256), 0, s, a.sens, a.filt, a.n,
                       a.w, a.smax, a.sens_out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Greedy machining plan (Sec. 3.4.1, post-processing): the negative space to
// remove, N = Omega_0 and [rho <= tau], as a bitset laid out like the masks;
// per step the popcount of (A_q and R) for every orientation q, then
// R = R and not A_q for the chosen one.
// ---------------------------------------------------------------------------
__global__ void k_negative_bits(const void* __restrict__ design, int density, double tau,
                                const uint8_t* __restrict__ fixture,
                                const uint8_t* __restrict__ domain, int nx, long long rows,
                                uint64_t* __restrict__ R) {
  const int words = (nx + 63) >> 6;
  const long long wave = (long long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (wave >= rows * words) return;
  const long long row = wave / words;
  const int x = (int)(wave % words) * 64 + (threadIdx.x & 63);
  bool b = false;
  if (x < nx) {
    const long long i = row * nx + x;
    const double rho = density ? (double)((const float*)design)[i]
                               : (double)((const uint8_t*)design)[i];
    b = in_omega0(fixture, domain, i) && rho <= tau;
  }
  const unsigned long long m = __ballot(b);
  if ((threadIdx.x & 63) == 0) R[wave] = m;
}

__global__ void k_cover_count(const uint64_t* __restrict__ masks, long long nw,
                              const uint64_t* __restrict__ R,
                              unsigned long long* __restrict__ counts) {
  const int q = blockIdx.y;
  const uint64_t* A = masks + (long long)q * nw;
  unsigned long long c = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (long long)gridDim.x * blockDim.x)
    c += __popcll(A[i] & R[i]);
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(counts + q, c);
}

__global__ void k_cover_remove(const uint64_t* __restrict__ A, long long nw,
                               uint64_t* __restrict__ R) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (long long)gridDim.x * blockDim.x)
    R[i] &= ~A[i];
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

hipError_t imf_launch_negative_bits(const void* design, int density, double tau,
                                    const uint8_t* fixture, const uint8_t* domain, int nx,
                                    long long rows, uint64_t* R, hipStream_t s) {
  const long long waves = rows * ((nx + 63) / 64);
  hipLaunchKernelGGL(k_negative_bits, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, design,
                     density, tau, fixture, domain, nx, rows, R);
  return hipGetLastError();
}

hipError_t imf_launch_cover_count(const uint64_t* masks, int nq, long long nw, const uint64_t* R,
                                  unsigned long long* counts, hipStream_t s) {
  hipError_t e;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, counts, nq);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const long long per = (nw + 255) / 256;
  const unsigned gx = (unsigned)(per < 64 ? (per > 0 ? per : 1) : 64);
  hipLaunchKernelGGL(k_cover_count, dim3(gx, nq), dim3(256), 0, s, masks, nw, R, counts);
  return hipGetLastError();
}

hipError_t imf_launch_cover_remove(const uint64_t* A, long long nw, uint64_t* R, hipStream_t s) {
  hipLaunchKernelGGL(k_cover_remove, dim3(grid_of(nw)), dim3(256), 0, s, A, nw, R);
  return hipGetLastError();
}

// Choice of one greedy step on the device: the largest count, the lowest
// orientation index among equal counts (one workgroup of 1024 threads).
// out[0] = that count, out[1] = its orientation.
__global__ void __launch_bounds__(1024) k_cover_best(const unsigned long long* __restrict__ counts,
                                                      int nq, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long sc[16];
  __shared__ int si[16];
  unsigned long long c = 0;
  int i = 0x7fffffff;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    const unsigned long long v = counts[q];
    if (v > c || (v == c && q < i)) {
      c = v;
      i = q;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long c2 = __shfl_xor(c, o);
    const int i2 = __shfl_xor(i, o);
    if (c2 > c || (c2 == c && i2 < i)) {
      c = c2;
      i = i2;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    sc[threadIdx.x >> 6] = c;
    si[threadIdx.x >> 6] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); w++)
      if (sc[w] > c || (sc[w] == c && si[w] < i)) {
        c = sc[w];
        i = si[w];
      }
    out[0] = c;
    out[1] = (unsigned long long)(i == 0x7fffffff ? 0 : i);
  }
}

hipError_t imf_launch_cover_best(const unsigned long long* counts, int nq, unsigned long long* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_cover_best, dim3(1), dim3(1024), 0, s, counts, nq, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free planner: the remaining negative space
// (nz * ny * ceil(nx/64) words), the per-orientation counts (n_orient words)
// and the step's choice (2 words).  Each GPU the library runs on holds its
// own copy from the library's load until the process ends.  In host code the
// array's name is not its device address: set-up takes that address once per
// device (with the device current) and every launch uses it.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned long long scratch[IMF_PLAN_SCRATCH_WORDS];

static std::mutex g_scratch_mu;
static unsigned long long* g_scratch_ptr[IMF_MAX_DEVICES] = {};

hipError_t imf_plan_scratch_init(int device) {
  if (device < 0 || device >= IMF_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  unsigned long long* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

unsigned long long* imf_plan_scratch(int device) {
  if (device < 0 || device >= IMF_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}
