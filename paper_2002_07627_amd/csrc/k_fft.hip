// FFT-based correlation (the Convolve step of Algorithm 1 and App. B: two
// forward transforms, a pointwise product, one inverse transform).
//
// All transforms are hand-written for gfx950: a tile of CT columns of length
// n is staged in LDS, transformed there by self-sorting (Stockham) radix stages
// (radices 2, 3, 4, 5, 7, 8; twiddles computed in float64, stored as float32
// and kept in LDS), and written back.  Columns are chosen so that every global
// access moves CT consecutive complex values (128 bytes for CT = 16) or whole
// contiguous columns.
//
// Spectrum layout: [ky][kx][kz] with kx in [0, px/2] (real-to-complex along x)
// and kz fastest, so the fused product + inverse z pass reads both spectra as
// contiguous columns.  The reflection of the tool (its conjugate-symmetric
// image) is the complex conjugate of its spectrum (Algorithm 1's Reflect).
#include "imf_internal.h"

#include <cmath>
#include <mutex>
#include <map>
#include <type_traits>

#define CT_MAX 16

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ float2 mul_mi(float2 a, bool inv) {
  return inv ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// small DFTs, y_k = sum_j v_j exp(-+ 2 pi i jk / R)
// ---------------------------------------------------------------------------
template <int R>
struct dft_consts;
template <>
struct dft_consts<5> {
  static constexpr float c[5] = {1.0f, 0.30901699437494745f, -0.8090169943749473f,
                                 -0.8090169943749476f, 0.30901699437494723f};
  static constexpr float s[5] = {0.0f, 0.9510565162951535f, 0.5877852522924732f,
                                 -0.587785252292473f, -0.9510565162951536f};
};
template <>
struct dft_consts<7> {
  static constexpr float c[7] = {1.0f, 0.6234898018587336f, -0.22252093395631434f,
                                 -0.900968867902419f, -0.9009688679024191f,
                                 -0.2225209339563146f, 0.6234898018587334f};
  static constexpr float s[7] = {0.0f, 0.7818314824680298f, 0.9749279121818236f,
                                 0.43388373911755823f, -0.433883739117558f,
                                 -0.9749279121818236f, -0.7818314824680299f};
};

template <int R>
__device__ __forceinline__ void dft(float2* v, bool inv);

template <>
__device__ __forceinline__ void dft<2>(float2* v, bool) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <>
__device__ __forceinline__ void dft<4>(float2* v, bool inv) {
  const float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
  const float2 s13 = cadd(v[1], v[3]), d13 = mul_mi(csub(v[1], v[3]), inv);
  v[0] = cadd(s02, s13);
  v[2] = csub(s02, s13);
  v[1] = cadd(d02, d13);
  v[3] = csub(d02, d13);
}
template <>
__device__ __forceinline__ void dft<8>(float2* v, bool inv) {
  const float h = 0.7071067811865476f;
  float2 a[4], b[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    a[k] = cadd(v[k], v[k + 4]);
    b[k] = csub(v[k], v[k + 4]);
  }
  // b_k *= W8^k
  b[1] = inv ? make_float2(h * (b[1].x - b[1].y), h * (b[1].x + b[1].y))
             : make_float2(h * (b[1].x + b[1].y), h * (b[1].y - b[1].x));
  b[2] = mul_mi(b[2], inv);
  b[3] = inv ? make_float2(-h * (b[3].x + b[3].y), h * (b[3].x - b[3].y))
             : make_float2(h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y));
  dft<4>(a, inv);
  dft<4>(b, inv);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    v[2 * k] = a[k];
    v[2 * k + 1] = b[k];
  }
}
template <>
__device__ __forceinline__ void dft<3>(float2* v, bool inv) {
  const float s3 = 0.8660254037844386f;
  const float2 t1 = cadd(v[1], v[2]);
  const float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  const float2 d = csub(v[1], v[2]);
  // -i s3 d (forward) / +i s3 d (inverse)
  const float2 t3 = mul_mi(make_float2(s3 * d.x, s3 * d.y), inv);
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}
template <int R>
__device__ __forceinline__ void dft_generic(float2* v, bool inv) {
  float2 y[R];
#pragma unroll
  for (int k = 0; k < R; k++) {
    float2 acc = v[0];
#pragma unroll
    for (int j = 1; j < R; j++) {
      const int m = (j * k) % R;
      const float c = dft_consts<R>::c[m];
      const float s = inv ? dft_consts<R>::s[m] : -dft_consts<R>::s[m];
      acc.x += v[j].x * c - v[j].y * s;
      acc.y += v[j].x * s + v[j].y * c;
    }
    y[k] = acc;
  }
#pragma unroll
  for (int k = 0; k < R; k++) v[k] = y[k];
}
template <>
__device__ __forceinline__ void dft<5>(float2* v, bool inv) { dft_generic<5>(v, inv); }
template <>
__device__ __forceinline__ void dft<7>(float2* v, bool inv) { dft_generic<7>(v, inv); }

// Composite radices R = R1 R2 computed in registers (a two-level
// Cooley-Tukey split: R2 DFTs of length R1 over the stride-R2 elements,
// twiddles exp(-+2 pi i n2 k1 / R), then R1 DFTs of length R2), so one
// Stockham stage through LDS does the work of two.  The twiddles are
// compile-time constants: cos and sin of 2 pi m / R from their Taylor series
// in double precision (|angle| <= pi / 4 after octant reduction, 14 terms),
// rounded once to float.
constexpr double kpi = 3.14159265358979323846;
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 14; k++) {
    t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 14; k++) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
// cos and sin of 2 pi m / R, exact at the multiples of pi / 4 that need it
constexpr void cis_of(int m, int R, double& c, double& s) {
  m %= R;
  // angle 2 pi m / R = (pi / 4) * (8 m / R): octant o and remainder r (in
  // units of pi / 4) from the exact rational 8 m / R
  const int o = (8 * m) / R;
  const double r = (double)(8 * m - o * R) / (double)R;  // in [0, 1)
  double a = r * kpi / 4.0, cr = 0, sr = 0;
  if (r > 0.5) {  // reflect within the octant: keeps |angle| <= pi / 8
    a = (1.0 - r) * kpi / 4.0;
    // cos(pi/4 - a) and sin(pi/4 - a)
    const double h = 0.70710678118654752440;
    const double ca = taylor_cos(a), sa = taylor_sin(a);
    cr = h * (ca + sa);
    sr = h * (ca - sa);
  } else {
    cr = taylor_cos(a);
    sr = taylor_sin(a);
  }
  // rotate by o * pi / 4
  const double h = 0.70710678118654752440;
  double oc = 1, os = 0;
  switch (o) {
    case 0: oc = 1; os = 0; break;
    case 1: oc = h; os = h; break;
    case 2: oc = 0; os = 1; break;
    case 3: oc = -h; os = h; break;
    case 4: oc = -1; os = 0; break;
    case 5: oc = -h; os = -h; break;
    case 6: oc = 0; os = -1; break;
    default: oc = h; os = -h; break;
  }
  if (r == 0.0) {
    c = oc;
    s = os;
  } else {
    c = oc * cr - os * sr;
    s = os * cr + oc * sr;
  }
}
template <int R>
struct cis_table {
  float c[R], s[R];
  constexpr cis_table() : c(), s() {
    for (int m = 0; m < R; m++) {
      double cc = 0, ss = 0;
      cis_of(m, R, cc, ss);
      c[m] = (float)cc;
      s[m] = (float)ss;
    }
  }
};
template <int R>
struct cis_const {
  static constexpr cis_table<R> t{};
};

template <int R1, int R2>
__device__ __forceinline__ void dft_split(float2* v, bool inv) {
  constexpr int R = R1 * R2;
  float2 t[R];
#pragma unroll
  for (int n2 = 0; n2 < R2; n2++) {
    float2 u[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; n1++) u[n1] = v[n2 + R2 * n1];
    dft<R1>(u, inv);
#pragma unroll
    for (int k1 = 0; k1 < R1; k1++) {
      const int m = (n2 * k1) % R;
      if (m == 0) {
        t[k1 * R2 + n2] = u[k1];
      } else {
        // exp(-+2 pi i m / R)
        const float c = cis_const<R>::t.c[m];
        const float s = inv ? cis_const<R>::t.s[m] : -cis_const<R>::t.s[m];
        t[k1 * R2 + n2] = cmul(u[k1], make_float2(c, s));
      }
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; k1++) {
    float2 w[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; n2++) w[n2] = t[k1 * R2 + n2];
    dft<R2>(w, inv);
#pragma unroll
    for (int k2 = 0; k2 < R2; k2++) v[k1 + R1 * k2] = w[k2];
  }
}
template <>
__device__ __forceinline__ void dft<6>(float2* v, bool inv) { dft_split<2, 3>(v, inv); }
template <>
__device__ __forceinline__ void dft<9>(float2* v, bool inv) { dft_split<3, 3>(v, inv); }
template <>
__device__ __forceinline__ void dft<10>(float2* v, bool inv) { dft_split<2, 5>(v, inv); }
template <>
__device__ __forceinline__ void dft<12>(float2* v, bool inv) { dft_split<4, 3>(v, inv); }
template <>
__device__ __forceinline__ void dft<14>(float2* v, bool inv) { dft_split<2, 7>(v, inv); }
template <>
__device__ __forceinline__ void dft<15>(float2* v, bool inv) { dft_split<3, 5>(v, inv); }
template <>
__device__ __forceinline__ void dft<16>(float2* v, bool inv) { dft_split<4, 4>(v, inv); }

// ---------------------------------------------------------------------------
// LDS tile: CT columns of length n, interleaved: element j of column c at
// j * (CT + 1) + c.  Threads take (column, row) = (t % CT, t / CT), so both the
// strided global accesses (CT consecutive columns) and the butterflies touch
// consecutive LDS words.
// ---------------------------------------------------------------------------
#define LIDX(j, c) (__umul24((j), CT + 1) + (c))  // j < 1024: a 24-bit multiply

// one self-sorting (Stockham) stage, in place: every thread keeps its
// butterflies in registers across the barrier
template <int R, int CT, int MAXE, int NTH = IMF_WG>
__device__ __forceinline__ void fft_stage(float2* X, const float2* tw, const imf_fft_len& L,
                                          int s, bool inv) {
  constexpr int JR = NTH / CT;
  constexpr int IT = (MAXE + R - 1) / R;
  float2 reg[IT * R];
  const int n = L.n;
  const int nb = n / R;
  const int Ns = L.Ns[s];
  const float invNs = L.invNs[s];
  const int step = L.step[s];
  const int c = threadIdx.x % CT;
  const int j0 = threadIdx.x / CT;
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int j = j0 + it * JR;
    if (j < nb) {
      float2 v[R];
#pragma unroll
      for (int k = 0; k < R; k++) v[k] = X[LIDX(j + k * nb, c)];
      if (Ns > 1) {
        const int jd = (int)(((float)j + 0.5f) * invNs);
        const int jm = j - jd * Ns;
#pragma unroll
        for (int k = 1; k < R; k++) {
          float2 w = tw[jm * k * step];
          if (inv) w.y = -w.y;
          v[k] = cmul(v[k], w);
        }
      }
      dft<R>(v, inv);
#pragma unroll
      for (int k = 0; k < R; k++) reg[it * R + k] = v[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int j = j0 + it * JR;
    if (j < nb) {
      const int jd = (int)(((float)j + 0.5f) * invNs);
      const int jm = j - jd * Ns;
      const int idx = jd * Ns * R + jm;
#pragma unroll
      for (int k = 0; k < R; k++) X[LIDX(idx + k * Ns, c)] = reg[it * R + k];
    }
  }
  __syncthreads();
}

// compile-time stage plan of a length n = 2^a 3^b 5^c 7^d: radix 8 while
// three factors of 2 remain, then the leftover power of two (1, 2 or 4) joined
// to the smallest odd prime when the product is at most 16 (2x3, 2x5, 2x7,
// 4x3), the odd primes paired while their product is at most 16 (3x3, 3x5),
// and a leftover 2 with no odd prime joined to the last 8 (16): three stages
// for most lengths up to 1024 (384 = 8 8 6, 288 = 8 12 3, 1024 = 8 8 16)
constexpr int ct_radix_split(int n, int idx) {
  int e2 = 0;
  while (n % 2 == 0) {
    n /= 2;
    e2++;
  }
  int odd[16] = {0}, no = 0;
  for (int p = 3; p <= 7; p += 2)
    while (n % p == 0) {
      n /= p;
      odd[no++] = p;
    }
  if (n != 1) return 1;
  int rs[24] = {0}, ns = 0;
  while (e2 >= 3) {
    rs[ns++] = 8;
    e2 -= 3;
  }
  int lf = 1 << e2;
  int i = 0;
  if (lf > 1 && no > 0 && lf * odd[0] <= 16) {
    rs[ns++] = lf * odd[0];
    lf = 1;
    i = 1;
  }
  while (i < no) {
    if (i + 1 < no && odd[i] * odd[i + 1] <= 16) {
      rs[ns++] = odd[i] * odd[i + 1];
      i += 2;
    } else {
      rs[ns++] = odd[i++];
    }
  }
  if (lf > 1) {
    if (lf == 2 && ns > 0 && rs[0] == 8 && no == 0)
      rs[0] = 16;
    else
      rs[ns++] = lf;
  }
  return idx < ns ? rs[idx] : 1;
}
// the base plan: radices 8, 4, 2, 3, 5, 7 in that order (one stage per
// factor, no composite radices)
constexpr int ct_radix_base(int n, int idx) {
  int s = 0;
  const int rs[6] = {8, 4, 2, 3, 5, 7};
  for (int r = 0; r < 6; r++)
    while (n % rs[r] == 0) {
      if (s == idx) return rs[r];
      n /= rs[r];
      s++;
    }
  return 1;
}
// radix of stage idx of length n under split 0 (composite) or 1 (base)
constexpr int ct_radix(int n, int idx, int split) {
  return split ? ct_radix_base(n, idx) : ct_radix_split(n, idx);
}
constexpr int ct_nstages(int n, int split) {
  int s = 0;
  while (ct_radix(n, s, split) > 1) s++;
  return s;
}
constexpr int ct_ns(int n, int idx, int split) {
  int p = 1;
  for (int i = 0; i < idx; i++) p *= ct_radix(n, i, split);
  return p;
}

// one stage with every size known at compile time
template <int R, int N, int NS, int CT, int NTH = IMF_WG>
__device__ __forceinline__ void fft_stage_ct(float2* X, const float2* tw, bool inv) {
  constexpr int JR = NTH / CT;
  constexpr int NB = N / R;
  constexpr int IT = (NB + JR - 1) / JR;
  constexpr int STEP = N / (NS * R);
  float2 reg[IT * R];
  const int c = threadIdx.x % CT;
  const int j0 = threadIdx.x / CT;
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int j = j0 + it * JR;
    if (IT * JR == NB || j < NB) {
      float2 v[R];
#pragma unroll
      for (int k = 0; k < R; k++) v[k] = X[LIDX(j + k * NB, c)];
      if (NS > 1) {
        const int jm = j % NS;
#pragma unroll
        for (int k = 1; k < R; k++) {
          float2 w = tw[jm * k * STEP];
          if (inv) w.y = -w.y;
          v[k] = cmul(v[k], w);
        }
      }
      dft<R>(v, inv);
#pragma unroll
      for (int k = 0; k < R; k++) reg[it * R + k] = v[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int j = j0 + it * JR;
    if (IT * JR == NB || j < NB) {
      const int jm = j % NS;
      const int idx = (j - jm) * R + jm;
#pragma unroll
      for (int k = 0; k < R; k++) X[LIDX(idx + k * NS, c)] = reg[it * R + k];
    }
  }
  __syncthreads();
}

template <int N, int CT, int S, int NTH, int SPLIT>
__device__ __forceinline__ void fft_stages_ct(float2* X, const float2* tw, bool inv) {
  if constexpr (S < ct_nstages(N, SPLIT)) {
    fft_stage_ct<ct_radix(N, S, SPLIT), N, ct_ns(N, S, SPLIT), CT, NTH>(X, tw, inv);
    fft_stages_ct<N, CT, S + 1, NTH, SPLIT>(X, tw, inv);
  }
}

// Transform all CT columns of the tile: NT > 0 is a compile-time length
// (stage plan SPLIT), NT == 0 the run-time plan L.
template <int CT, int MAXE, int NT, int NTH = IMF_WG, int SPLIT = 0>
__device__ void fft_tile(float2* X, const float2* tw, const imf_fft_len& L, bool inv) {
  if constexpr (NT > 0) {
    fft_stages_ct<NT, CT, 0, NTH, SPLIT>(X, tw, inv);
  } else {
    for (int s = 0; s < L.nstages; s++) {
      switch (L.radix[s]) {
        case 8: fft_stage<8, CT, MAXE, NTH>(X, tw, L, s, inv); break;
        case 4: fft_stage<4, CT, MAXE, NTH>(X, tw, L, s, inv); break;
        case 2: fft_stage<2, CT, MAXE, NTH>(X, tw, L, s, inv); break;
        case 3: fft_stage<3, CT, MAXE, NTH>(X, tw, L, s, inv); break;
        case 5: fft_stage<5, CT, MAXE, NTH>(X, tw, L, s, inv); break;
        case 7: fft_stage<7, CT, MAXE, NTH>(X, tw, L, s, inv); break;
        default: break;
      }
    }
  }
}

__device__ __forceinline__ void load_twiddles(float2* tw_lds, const float2* tw, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw_lds[i] = tw[i];
}

// The hardware deals workgroups to the 8 XCDs round robin.  Column-tile
// kernels are launched on a flat grid of 8 * ceil(GX*GY*GZ / 8) workgroups and
// remap so that each XCD walks a contiguous range of (tile, plane, orientation)
// triples: neighbouring column tiles, which share 128-byte lines, meet in the
// same L2.
__device__ __forceinline__ bool xcd_blocks(int GX, int GY, int GZ, int& bx, int& by, int& bz) {
  const long long total = (long long)GX * GY * GZ;
  const long long per = (total + 7) / 8;
  const long long id = blockIdx.x;
  const long long lg = (id % 8) * per + id / 8;
  if (lg >= total) return false;
  bx = (int)(lg % GX);
  const long long r = lg / GX;
  by = (int)(r % GY);
  bz = (int)(r / GY);
  return true;
}
static inline unsigned xcd_grid(long long GX, long long GY, long long GZ) {
  return (unsigned)((GX * GY * GZ + 7) / 8 * 8);
}

// min of v and the value of the lane N below in the same 16-lane row; the
// row's first N lanes keep v.  One VALU instruction with a DPP row shift on
// its first operand: without bound_ctrl a lane whose source lies outside its
// row is not written, so it keeps its own value.  Every lane of the wave must
// be active.  The nop gives the two wait states a DPP read needs after a
// VALU write of the same register.
template <int N>
__device__ __forceinline__ float dpp_min_shr(float v) {
  static_assert(N == 1 || N == 2 || N == 4 || N == 8, "row shift");
  if constexpr (N == 1)
    asm volatile("s_nop 1\n\tv_min_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf"
                 : "+v"(v));
  else if constexpr (N == 2)
    asm volatile("s_nop 1\n\tv_min_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf"
                 : "+v"(v));
  else if constexpr (N == 4)
    asm volatile("s_nop 1\n\tv_min_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf"
                 : "+v"(v));
  else
    asm volatile("s_nop 1\n\tv_min_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf"
                 : "+v"(v));
  return v;
}

__device__ __forceinline__ int pmod(long long a, int n) {
  long long r = a % n;
  return (int)(r < 0 ? r + n : r);
}

// ---------------------------------------------------------------------------
// twiddle tables: tw[m] = exp(-2 pi i m / n), computed in float64
// ---------------------------------------------------------------------------
__global__ void k_twiddles(float2* tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) {
    double s, c;
    sincospi(2.0 * (double)m / (double)n, &s, &c);
    tw[m] = make_float2((float)c, (float)-s);
  }
}

hipError_t imf_launch_twiddles(float2* tw, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, tw, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// (1) forward x pass of the obstacle field: rho_O = max(design, fixture),
//     two real rows per complex column, output rows of px/2 + 1 values
// ---------------------------------------------------------------------------
template <int CT, int MAXE, int NT>
__global__ void __launch_bounds__(IMF_WG) k_fwd_x_r2c(imf_fwd_design_args a, imf_fft_len L,
                                                      const float2* __restrict__ twg) {
  extern __shared__ float2 smem[];
  const int n = L.n, h = n / 2 + 1;
  float2* X = smem;
  float2* tw = smem + (CT + 1) * n;
  load_twiddles(tw, twg, n);
  const long long rows = (long long)a.ny * a.nz;
  const long long row0 = (long long)blockIdx.x * 2 * CT;
  for (int i = threadIdx.x; i < 2 * CT * n; i += IMF_WG) {
    const int rr = i / n, x = i - rr * n;
    const long long row = row0 + rr;
    float v = 0.f;
    if (row < rows && x < a.nx) {
      const long long idx = row * a.nx + x;
      const float d = a.density ? ((const float*)a.design)[idx]
                                : (float)((const uint8_t*)a.design)[idx];
      const bool fx = a.fixture && a.fixture[idx];
      v = fx ? 1.0f : d;
    }
    float* p = (float*)&X[LIDX(x, rr >> 1)];
    p[rr & 1] = v;
  }
  __syncthreads();
  fft_tile<CT, MAXE, NT>(X, tw, L, false);
  for (int i = threadIdx.x; i < 2 * CT * h; i += IMF_WG) {
    const int rr = i / h, k = i - rr * h;
    const long long row = row0 + rr;
    if (row >= rows) continue;
    const float2 A = X[LIDX(k, rr >> 1)];
    const float2 Bc = X[LIDX(k == 0 ? 0 : n - k, rr >> 1)];
    const float2 B = make_float2(Bc.x, -Bc.y);
    float2 out;
    if ((rr & 1) == 0) {
      out = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y + B.y));
    } else {
      const float2 d = csub(A, B);
      out = make_float2(0.5f * d.y, -0.5f * d.x);
    }
    a.work1[row * h + k] = out;
  }
}

// ---------------------------------------------------------------------------
// (2) generic strided pass: columns are CT consecutive elements (stride 1)
//     of a plane; element j of a column sits at j * jstride.
//     Input j < n_in goes to position (j + shift_in) mod n; output j' < n_out
//     comes from position (j' + shift_out) mod n.
// ---------------------------------------------------------------------------
struct strided_io {
  const float2* in;
  long long in_q, in_plane, in_j;
  float2* out;
  long long out_q, out_plane, out_j;
  int ncols;
};

// pass kinds for the per-orientation geometry
enum { PASS_DESIGN_Y = 0, PASS_TOOL_Y = 1, PASS_INV_Y = 2 };

template <int CT, int MAXE, int NT, int KIND, int NTH = IMF_WG, int SPLIT = 0>
__global__ void __launch_bounds__(NTH) k_pass_strided(strided_io io, imf_fft_len L,
                                                         const float2* __restrict__ twg,
                                                         const imf_orient_desc* __restrict__ desc,
                                                         int planes_fixed, int n_in_fixed,
                                                         int n_out_fixed, int inv_arg, int GX,
                                                         int GY, int GZ) {
  extern __shared__ float2 smem[];
  // the inverse y pass and the tool's forward y pass have a fixed direction
  // (compile time: no per-twiddle select); the design pass takes it as given
  const int inv = KIND == PASS_INV_Y ? 1 : (KIND == PASS_TOOL_Y ? 0 : inv_arg);
  const int n = NT > 0 ? NT : L.n;
  int bx, plane, q;
  if (!xcd_blocks(GX, GY, GZ, bx, plane, q)) return;
  int planes = planes_fixed, n_in = n_in_fixed, n_out = n_out_fixed, sh_in = 0, sh_out = 0;
  if (KIND == PASS_TOOL_Y) {
    planes = desc[q].tdim[2];
    n_in = desc[q].tdim[1];
    sh_in = pmod(desc[q].tlo[1], n);
  } else if (KIND == PASS_INV_Y) {
    planes = desc[q].box_dim[2];
    n_out = desc[q].box_dim[1];
    sh_out = pmod(desc[q].box_lo[1], n);
  }
  if (plane >= planes) return;
  float2* X = smem;
  float2* tw = smem + (CT + 1) * n;
  const int c0 = bx * CT;
  const float2* in = io.in + q * io.in_q + plane * io.in_plane + c0;
  float2* out = io.out + q * io.out_q + plane * io.out_plane + c0;
  if constexpr (NT > 0) {
    // every load of the tile in flight at once (registers), the twiddles
    // behind them, then into LDS
    constexpr int PE = (CT * NT + NTH - 1) / NTH;
    float2 v[PE];
#pragma unroll
    for (int e = 0; e < PE; e++) {
      const int i = threadIdx.x + e * NTH;
      const int j = i / CT, c = i - j * CT;
      v[e] = make_float2(0.f, 0.f);
      if (j < n_in && c0 + c < io.ncols)
        v[e] = KIND == PASS_DESIGN_Y ? in[(long long)j * io.in_j + c]
                                     : in[__umul24(j, (unsigned)io.in_j) + c];
    }
    load_twiddles(tw, twg, n);
#pragma unroll
    for (int e = 0; e < PE; e++) {
      const int i = threadIdx.x + e * NTH;
      const int j = i / CT, c = i - j * CT;
      if (j < NT) {
        int pos = j + sh_in;
        if (pos >= NT) pos -= NT;
        X[LIDX(pos, c)] = v[e];
      }
    }
    __syncthreads();
    fft_tile<CT, MAXE, NT, NTH, SPLIT>(X, tw, L, inv != 0);
#pragma unroll
    for (int e = 0; e < PE; e++) {
      const int i = threadIdx.x + e * NTH;
      const int j = i / CT, c = i - j * CT;
      int pos = j + sh_out;
      if (pos >= NT) pos -= NT;
      if (j < n_out) v[e] = X[LIDX(pos, c)];
    }
#pragma unroll
    for (int e = 0; e < PE; e++) {
      const int i = threadIdx.x + e * NTH;
      const int j = i / CT, c = i - j * CT;
      if (j < n_out && c0 + c < io.ncols) {
        if (KIND == PASS_DESIGN_Y)
          out[(long long)j * io.out_j + c] = v[e];
        else
          out[__umul24(j, (unsigned)io.out_j) + c] = v[e];
      }
    }
  } else {
    load_twiddles(tw, twg, n);
    for (int i = threadIdx.x; i < CT * n; i += NTH) {
      const int j = i / CT, c = i - j * CT;
      float2 v = make_float2(0.f, 0.f);
      if (j < n_in && c0 + c < io.ncols) v = in[j * io.in_j + c];
      int pos = j + sh_in;
      if (pos >= n) pos -= n;
      X[LIDX(pos, c)] = v;
    }
    __syncthreads();
    fft_tile<CT, MAXE, NT, NTH, SPLIT>(X, tw, L, inv != 0);
    for (int i = threadIdx.x; i < CT * n_out; i += NTH) {
      const int j = i / CT, c = i - j * CT;
      if (c0 + c >= io.ncols) continue;
      int pos = j + sh_out;
      if (pos >= n) pos -= n;
      out[j * io.out_j + c] = X[LIDX(pos, c)];
    }
  }
}

// ---------------------------------------------------------------------------
// (3) forward z pass: strided input (plane stride), contiguous output columns
//     out[ky][kx][kz].  The tile is CT consecutive kx at one ky.
// ---------------------------------------------------------------------------
template <int CT, int MAXE, int NT, int TOOL, int NTH = IMF_WG>
__global__ void __launch_bounds__(NTH) k_pass_z_fwd(const float2* __restrict__ in,
                                                       long long in_q, long long in_j,
                                                       float2* __restrict__ out, int h,
                                                       int n_in_fixed, imf_fft_len L,
                                                       const float2* __restrict__ twg,
                                                       const imf_orient_desc* __restrict__ desc,
                                                       long long spec_q_fixed, int GX, int GY,
                                                       int GZ) {
  extern __shared__ float2 smem[];
  const int n = L.n;
  int bx, ky, q;
  if (!xcd_blocks(GX, GY, GZ, bx, ky, q)) return;
  int n_in = n_in_fixed, sh = 0;
  float2* obase = out + q * spec_q_fixed;
  if (TOOL) {
    n_in = desc[q].tdim[2];
    sh = pmod(desc[q].tlo[2], n);
    obase = desc[q].spec;
  }
  float2* X = smem;
  float2* tw = smem + (CT + 1) * n;
  load_twiddles(tw, twg, n);
  const int c0 = bx * CT;
  // element (j, ky, kx) of the input at j * in_j + ky * h + kx
  const float2* src = in + q * in_q + (long long)ky * h + c0;
  for (int i = threadIdx.x; i < CT * n; i += NTH) {
    const int j = i / CT, c = i - j * CT;
    float2 v = make_float2(0.f, 0.f);
    if (j < n_in && c0 + c < h) v = src[j * in_j + c];
    int pos = j + sh;
    if (pos >= n) pos -= n;
    X[LIDX(pos, c)] = v;
  }
  __syncthreads();
  fft_tile<CT, MAXE, NT, NTH>(X, tw, L, false);
  float2* dst = obase + ((long long)ky * h + c0) * n;
  const int ncol = min(CT, h - c0);
  for (int i = threadIdx.x; i < ncol * n; i += NTH) {
    const int c = i / n, k = i - c * n;
    dst[(long long)c * n + k] = X[LIDX(k, c)];
  }
}

// ---------------------------------------------------------------------------
// (4) tool x pass: direct DFT of the x-runs of T.  One thread per (run, kx)
//     sums all runs of its row when it holds the row's first run.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(IMF_WG) k_tool_x(const imf_orient_desc* __restrict__ desc,
                                                   const float2* __restrict__ tw, int px,
                                                   float2* __restrict__ work1, long long w1_q,
                                                   int max_ty) {
  const int q = blockIdx.y;
  const imf_orient_desc& d = desc[q];
  const int h = px / 2 + 1;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long r = idx / h;
  const int k = (int)(idx - r * h);
  if (r >= d.n_truns) return;
  const imf_run* rl = d.truns;
  const imf_run me = rl[r];
  if (r > 0 && rl[r - 1].y == me.y && rl[r - 1].z == me.z) return;
  float2 acc = make_float2(0.f, 0.f);
  for (long long rr = r; rr < d.n_truns; rr++) {
    const imf_run u = rl[rr];
    if (u.y != me.y || u.z != me.z) break;
    int m = pmod((long long)k * u.x, px);
    for (int j = 0; j < u.len; j++) {
      const float2 w = tw[m];
      acc.x += w.x;
      acc.y += w.y;
      m += k;
      if (m >= px) m -= px;
    }
  }
  const int iy = me.y - d.tlo[1], iz = me.z - d.tlo[2];
  work1[q * w1_q + ((long long)iz * max_ty + iy) * h + k] = acc;
}

// ---------------------------------------------------------------------------
// (5) fused spectral product + inverse z pass.  rho_hat and the tool spectrum
//     are read as contiguous columns; Y = rho_hat conj(T) / (px py pz) is
//     inverted along z and the query-box range of z is written strided.
//     The rho_hat tile is kept in registers and reused for every orientation
//     of the batch.
// ---------------------------------------------------------------------------
// FUSE: some orientations of the batch have no spectrum (desc.tmid set);
// the instance without it is the all-cached path
template <int CT, int MAXE, int NT, int NTH = IMF_WG, int SPLIT = 0, bool FUSE = false>
__global__ void __launch_bounds__(NTH) k_inv_z_product(imf_inv_args a, imf_fft_len L,
                                                          const float2* __restrict__ twg, int GX,
                                                          int GY) {
  extern __shared__ float2 smem[];
  const int n = NT > 0 ? NT : L.n;
  const int h = a.px / 2 + 1;
  if (a.cellmin) {  // the x pass lowers these cell minima by atomic min
    const long long nc = (long long)a.nq * a.cell_stride;
    for (long long i = (long long)blockIdx.x * NTH + threadIdx.x; i < nc;
         i += (long long)gridDim.x * NTH)
      a.cellmin[i] = IMF_ORD_INF;
  }
  int bx, ky, bz;
  if (!xcd_blocks(GX, GY, 1, bx, ky, bz)) return;
  const int c0 = bx * CT;
  const int ncol = min(CT, h - c0);
  float2* X = smem;
  float2* tw = smem + (CT + 1) * n;
  load_twiddles(tw, twg, n);
  const float scale = 1.0f / ((float)a.px * (float)a.py * (float)a.pz);
  const float2* rsrc = a.rho_hat + ((long long)ky * h + c0) * n;
  constexpr int RE = NT > 0 ? (CT * NT + NTH - 1) / NTH : MAXE;
  float2 rho[RE];
#pragma unroll
  for (int e = 0; e < RE; e++) {
    const int i = threadIdx.x + e * NTH;
    rho[e] = i < ncol * n ? rsrc[i] : make_float2(0.f, 0.f);
  }
  // the next orientation's tool spectrum tile is loaded into registers while
  // the current one is transformed
  float2 tp[RE];
  auto fetch = [&](int q) {
    if (FUSE && a.desc[q].tmid) return;  // generated in LDS instead
    const float2* tsrc = a.desc[q].spec + ((long long)ky * h + c0) * n;
#pragma unroll
    for (int e = 0; e < RE; e++) {
      const int i = threadIdx.x + e * NTH;
      tp[e] = i < ncol * n ? tsrc[i] : make_float2(0.f, 0.f);
    }
  };
  if (a.nq > 0) fetch(0);
  for (int q = 0; q < a.nq; q++) {
    const imf_orient_desc& d = a.desc[q];
    __syncthreads();
    if (FUSE && d.tmid) {  // uniform: the tool column tile from its x and y transforms
      // the tdim z rows it has (the tool placed at z offset tlo), zero
      // elsewhere, transformed forward along z here: the same transform the
      // spectrum would have been computed with
      const float2* src = d.tmid + (long long)ky * h + c0;
      const int nin = d.tdim[2], shz = pmod(d.tlo[2], n);
      const unsigned ps = (unsigned)(a.py * h);  // plane stride, < 2^24
      for (int i = threadIdx.x; i < CT * n; i += NTH) {
        const int j = i / CT, c = i - j * CT;
        float2 v = make_float2(0.f, 0.f);
        if (j < nin && c < ncol) v = src[__umul24(j, ps) + c];
        int pos = j + shz;
        if (pos >= n) pos -= n;
        X[LIDX(pos, c)] = v;
      }
      __syncthreads();
      fft_tile<CT, MAXE, NT, NTH, SPLIT>(X, tw, L, false);
#pragma unroll
      for (int e = 0; e < RE; e++) {
        const int i = threadIdx.x + e * NTH;
        if (i < CT * n) {
          const int c = i / n, k = i - c * n;
          const float2 t = X[LIDX(k, c)];
          const float2 r = rho[e];
          X[LIDX(k, c)] =
              make_float2((r.x * t.x + r.y * t.y) * scale, (r.y * t.x - r.x * t.y) * scale);
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < RE; e++) {
        const int i = threadIdx.x + e * NTH;
        if (i < CT * n) {
          const int c = i / n, k = i - c * n;
          const float2 t = tp[e];
          const float2 r = rho[e];
          // r * conj(t) * scale (zero past the last column: both are zero there)
          X[LIDX(k, c)] =
              make_float2((r.x * t.x + r.y * t.y) * scale, (r.y * t.x - r.x * t.y) * scale);
        }
      }
    }
    if (q + 1 < a.nq) fetch(q + 1);
    __syncthreads();
    fft_tile<CT, MAXE, NT, NTH, SPLIT>(X, tw, L, true);
    const int mz = d.box_dim[2];
    const int sh = pmod(d.box_lo[2], n);
    float2* dst = a.w1 + q * a.w1_stride + (long long)ky * h + c0;
    // a plane of w1 holds py (px/2 + 1) < 2^24 elements, an orientation's
    // planes fewer than 2^31: 24-bit multiplies, 32-bit offsets
    const unsigned zs = (unsigned)(a.py * h);
    for (int i = threadIdx.x; i < CT * mz; i += NTH) {
      const int z = i / CT, c = i - z * CT;
      if (c >= ncol) continue;
      int pos = z + sh;
      if (pos >= n) pos -= n;
      dst[__umul24(z, zs) + c] = X[LIDX(pos, c)];
    }
  }
}

// ---------------------------------------------------------------------------
// (6) inverse x pass (complex-to-real, two rows per complex column) with the
//     rounding / guard-band epilogue.  Writes g over the query box.
// ---------------------------------------------------------------------------
// The compile-time plans are held to 8 waves per SIMD: the epilogue's scalar
// state would otherwise take the SGPR count just past that occupancy's limit
// (the few scalars over it live in vector lanes instead).
template <int CT, int MAXE, int NT, int NTH = IMF_WG, int SPLIT = 0, bool DEFER = false>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(NT > 0 ? 8 : 1)))
k_inv_x_c2r(imf_inv_args a, imf_fft_len L, const float2* __restrict__ twg) {
  extern __shared__ float2 smem[];
  const int n = NT > 0 ? NT : L.n, h = n / 2 + 1;
  const int q = blockIdx.z;
  const imf_orient_desc& d = a.desc[q];
  // box rows (my mz <= 2^20) and voxels (< 2^31) fit 32-bit indices
  const int mx = d.box_dim[0], my = d.box_dim[1], mz = d.box_dim[2];
  const int rows = my * mz;
  const int row0 = blockIdx.x * 2 * CT;
  if (row0 >= rows) return;
  float2* X = smem;
  float2* tw = smem + (CT + 1) * n;
  const float2* src = a.w2 + q * a.w2_stride;
  // the tile's 2 CT half-spectrum rows: every load in flight at once
  // (registers), the twiddles behind them, then into LDS
  constexpr int PE = NT > 0 ? (CT * (NT / 2 + 1) + NTH - 1) / NTH : MAXE;
  float2 A[PE], B[PE];
  // ra / my through a float reciprocal: ra < 2^21 (box rows <= 2^20), so the
  // float (ra + 1/2) / my is within 2^-23 ra / my < 1 / (4 my) of its value,
  // less than the 1 / (2 my) that separates it from an integer
  const float inv_my = 1.0f / (float)my;
#pragma unroll
  for (int e = 0; e < PE; e++) {
    const int i = threadIdx.x + e * NTH;
    const int c = i / h, k = i - c * h;
    const int ra = row0 + 2 * c;
    // rows ra and ra + 1 of the box: (z, y) of the first, the second follows
    const int za = (int)(((float)ra + 0.5f) * inv_my), ya = ra - (int)__umul24(za, my);
    const int zb = ya + 1 == my ? za + 1 : za, yb = ya + 1 == my ? 0 : ya + 1;
    A[e] = make_float2(0.f, 0.f);
    B[e] = make_float2(0.f, 0.f);
    // element indices of one orientation's rows: max_mz max_my (px/2 + 1) <
    // 2^31, rows and row lengths < 2^24 (24-bit multiplies)
    if (i < CT * h) {
      if (ra < rows) A[e] = src[__umul24(__umul24(za, a.max_my) + ya, h) + k];
      if (ra + 1 < rows) B[e] = src[__umul24(__umul24(zb, a.max_my) + yb, h) + k];
    }
  }
  load_twiddles(tw, twg, n);
#pragma unroll
  for (int e = 0; e < PE; e++) {
    const int i = threadIdx.x + e * NTH;
    const int c = i / h, k = i - c * h;
    if (i < CT * h) {
      // Z(k) = A + iB;  Z(n-k) = conj(A) + i conj(B)
      X[LIDX(k, c)] = make_float2(A[e].x - B[e].y, A[e].y + B[e].x);
      if (k > 0 && k < n - k) X[LIDX(n - k, c)] = make_float2(A[e].x + B[e].y, B[e].x - A[e].y);
    }
  }
  __syncthreads();
  fft_tile<CT, MAXE, NT, NTH, SPLIT>(X, tw, L, true);
  const int sh = pmod(d.box_lo[0], n);
  float* dst = a.g + q * a.g_stride;
  float local_err = 0.f;
  // Each wave takes whole rows, 64 consecutive x at a time (chunks aligned to
  // the box's x = 0, so the bound's cells, whose widths divide 64, never
  // straddle a chunk); the row's coordinates are wave-uniform (scalar) and the
  // cell minima are reduced across lanes by DPP row shifts.
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nch = (mx + 63) >> 6;
  const int gl = a.cellmin ? min(a.cwx, 16) : 16;  // lanes per reduced group
  const int cdx = (mx + a.cwx - 1) / a.cwx + 1, cdy = (my + a.cwy - 1) / a.cwy + 1;
  // the row's value at tile position j is float FS j + rr of the tile
  // (complex column rr / 2, real part for even rr, imaginary for odd)
  constexpr unsigned FS = 2 * (CT + 1);  // floats per tile row
  const float* Xf = reinterpret_cast<const float*>(X);
  const unsigned tile_end = (unsigned)n * FS;
  // (z, y) of the tile's first row; a wave's rows follow by counting
  const int z0 = row0 / my, y0 = row0 - z0 * my;
  // One 64-voxel chunk of a row: its values (rounded when binary) and which
  // of them are rare entries, overlaps to recompute exactly (guard band) and
  // entries of the expected threshold's bracket.  FULL: every lane lies
  // inside the row.
  struct ChunkVals {
    float v;
    bool in, flag, brk;
  };
  auto eval = [&](unsigned i0, int ch, auto full) {
    constexpr bool FULL = decltype(full)::value;
    ChunkVals c;
    const int x = ch * 64 + lane;
    c.in = FULL || x < mx;
    // tile position (x + sh) mod n: for x < mx, x + sh < 2n and below n the
    // unsigned difference wraps above the sum (rr < FS); lanes past the row's
    // end read an in-tile value that is discarded
    const unsigned t = i0 + (unsigned)ch * (64 * FS);
    c.v = Xf[FULL ? min(t, t - tile_end) : min(min(t, t - tile_end), tile_end - 1)];
    c.flag = false;
    if (a.binary) {
      const float G = rintf(c.v);
      const float e = c.in ? fabsf(c.v - G) : 0.f;
      local_err = fmaxf(local_err, e);
      c.flag = e > a.delta;
      c.v = G;
    } else if (a.nth) {  // within either band (the second repeats the first for one)
      c.flag = c.in & ((fabsf(c.v - a.fth_c[0]) <= a.fth_r[0]) |
                       (fabsf(c.v - a.fth_c[1]) <= a.fth_r[1]));
    }
    c.brk = a.blist && c.in && c.v > a.fblo && c.v <= a.fbhi;
    return c;
  };
  // The rare entries are appended where they are found (an atomic per chunk
  // that has any), or with DEFER only counted here (wave-wide ballots), with
  // a bit per chunk that has any: the wave then reserves its list slots with
  // one atomic per list at the end and writes the entries in a second sweep
  // over those chunks (the tile stays in LDS).  An atomic per chunk makes the
  // wave wait for its return, and with it for every store it has in flight:
  // with many entries (a wide bracket) the deferred form is faster, with few
  // the immediate one, whose loop keeps fewer scalars live.
  unsigned long long emask = 0;  // bit 16 rowi + chunk (rows of this wave)
  int nflag = 0, nbrk = 0;
  const bool track = nch <= 16 && 2 * CT <= 4 * (NTH / 64);  // the mask holds every chunk
  int rowi = 0;
  for (int rr = wave; rr < 2 * CT; rr += NTH / 64, rowi++) {
    const int row = row0 + rr;
    if (row >= rows) break;
    int zz = z0, yy = y0 + rr;
    while (yy >= my) {
      yy -= my;
      zz++;
    }
    float* drow = dst + (long long)row * mx;
    unsigned int* cmrow =
        a.cellmin
            ? a.cellmin + q * a.cell_stride + ((zz >> a.lcwz) * cdy + (yy >> a.lcwy)) * cdx
            : nullptr;
    const unsigned i0 = __umul24((unsigned)(lane + sh), FS) + (unsigned)rr;
    auto chunk = [&](int ch, auto full) {
      constexpr bool FULL = decltype(full)::value;
      const int x = ch * 64 + lane;
      ChunkVals c = eval(i0, ch, full);
      if (__builtin_expect(__ballot(c.flag | c.brk) != 0, 0)) {
        if constexpr (DEFER) {
          nflag += __popcll(__ballot(c.flag));
          nbrk += __popcll(__ballot(c.brk));
          if (track) emask |= 1ull << (16 * rowi + ch);
        } else {
          const int li = row * mx + x;
          if (c.flag) {
            const int slot = atomicAdd(a.flag_cnt, 1);
            if (slot < a.flag_cap) a.flags[slot] = make_int2(q, li);
          }
          if (c.brk) {  // spread over the orientation's lists by workgroup
            const long long sl =
                (long long)(a.q0 + q) * IMF_BR_SLICES + (blockIdx.x % IMF_BR_SLICES);
            const unsigned slot = atomicAdd(a.bcnt + sl, 1u);
            if (slot < (unsigned)a.bslot)
              a.blist[sl * a.bslot + slot] = make_int4(a.q0 + q, li, __float_as_int(c.v), 0);
          }
        }
      }
      float v = c.v;
      if (FULL) {
        drow[x] = v;
      } else {
        if (c.in) drow[x] = v;
        v = c.in ? v : INFINITY;
      }
      if (cmrow) {
        // minima of the row's cells over the values just written (rounded
        // when binary; +inf past the row's end), one atomic min per group of
        // gl lanes; the recheck lowers a cell again when it corrects a value
        float m = dpp_min_shr<1>(v);
        m = dpp_min_shr<2>(m);
        m = dpp_min_shr<4>(m);
        if (gl == 16) m = dpp_min_shr<8>(m);
        if ((lane & (gl - 1)) == gl - 1 && (FULL || x - (gl - 1) < mx))
          atomicMin(cmrow + ((unsigned)x >> a.lcwx), f2ord(m));
      }
    };
    const int nfull = mx >> 6;
    for (int ch = 0; ch < nfull; ch++) chunk(ch, std::true_type{});
    if (nfull < nch) chunk(nfull, std::false_type{});
  }
  if (DEFER && (nflag | nbrk)) {  // wave-uniform
    // bracket lists: spread over the orientation's slices by workgroup
    const long long sl = (long long)(a.q0 + q) * IMF_BR_SLICES + (blockIdx.x % IMF_BR_SLICES);
    int fbase = 0;
    unsigned bbase = 0;
    if (lane == 0) {
      if (nflag) fbase = atomicAdd(a.flag_cnt, nflag);
      if (nbrk) bbase = atomicAdd(a.bcnt + sl, (unsigned)nbrk);
    }
    fbase = __shfl(fbase, 0);
    bbase = (unsigned)__shfl((int)bbase, 0);
    const unsigned long long below = (1ull << lane) - 1ull;
    rowi = 0;
    for (int rr = wave; rr < 2 * CT; rr += NTH / 64, rowi++) {
      const int row = row0 + rr;
      if (row >= rows) break;
      const unsigned i0 = __umul24((unsigned)(lane + sh), FS) + (unsigned)rr;
      for (int ch = 0; ch < nch; ch++) {
        if (track && !((emask >> (16 * rowi + ch)) & 1ull)) continue;
        const ChunkVals c = eval(i0, ch, std::false_type{});
        const unsigned long long bf = __ballot(c.flag), bb = __ballot(c.brk);
        const int li = row * mx + ch * 64 + lane;
        if (c.flag) {
          const int slot = fbase + __popcll(bf & below);
          if (slot < a.flag_cap) a.flags[slot] = make_int2(q, li);
        }
        if (c.brk) {
          const unsigned slot = bbase + (unsigned)__popcll(bb & below);
          if (slot < (unsigned)a.bslot)
            a.blist[sl * a.bslot + slot] = make_int4(a.q0 + q, li, __float_as_int(c.v), 0);
        }
        fbase += __popcll(bf);
        bbase += (unsigned)__popcll(bb);
      }
    }
  }
  if (a.binary) {
    for (int o = 32; o > 0; o >>= 1) local_err = fmaxf(local_err, __shfl_xor(local_err, o));
    // a statistic only: most waves are below the running maximum, so read it
    // first and leave the contended atomic to the few that raise it
    if ((threadIdx.x & 63) == 0 &&
        __float_as_uint(local_err) > __atomic_load_n(a.max_err_bits, __ATOMIC_RELAXED))
      atomicMax(a.max_err_bits, __float_as_uint(local_err));
  }
}

// ---------------------------------------------------------------------------
// dispatch on the transform length (CT columns x MAXE elements per thread)
// ---------------------------------------------------------------------------
// Dispatch on the transform length: compile-time plans for the lengths the
// planner prefers, the run-time plan otherwise.  CT columns per tile; MAXE
// elements per thread bound the run-time path's registers.
#define CASE_N(NV, CTV, MAXEV, ...)                   \
  case NV: {                                          \
    constexpr int NT = NV, CT = CTV, MAXE = MAXEV;    \
    __VA_ARGS__;                                      \
  } break;
#define DISPATCH(n, ...)                                   \
  do {                                                     \
    switch (n) {                                           \
      CASE_N(64, 16, 16, __VA_ARGS__)                      \
      CASE_N(96, 16, 16, __VA_ARGS__)                      \
      CASE_N(128, 16, 16, __VA_ARGS__)                     \
      CASE_N(160, 16, 16, __VA_ARGS__)                     \
      CASE_N(192, 16, 16, __VA_ARGS__)                     \
      CASE_N(216, 16, 16, __VA_ARGS__)                     \
      CASE_N(224, 16, 16, __VA_ARGS__)                     \
      CASE_N(256, 16, 16, __VA_ARGS__)                     \
      CASE_N(288, 8, 16, __VA_ARGS__)                      \
      CASE_N(320, 8, 16, __VA_ARGS__)                      \
      CASE_N(384, 8, 16, __VA_ARGS__)                      \
      CASE_N(448, 8, 16, __VA_ARGS__)                      \
      CASE_N(512, 8, 16, __VA_ARGS__)                      \
      CASE_N(576, 8, 32, __VA_ARGS__)                      \
      CASE_N(640, 8, 32, __VA_ARGS__)                      \
      CASE_N(768, 8, 32, __VA_ARGS__)                      \
      CASE_N(1024, 8, 32, __VA_ARGS__)                     \
      default:                                             \
        if ((n) <= 256) {                                  \
          constexpr int NT = 0, CT = 16, MAXE = 16;        \
          __VA_ARGS__;                                     \
        } else if ((n) <= 512) {                           \
          constexpr int NT = 0, CT = 16, MAXE = 32;        \
          __VA_ARGS__;                                     \
        } else {                                           \
          constexpr int NT = 0, CT = 8, MAXE = 32;         \
          __VA_ARGS__;                                     \
        }                                                  \
    }                                                      \
  } while (0)

// threads per workgroup of the per-orientation passes (tool spectra and the
// inverse transform): twice the default, so each thread keeps half the
// butterflies in registers and a CU holds more waves to hide HBM latency
#ifndef IMF_INV_NTH
#define IMF_INV_NTH 512
#endif

// Transform plans of the inverse passes, chosen per pass by the autotuner:
// bit 0 the stage plan (0: composite radices, three stages for most lengths;
// 1: one stage per factor 8, 4, 2, 3, 5, 7), bit 1 the tile (0: the default
// CT columns with IMF_INV_NTH threads; 1: half the columns with half the
// threads, twice the workgroups per CU).  Plans other than 0 exist for the
// lengths 192 to 768; elsewhere every plan is plan 0.  Inside, NTHP and SPLIT
// are the workgroup size and the stage plan.
#define CASE_P(NV, CTV, MAXEV, NTHV, SPV, ...)                              \
  case NV: {                                                                \
    constexpr int NT = NV, CT = CTV, MAXE = MAXEV, NTHP = NTHV, SPLIT = SPV; \
    __VA_ARGS__;                                                            \
  }                                                                         \
    done = true;                                                            \
    break;
#define PLAN_LENGTHS(SPV, NTHV, HALF, ...)                                      \
  CASE_P(192, 16 / HALF, 16, NTHV, SPV, __VA_ARGS__)                            \
  CASE_P(216, 16 / HALF, 16, NTHV, SPV, __VA_ARGS__)                            \
  CASE_P(256, 16 / HALF, 16, NTHV, SPV, __VA_ARGS__)                            \
  CASE_P(288, 8 / HALF, 16, NTHV, SPV, __VA_ARGS__)                             \
  CASE_P(320, 8 / HALF, 16, NTHV, SPV, __VA_ARGS__)                             \
  CASE_P(384, 8 / HALF, 16, NTHV, SPV, __VA_ARGS__)                             \
  CASE_P(448, 8 / HALF, 16, NTHV, SPV, __VA_ARGS__)                             \
  CASE_P(512, 8 / HALF, 16, NTHV, SPV, __VA_ARGS__)                             \
  CASE_P(576, 8 / HALF, 32, NTHV, SPV, __VA_ARGS__)                             \
  CASE_P(640, 8 / HALF, 32, NTHV, SPV, __VA_ARGS__)                             \
  CASE_P(768, 8 / HALF, 32, NTHV, SPV, __VA_ARGS__)
#define DISPATCH_PLAN(n, plan, ...)                                   \
  do {                                                                \
    bool done = false;                                                \
    switch ((plan) & 3) {                                             \
      case 1:                                                         \
        switch (n) { PLAN_LENGTHS(1, IMF_INV_NTH, 1, __VA_ARGS__) }   \
        break;                                                        \
      case 2:                                                         \
        switch (n) { PLAN_LENGTHS(0, IMF_INV_NTH / 2, 2, __VA_ARGS__) } \
        break;                                                        \
      case 3:                                                         \
        switch (n) { PLAN_LENGTHS(1, IMF_INV_NTH / 2, 2, __VA_ARGS__) } \
        break;                                                        \
      default: break;                                                 \
    }                                                                 \
    if (!done) {                                                      \
      constexpr int NTHP = IMF_INV_NTH, SPLIT = 0;                    \
      DISPATCH(n, __VA_ARGS__);                                       \
    }                                                                 \
  } while (0)

// transform lengths with plans other than 0 (the lengths of PLAN_LENGTHS)
bool imf_fft_plan_variants(int n) {
  switch (n) {
    case 192: case 216: case 256: case 288: case 320: case 384: case 448: case 512: case 576:
    case 640: case 768:
      return true;
    default:
      return false;
  }
}

static size_t smem_bytes(int n, int ct) { return (size_t)((ct + 1) * n + n) * sizeof(float2); }

static hipError_t set_smem(const void* fn, size_t bytes) {
  if (bytes > 64 * 1024)
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipSuccess;
}

// Workgroups of one inverse pass (0 product + z, 1 y, 2 x) of length n under
// a transform plan that fit one CU at once (registers and LDS), 0 if unknown.
static int inverse_pass_occupancy(int pass, int n, int plan) {
  int nb = 0;
  DISPATCH_PLAN(n, plan, {
    const size_t sm = smem_bytes(n, CT);
    const void* k = pass == 0 ? (const void*)k_inv_z_product<CT, MAXE, NT, NTHP, SPLIT, false>
                    : pass == 1
                        ? (const void*)k_pass_strided<CT, MAXE, NT, PASS_INV_Y, NTHP, SPLIT>
                        : (const void*)k_inv_x_c2r<CT, MAXE, NT, NTHP, SPLIT, false>;
    if (set_smem(k, sm) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, NTHP, sm) != hipSuccess)
      nb = 0;
  });
  (void)hipGetLastError();
  return nb;
}

// The transform plans of the inverse passes used when no autotuned entry
// sets them: per pass the base radices (plan 1) where their registers let
// more workgroups share a CU than the composite radices' do (at length 576
// the composite y pass holds 85 VGPRs, two workgroups per CU, the base one 80,
// three: 161 -> 122 ms per 384^3 x 512 iteration), else plan 0.
int imf_fft_default_plan(int pz, int py, int px) {
  static std::mutex mu;
  static std::map<long long, int> memo;
  const long long key = ((long long)pz << 40) | ((long long)py << 20) | px;
  std::lock_guard<std::mutex> lk(mu);
  auto it = memo.find(key);
  if (it != memo.end()) return it->second;
  int plan = 0;
  const int len[3] = {pz, py, px};
  for (int pass = 0; pass < 3; pass++) {
    if (!imf_fft_plan_variants(len[pass])) continue;
    const int b0 = inverse_pass_occupancy(pass, len[pass], 0);
    const int b1 = inverse_pass_occupancy(pass, len[pass], 1);
    if (b0 > 0 && b1 > b0) plan |= 1 << (2 * pass);
  }
  memo[key] = plan;
  return plan;
}

hipError_t imf_launch_fwd_design(const imf_fwd_design_args& a, const imf_fft_len& fx,
                                 const imf_fft_len& fy, const imf_fft_len& fz,
                                 const float2* twx, const float2* twy, const float2* twz,
                                 hipStream_t s) {
  const int h = a.px / 2 + 1;
  hipError_t e;
  DISPATCH(fx.n, {
    const long long rows = (long long)a.ny * a.nz;
    const size_t sm = smem_bytes(fx.n, CT);
    auto k = k_fwd_x_r2c<CT, MAXE, NT>;
    if ((e = set_smem((const void*)k, sm)) != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)((rows + 2 * CT - 1) / (2 * CT))), dim3(IMF_WG), sm, s,
                       a, fx, twx);
  });
  if ((e = hipGetLastError()) != hipSuccess) return e;
  DISPATCH(fy.n, {
    strided_io io{a.work1, 0, (long long)a.ny * h, h, a.work2, 0, (long long)a.py * h, h, h};
    const size_t sm = smem_bytes(fy.n, CT);
    auto k = k_pass_strided<CT, MAXE, NT, PASS_DESIGN_Y>;
    if ((e = set_smem((const void*)k, sm)) != hipSuccess) return e;
    const int GX = (h + CT - 1) / CT;
    hipLaunchKernelGGL(k, dim3(xcd_grid(GX, a.nz, 1)), dim3(IMF_WG), sm, s, io, fy, twy,
                       (const imf_orient_desc*)nullptr, a.nz, a.ny, a.py, 0, GX, a.nz, 1);
  });
  if ((e = hipGetLastError()) != hipSuccess) return e;
  DISPATCH(fz.n, {
    const size_t sm = smem_bytes(fz.n, CT);
    auto k = k_pass_z_fwd<CT, MAXE, NT, 0>;
    if ((e = set_smem((const void*)k, sm)) != hipSuccess) return e;
    const int GX = (h + CT - 1) / CT;
    hipLaunchKernelGGL(k, dim3(xcd_grid(GX, a.py, 1)), dim3(IMF_WG), sm, s, a.work2, 0LL,
                       (long long)a.py * h, a.out, h, a.nz, fz, twz,
                       (const imf_orient_desc*)nullptr, 0LL, GX, a.py, 1);
  });
  return hipGetLastError();
}

hipError_t imf_launch_tool_fft(const imf_tool_fft_args& a, const imf_fft_len& fy,
                               const imf_fft_len& fz, const float2* twx, const float2* twy,
                               const float2* twz, hipStream_t s, int stage) {
  const int h = a.px / 2 + 1;
  hipError_t e = hipSuccess;
  // x: direct DFT of the runs (rows without runs stay zero)
  if (stage < 0 || stage == 0) {
    if ((e = hipMemsetAsync(a.work1, 0, sizeof(float2) * a.w1_stride * a.nq, s)) != hipSuccess)
      return e;
    const long long max_runs = (long long)a.max_ty * a.max_tz * IMF_MAX_RUNS_PER_ROW;
    dim3 grid((unsigned)((max_runs * h + IMF_WG - 1) / IMF_WG), a.nq);
    hipLaunchKernelGGL(k_tool_x, grid, dim3(IMF_WG), 0, s, a.desc, twx, a.px, a.work1,
                       a.w1_stride, a.max_ty);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (stage < 0 || stage == 1) DISPATCH(fy.n, {
    strided_io io{a.work1, a.w1_stride, (long long)a.max_ty * h, h,
                  a.work2, a.w2_stride, (long long)a.py * h, h, h};
    const size_t sm = smem_bytes(fy.n, CT);
    auto k = k_pass_strided<CT, MAXE, NT, PASS_TOOL_Y, IMF_INV_NTH>;
    if ((e = set_smem((const void*)k, sm)) != hipSuccess) return e;
    const int GX = (h + CT - 1) / CT;
    hipLaunchKernelGGL(k, dim3(xcd_grid(GX, a.max_tz, a.nq)), dim3(IMF_INV_NTH), sm, s, io, fy, twy,
                       a.desc, 0, 0, a.py, 0, GX, a.max_tz, a.nq);
  });
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (stage < 0 || stage == 2) DISPATCH(fz.n, {
    const size_t sm = smem_bytes(fz.n, CT);
    auto k = k_pass_z_fwd<CT, MAXE, NT, 1, IMF_INV_NTH>;
    if ((e = set_smem((const void*)k, sm)) != hipSuccess) return e;
    const int GX = (h + CT - 1) / CT;
    hipLaunchKernelGGL(k, dim3(xcd_grid(GX, a.py, a.nq)), dim3(IMF_INV_NTH), sm, s, a.work2,
                       a.w2_stride, (long long)a.py * h, (float2*)nullptr, h, 0, fz, twz, a.desc,
                       0LL, GX, a.py, a.nq);
  });
  return hipGetLastError();
}

// float nearest below / above a double (outward rounding of a bound)
static float f_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = std::nextafter(f, -INFINITY);
  return f;
}
static float f_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, INFINITY);
  return f;
}

hipError_t imf_launch_inverse(const imf_inv_args& a_in, const imf_fft_len& fx,
                              const imf_fft_len& fy, const imf_fft_len& fz, const float2* twx,
                              const float2* twy, const float2* twz, hipStream_t s, int stage) {
  imf_inv_args a = a_in;
  // each band (th[k] - band, th[k] + band) as |v - c| <= r in float: c near
  // its middle, r its half-width from c, widened by 2^-20 so that the rounded
  // difference of any float inside stays within r (a superset of the band;
  // what it admits is recomputed exactly); one band: the second repeats it
  for (int k = 0; k < 2; k++) {
    const int kk = a.nth < 2 ? 0 : k;
    const double lo = a.th[kk] - a.band, hi = a.th[kk] + a.band;
    const float c = (float)(0.5 * (lo + hi));
    a.fth_c[k] = c;
    a.fth_r[k] = f_up(std::max(hi - (double)c, (double)c - lo) * (1.0 + 0x1p-20));
  }
  a.fblo = f_down(a.blo);
  a.fbhi = f_up(a.bhi);
  // cell widths are powers of two (the block shapes): shifts
  a.lcwx = a.lcwy = a.lcwz = 0;
  while ((1 << a.lcwx) < a.cwx) a.lcwx++;
  while ((1 << a.lcwy) < a.cwy) a.lcwy++;
  while ((1 << a.lcwz) < a.cwz) a.lcwz++;
  if (a.cellmin &&
      ((1 << a.lcwx) != a.cwx || (1 << a.lcwy) != a.cwy || (1 << a.lcwz) != a.cwz))
    return hipErrorInvalidValue;
  const int h = a.px / 2 + 1;
  hipError_t e = hipSuccess;
  if (stage < 0 || stage == 0) DISPATCH_PLAN(fz.n, a.fplan[0], {
    const size_t sm = smem_bytes(fz.n, CT);
    auto k = a.fused ? k_inv_z_product<CT, MAXE, NT, NTHP, SPLIT, true>
                     : k_inv_z_product<CT, MAXE, NT, NTHP, SPLIT, false>;
    if ((e = set_smem((const void*)k, sm)) != hipSuccess) return e;
    const int GX = (h + CT - 1) / CT;
    hipLaunchKernelGGL(k, dim3(xcd_grid(GX, a.py, 1)), dim3(NTHP), sm, s, a, fz, twz, GX, a.py);
  });
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (stage < 0 || stage == 1) DISPATCH_PLAN(fy.n, a.fplan[1], {
    strided_io io{a.w1, a.w1_stride, (long long)a.py * h, h,
                  a.w2, a.w2_stride, (long long)a.max_my * h, h, h};
    const size_t sm = smem_bytes(fy.n, CT);
    auto k = k_pass_strided<CT, MAXE, NT, PASS_INV_Y, NTHP, SPLIT>;
    if ((e = set_smem((const void*)k, sm)) != hipSuccess) return e;
    const int GX = (h + CT - 1) / CT;
    hipLaunchKernelGGL(k, dim3(xcd_grid(GX, a.max_mz, a.nq)), dim3(NTHP), sm, s, io, fy, twy,
                       a.desc, 0, a.py, 0, 1, GX, a.max_mz, a.nq);
  });
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (stage < 0 || stage == 2) DISPATCH_PLAN(fx.n, a.fplan[2], {
    const size_t sm = smem_bytes(fx.n, CT);
    auto k = a.defer ? k_inv_x_c2r<CT, MAXE, NT, NTHP, SPLIT, true>
                     : k_inv_x_c2r<CT, MAXE, NT, NTHP, SPLIT, false>;
    if ((e = set_smem((const void*)k, sm)) != hipSuccess) return e;
    const long long rows = (long long)a.max_my * a.max_mz;
    hipLaunchKernelGGL(k, dim3((unsigned)((rows + 2 * CT - 1) / (2 * CT)), 1, a.nq), dim3(NTHP),
                       sm, s, a, fx, twx);
  });
  return hipGetLastError();
}

// columns of a [n][ncols] complex array (single-step check entry point)
hipError_t imf_launch_columns(const float2* in, float2* out, int ncols, long long jstride,
                              const imf_fft_len& L, const float2* tw, int inverse, hipStream_t s) {
  hipError_t e;
  DISPATCH(L.n, {
    strided_io io{in, 0, 0, jstride, out, 0, 0, jstride, ncols};
    const size_t sm = smem_bytes(L.n, CT);
    auto k = k_pass_strided<CT, MAXE, NT, PASS_DESIGN_Y>;
    if ((e = set_smem((const void*)k, sm)) != hipSuccess) return e;
    const int GX = (ncols + CT - 1) / CT;
    hipLaunchKernelGGL(k, dim3(xcd_grid(GX, 1, 1)), dim3(IMF_WG), sm, s, io, L, tw,
                       (const imf_orient_desc*)nullptr, 1, L.n, L.n, inverse, GX, 1, 1);
  });
  return hipGetLastError();
}
