// Internal declarations shared by the HIP kernels and the host runtime of the
// IMF library.  Not part of the public interface (include/imf.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define IMF_MAX_RUNS_PER_ROW 4
#define IMF_WG 256
// sharp-point runs the minimum pass stages in LDS per workgroup (the rest are
// read from memory one by one)
#define IMF_MF_LDS_RUNS 1024

// A run of voxels of an oriented tool raster: offsets start + j * e (e a
// coordinate axis, or for the sharp-point runs the lattice vector sv of the
// orientation), 0 <= j < len.  Offsets are relative to the cutter tip.
struct imf_run {
  int x, y, z, len;
};

// Geometry of one oriented tool, as the raster kernels need it.
struct imf_raster_desc {
  int kind;            // 0 flat, 1 ball, 2 2D rectangle, 3 voxel model
  int ndim;
  int lattice;         // 1: exact integer predicate on v, 0: float64 on d
  int sharp;           // 0 all cutter voxels, 1 boundary voxels, 2 tip voxel
  double r, L, rh, LH; // cutter radius/half-width, cutter length, holder radius, L + holder length
  double d[3];         // unit direction (tip toward holder)
  long long v[3];      // lattice direction
  long long vn;        // |v|^2
  long long r2, L2, rh2, LH2;  // doubled sizes (lattice mode)
  int lo[3], dim[3];   // bounding box of the raster in offsets
  int s_axis;          // axis along which the sharp-point runs are formed
  const uint8_t* vox;  // voxel model: device labels [vdim z][y][x], tip at vorg
  int vdim[3], vorg[3];
  double R[9];         // voxel model: rotation, row-major (tool frame to grid)
  long long flags_off; // byte offset of this orientation's flag volume
  long long rows_off;  // offset (in rows) of this orientation's row slots
};

// Extents reported by the raster kernels (atomics): [0..2] min of T, [3..5]
// max of T, [6..8] min of S, [9..11] max of S, [12] |T|, [13] |S|, [14] run
// slot overflow flag, [15] number of x-runs of T, [16] number of runs of S
// along s_axis, [17] number of x-runs of S.
#define IMF_EXT_INTS 20

// Order-preserving map of float to unsigned int (atomic min / max of floats,
// and cell minima that several workgroups lower).
__device__ __forceinline__ unsigned int f2ord(float f) {
  // negative: every bit flipped; otherwise the sign bit set
  const unsigned int b = __float_as_uint(f);
  return b ^ ((unsigned int)((int)b >> 31) | 0x80000000u);
}
__device__ __forceinline__ float ord2f(unsigned int u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
#define IMF_ORD_INF 0xFF800000u  // f2ord(+infinity)

// Integer floor and ceiling of p / q for q > 0.
__host__ __device__ inline int imf_floor_div(int p, int q) {
  return p >= 0 ? p / q : -((-p + q - 1) / q);
}
__host__ __device__ inline int imf_ceil_div(int p, int q) { return -imf_floor_div(-p, q); }

// Lattice lines of a query box along v (v[1] or v[2] nonzero), as the
// streamed level pass walks them.  Seed axis a is z if v[2] != 0, else y;
// every lattice line meets the window of |v[a]| planes at the entry side of
// axis a (a in [0, |v[a]|) if v[a] > 0, else the last |v[a]| planes) in
// exactly one point, its seed (x, b, a), and from there steps s = 0, 1, ...
// of +v.  Seeds of lines that can meet the box: b in [lob, lob + nb0), x in
// chunks of 64 from lox.  Waves: (x chunk, b, residue of a).
struct imf_vlines {
  int a, b, ua, S;  // seed axis, the other of y / z, |v[a]|, steps covering axis a
  int lob, nb0, lox, nxc;
  long long waves;
};
__host__ __device__ inline imf_vlines imf_vlines_of(const int v[3], const int dim[3]) {
  imf_vlines L;
  L.a = v[2] != 0 ? 2 : 1;
  L.b = L.a == 2 ? 1 : 2;
  L.ua = v[L.a] < 0 ? -v[L.a] : v[L.a];
  L.S = imf_ceil_div(dim[L.a], L.ua);
  const int vb = v[L.b], vx = v[0];
  L.lob = vb > 0 ? -vb * (L.S - 1) : 0;
  L.nb0 = dim[L.b] + (vb < 0 ? -vb : vb) * (L.S - 1);
  L.lox = vx > 0 ? -vx * (L.S - 1) : 0;
  L.nxc = imf_ceil_div(dim[0] + (vx < 0 ? -vx : vx) * (L.S - 1), 64);
  L.waves = (long long)L.nxc * L.nb0 * L.ua;
  return L;
}

// Per-orientation data used by the correlation, min filter and masks.
struct imf_orient_desc {
  int box_lo[3];       // first translation of the query box (t = x - k)
  int box_dim[3];      // query box size M per axis
  int s_axis;          // axis of the sharp-point runs (0, 1, 2), or 3: along sv
  int sv[3];           // lattice vector of the sharp-point runs (e_axis for an axis)
  int n_sruns;         // number of sharp-point runs
  int n_sruns1;        // the first n_sruns1 have power-of-two lengths (one lookup each)
  int n_truns;         // number of tool x-runs
  int tlo[3], tdim[3]; // bounding box of the tool raster (offsets)
  int nlvl;            // sparse-table levels this orientation's runs need
  unsigned lvl_used;   // bit s-1 set: some run reads level s (others are not stored)
  int out_q;           // index of the orientation in the request (masks, gamma stack)
  int set;             // fixture set of the orientation (its prefix sums)
  const imf_run* sruns;  // sharp-point runs along sv (x-runs for the sweep route)
  const imf_run* truns;  // x-runs of the tool T, row order (z, y)
  float2* spec;          // this orientation's tool spectrum [py][px/2+1][pz]
  // or (spectrum not kept): the tool after its x and y transforms,
  // [tdim z][py][px/2+1] at this address; the product pass finishes the z
  // transform of each column tile in LDS instead of reading a spectrum
  const float2* tmid;
};

// Logical block order of the sharp-point minimum: bricks of 128 x 16 x 16
// voxels (x chunk slowest, then z, y fastest), blocks of WX x WY x WZ voxels
// inside a brick x, y, z fastest first.
struct mf_geom {
  int WX, WY, WZ;
  int nbx, nby, nbz;      // blocks per axis
  int brx, bry, brz;      // blocks per brick and axis
  int nry, nrz;           // bricks along y, z
  long long nlog;         // logical indices (bricks x blocks per brick)
  __host__ __device__ mf_geom(int wx, int wy, int wz, int nx, int ny, int nz)
      : WX(wx), WY(wy), WZ(wz) {
    nbx = (nx + wx - 1) / wx;
    nby = (ny + wy - 1) / wy;
    nbz = (nz + wz - 1) / wz;
    brx = 128 / wx;
    bry = 16 / wy < nby ? 16 / wy : nby;
    brz = 16 / wz < nbz ? 16 / wz : nbz;
    const int nrx = (nbx + brx - 1) / brx;
    nry = (nby + bry - 1) / bry;
    nrz = (nbz + brz - 1) / brz;
    nlog = (long long)nrx * nry * nrz * brx * bry * brz;
  }
  // block -> logical index (the inverse of block())
  __device__ __forceinline__ long long logical(int bx, int by, int bz) const {
    const long long brick = ((long long)(bx / brx) * nrz + bz / brz) * nry + by / bry;
    const int wib = ((bz % brz) * bry + by % bry) * brx + bx % brx;
    return brick * (brx * bry * brz) + wib;
  }
  // logical index -> block (false for the padding of partial bricks)
  __device__ __forceinline__ bool block(long long lg, int& bx, int& by, int& bz) const {
    const int br = brx * bry * brz;
    const long long brick = lg / br;
    const int wib = (int)(lg - brick * br);
    const int ry = (int)(brick % nry);
    const long long r = brick / nry;
    const int rz = (int)(r % nrz);
    const int rx = (int)(r / nrz);
    bx = rx * brx + wib % brx;
    by = ry * bry + (wib / brx) % bry;
    bz = rz * brz + wib / (brx * bry);
    return bx < nbx && by < nby && bz < nbz;
  }
};

// One x-run of T at translation t: the prefix-sum row and the two indices
// whose difference is the run's sum.  A run outside the grid (or clipped to
// nothing) gets row 0 and indices 0, 0 (a difference of 0), so callers load
// without branching.
__device__ __forceinline__ void exact_run_terms(const imf_run u, const long long* ps, int nx,
                                                int ny, int nz, int tx, int ty, int tz,
                                                const long long*& row, int& a0, int& a1) {
  const int y = ty + u.y, z = tz + u.z;
  const int x0 = max(tx + u.x, 0), x1 = min(tx + u.x + u.len, nx);
  const bool ok = y >= 0 && y < ny && z >= 0 && z < nz && x1 > x0;
  row = ps + ((long long)(ok ? z : 0) * ny + (ok ? y : 0)) * (nx + 1);
  a0 = ok ? x0 : 0;
  a1 = ok ? x1 : 0;
}

// exact overlap at translation t: sum over x-runs of T of row sums (Eq. ident).
// Four runs at a time, their loads in flight together (the integer sum does
// not depend on the order).
__device__ __forceinline__ long long exact_overlap(const imf_orient_desc& d,
                                                   const long long* __restrict__ ps, int nx,
                                                   int ny, int nz, int tx, int ty, int tz) {
  const imf_run* rl = d.truns;
  const int n = d.n_truns;
  long long s = 0;
  int r = 0;
  for (; r + 4 <= n; r += 4) {
    long long hi[4], lo[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const long long* row;
      int a0, a1;
      exact_run_terms(rl[r + k], ps, nx, ny, nz, tx, ty, tz, row, a0, a1);
      hi[k] = row[a1];
      lo[k] = row[a0];
    }
#pragma unroll
    for (int k = 0; k < 4; k++) s += hi[k] - lo[k];
  }
  for (; r < n; r++) {
    const long long* row;
    int a0, a1;
    exact_run_terms(rl[r], ps, nx, ny, nz, tx, ty, tz, row, a0, a1);
    s += row[a1] - row[a0];
  }
  return s;
}

__device__ __forceinline__ float wave_max_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// FFT plan for one transform length: stages of the self-sorting transform.
// Stage s has radix[s], Ns[s] = product of the earlier radices, and
// step[s] = n / (Ns[s] * radix[s]) (twiddle index stride).
struct imf_fft_len {
  int n;               // length
  int nstages;
  int radix[8];
  int Ns[8];
  int step[8];
  float invNs[8];
};

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
hipError_t imf_launch_raster(const imf_raster_desc* d_desc, int n_orient, int max_vol,
                             uint8_t* flags, int* ext, hipStream_t s);
hipError_t imf_launch_sharp_subset(const imf_raster_desc* d_desc, int n_orient, int max_vol,
                                   uint8_t* flags, int* ext, hipStream_t s);
// Runs of one kind for every orientation: list 0 = x-runs of T, list 1 =
// runs of S along s_axis, list 2 = x-runs of S.  Row slots hold up to
// IMF_MAX_RUNS_PER_ROW runs per row; rows_off of the descriptor indexes them.
hipError_t imf_launch_runs(const imf_raster_desc* d_desc, int n_orient, int max_rows,
                           const uint8_t* flags, imf_run* slots, int* cnt, int* ext,
                           hipStream_t s);
// Compact the row slots into one list per (orientation, kind) at out_base.
hipError_t imf_launch_compact(const imf_raster_desc* d_desc, int n_orient, int max_rows,
                              const imf_run* slots, const int* cnt,
                              const long long* out_base /* [n_orient][3] */, imf_run* out,
                              hipStream_t s);

hipError_t imf_launch_twiddles(float2* tw, int n, hipStream_t s);
// transform the columns of a [n][ncols] complex array (element j at j * jstride)
hipError_t imf_launch_columns(const float2* in, float2* out, int ncols, long long jstride,
                              const imf_fft_len& L, const float2* tw, int inverse, hipStream_t s);

// forward R2C 3D FFT of the obstacle field rho_O = max(design, fixture)
struct imf_fwd_design_args {
  const void* design; int density; const uint8_t* fixture;
  int nx, ny, nz;
  int px, py, pz;
  float2* work1;  // [nz][ny][px/2+1]
  float2* work2;  // [nz][py][px/2+1]
  float2* out;    // [py][px/2+1][pz]
};
hipError_t imf_launch_fwd_design(const imf_fwd_design_args& a, const imf_fft_len& fx,
                                 const imf_fft_len& fy, const imf_fft_len& fz,
                                 const float2* twx, const float2* twy, const float2* twz,
                                 hipStream_t s);

// tool spectra of a batch of orientations into desc.spec
struct imf_tool_fft_args {
  const imf_orient_desc* desc; int nq;
  int px, py, pz;
  int max_ty, max_tz;     // max tool bbox extents over the batch
  float2* work1;          // per q: [max_tz][max_ty][px/2+1]
  float2* work2;          // per q: [max_tz][py][px/2+1]
  long long w1_stride, w2_stride;
};
// stage: -1 all, 0 x (direct DFT of the runs), 1 y pass, 2 z pass
hipError_t imf_launch_tool_fft(const imf_tool_fft_args& a, const imf_fft_len& fy,
                               const imf_fft_len& fz, const float2* twx, const float2* twy,
                               const float2* twz, hipStream_t s, int stage = -1);

// inverse: g_q = C2R3D(rho_hat * conj(T_q)) / (px py pz), over the query boxes
struct imf_inv_args {
  const imf_orient_desc* desc; int nq;
  const float2* rho_hat;  // [py][px/2+1][pz]
  int px, py, pz;
  int max_mx, max_my, max_mz;
  float2* w1; long long w1_stride;   // per q: [max_mz][py][px/2+1]
  float2* w2; long long w2_stride;   // per q: [max_mz][max_my][px/2+1]
  float* g; long long g_stride;      // per q: [mz][my][mx] packed with the q's own dims
  // epilogue
  int binary;           // 1: round to integers and flag |g - rint g| > delta
  float delta;
  int nth;              // density: thresholds known in advance (0-2); flag |g - th| <= band
  double th[2], band;
  unsigned int* max_err_bits;        // atomic max of |g - rint g| (binary)
  int* flag_cnt; int flag_cap; int2* flags;   // (q, linear box index)
  // optional: minima of g over the bound's cells (cwx x cwy x cwz, aligned to
  // the box), per q [cdz][cdy][cdx] as f2ord values, lowered by atomic min
  unsigned int* cellmin; long long cell_stride; int cwx, cwy, cwz;
  // optional (density at lambda F_max with an expected threshold): overlaps
  // with blo < g <= bhi appended as (q0 + q, box index, g bits, 0) to one of
  // IMF_BR_SLICES lists per orientation (slice of the workgroup: the appends
  // spread over many counters), list s at blist + s * bslot, count bcnt[s]
  int4* blist; unsigned int* bcnt; int bslot; double blo, bhi; int q0;
  // transform plan of the z, y and x passes (0-3: bit 0 base radices instead
  // of composite ones, bit 1 half-width tiles); 0 is the default
  int fplan[3];
  // 1: some descriptors of the batch carry tmid (no spectrum)
  int fused;
  // 1: the x pass counts its guard-band and bracket entries and writes them
  // after its rows, with one list reservation per wave (many entries expected)
  int defer;
  // set by imf_launch_inverse from the fields above, so float compares
  // select a superset of the double intervals: |g - fth_c[k]| <= fth_r[k]
  // for (th[k] - band, th[k] + band), fblo < g <= fbhi (bounds rounded
  // outward) for (blo, bhi]; log2 of cwx, cwy, cwz
  float fth_c[2], fth_r[2], fblo, fbhi;
  int lcwx, lcwy, lcwz;
};
#define IMF_BR_SLICES 64
// true when the inverse passes of length n have transform plans other than 0
bool imf_fft_plan_variants(int n);
// transform plans (z | y << 2 | x << 4) of the inverse passes used when no
// autotuned entry sets them (by occupancy of each pass's kernels)
int imf_fft_default_plan(int pz, int py, int px);
// stage: -1 all, 0 product + z pass, 1 y pass, 2 x pass (complex-to-real) + epilogue
hipError_t imf_launch_inverse(const imf_inv_args& a, const imf_fft_len& fx,
                              const imf_fft_len& fy, const imf_fft_len& fz, const float2* twx,
                              const float2* twy, const float2* twz, hipStream_t s,
                              int stage = -1);

// exact overlap by prefix sums along x (direct correlation and guard-band recheck)
// bad (may be null): counts design voxels outside the representable value
// set (binary: > 1; density: outside [0, 1] or off the 2^-24 grid)
hipError_t imf_launch_prefix_x(const void* design, int density, const uint8_t* fixture, int nx,
                               int ny, int nz, long long* ps, unsigned int* bad, hipStream_t s);
// density: the exact value rounded to float32, then moved by ulps where needed
// so that g32 <= th equals g <= th for each of the nth known thresholds
hipError_t imf_launch_direct(const imf_orient_desc* desc, int nq, const long long* ps, int nx,
                             int ny, int nz, int density, float* g, long long g_stride,
                             int max_vol, int nth, double th0, double th1, hipStream_t s);
hipError_t imf_launch_recheck(const imf_orient_desc* desc, const long long* ps, int nx, int ny, int nz, int density,
                              const int* flag_cnt, const int2* flags, int flag_cap,
                              int nth, double th0, double th1, float* g, long long g_stride,
                              unsigned int* cellmin, long long cell_stride, int cwx, int cwy,
                              int cwz, unsigned int* err_bits, hipStream_t s);

// sharp-point min filter with running minimum, masks, optional gamma stack
struct imf_min_args {
  const imf_orient_desc* desc; int nq;
  const float* g; long long g_stride;
  float* lvl; long long lvl_stride; int nlvl;   // sparse-table levels per q
  int max_m;                // largest box extent along any run axis (LDS of the level pass)
  long long max_lines;      // workgroups of the level pass (LDS form: x lines)
  long long stream_waves;   // waves of the streamed level pass (y and z lines)
  long long vstream_waves;  // waves of the level pass along lattice vectors
  long long x_rows;         // rows of the shuffle level pass (x lines)
  int lds_levels;           // some orientation needs more levels than the register forms
  int nx, ny, nz;
  float* f;                 // running min [nz][ny][nx]
  const uint8_t* omega0;    // [nz][ny][nx]
  int masks_on; double theta; uint64_t* masks;  // masks, indexed by each descriptor's out_q
  float* gamma_stack;                  // optional, indexed by out_q
  // branch and bound: the output is cut into blocks of the wave shape; for
  // every orientation a lower bound of gamma over a block is the minimum of g
  // over the coarse cells (same shape, aligned to the query box) that cover
  // block - S.  Blocks whose bound is >= their maximum of f, and above the
  // mask threshold bound, cannot change f or set a mask bit and are skipped.
  int bnb;                  // 0: plain, 1: branch and bound
  int shape;                // wave block: 0 = 64x1x1, 1 = 32x2x1, 2 = 16x2x2, 3 = 16x4x1
  unsigned int* cellmin; long long cell_stride;   // per q: [cdz][cdy][cdx], f2ord values
  int cellmin_fused;                    // 1: the inverse x pass and the recheck wrote them
  long long cell_waves;                    // waves of the cell-minimum pass (largest box)
  int* fp; int fp_cap;                     // per q: [0] count, then cell-index offsets
  float* fblock;            // max of f per block (+inf before the first orientation)
  int* list; long long list_stride;  // per q: blocks left to compute, packed
                                     // bx | by << 10 | bz << 21
  int* count;               // per q: length of that list
  int* kept;                // statistics: list length per global orientation, or NULL
  unsigned long long* wmask; int* woff; long long wstride;  // per q and 64 logical blocks:
                            // kept-block bits of the bound pass, exclusive list offsets
  unsigned int* fmax_up;    // two-phase: max of f over all voxels at the start of the batch
                            // (order-preserving bits; lambda times it bounds the threshold)
  double theta_lambda;      // lambda of the threshold bound lambda * fmax_up
  double e_theta;           // bound E on the float32 overlap error (0: exact overlaps)
  double fmargin;           // skip only where the bound exceeds max f by this (0: >=)
  int theta_known;
  int q0;                   // global index of the batch's first orientation
  int n_cu, wg_per_cu;      // resident workgroups of the list pass: CUs x per CU
  unsigned long long* skipped;  // statistics: skipped (block, orientation) pairs
  unsigned long long* keepbits;  // per orientation (request order): kept-block bits, or NULL
  int sync_waves;               // list pass: 0, or 1 / 2 for 4 / 8 waves per workgroup in step
  // compact gamma stack (with keepbits): the kept blocks of each orientation
  // only, 64 values per block in list order from gbase[out_q] (-1: the pool
  // of gcap floats overflowed, *gover set, no values stored); koff[out_q]
  // holds the list offset of every 64 logical blocks (their exclusive
  // prefix of kept blocks).  gbase NULL: gamma_stack is [out_q][N].
  long long* gbase; int* koff; unsigned long long* gused; unsigned int* gover;
  long long gcap;
};
// stage 0: sparse-table levels of the batch (and cell minima, footprints and
// the threshold bound with branch and bound); stage 1: the bound pass of
// orientation q (branch and bound only); stage 2: the minimum pass of
// orientation q; -1: everything for every orientation of the batch
hipError_t imf_launch_minfilter(const imf_min_args& a, hipStream_t s, int stage = -1, int q = 0);
// blocks of the output for a wave shape
void imf_block_dims(int shape, int& wx, int& wy, int& wz);
// logical block indices of the minimum pass (blocks and brick padding)
long long imf_block_logical(int shape, int nx, int ny, int nz);

// sweep route: A = Omega_0 and (D^c dilated by S) with D^c = {g <= theta}
struct imf_sweep_args {
  const imf_orient_desc* desc; int nq;   // sruns hold the x-runs of S
  const float* g; long long g_stride; double theta;
  int nx, ny, nz; const uint8_t* omega0;
  uint64_t* dc; long long dc_stride;   // scratch bitset per q over the box
  uint64_t* masks;                     // indexed by each descriptor's out_q
};
hipError_t imf_launch_sweep(const imf_sweep_args& a, hipStream_t s);

// exact threshold decisions of density requests at lambda F_max (k_exact.hip)
struct imf_exact_args {
  const imf_orient_desc* desc;  // [2 nO]: processing order, then the same orientations
                                // with the x-runs of S as sruns
  int nO;
  int nx, ny, nz;
  long long N;
  const long long* ps; long long ps_stride;   // x prefix sums of rho_O, per fixture set
  const float* f; const uint8_t* omega0;
  const float* gamma;            // gamma stack [request orientation][N], or NULL
  const unsigned long long* keep; long long kstride;  // kept-block bits per orientation or NULL
  const long long* gbase; const int* koff;  // compact gamma stack (imf_min_args), or NULL
  int WX, WY, WZ;                // block shape of those bits
  const float* gst; long long gst_stride;   // g of every orientation (processing index), or NULL
  double E;                      // bound on |g32 - g| (voxel units)
  double scale;                  // voxel units per fixed-point unit (2^-24, or 1)
  double lambda;
  const unsigned int* fmax_bits; // float32 maximum of f over Omega_0 (order-preserving bits)
  unsigned long long* Fq;        // exact F_max in fixed-point units
  int* cand; unsigned int* cand_cnt; int cand_cap;    // candidate voxels of the maximum
  int4* band; unsigned int* band_cnt; int band_cap;   // band entries (q, box index, g bits, 0)
  unsigned int* err_bits;        // largest |g32 - g| seen by an exact recomputation (float bits)
  unsigned int* n_exact;         // exact recomputations
  uint64_t* masks;               // masks at lambda F_max, [request orientation][nz][ny][words]
  const unsigned int* skip_scan; // nonzero: the band list is already complete, or NULL
  // bracket lists of the inverse x pass (IMF_BR_SLICES per orientation), or NULL
  const int4* blist; const unsigned int* bcnt; int bslot;
  unsigned int* blisted;         // total entries the bracket lists hold
  const uint64_t* om_bits;       // Omega_0 as row bits [nz][ny][words] (the band's sweep)
};
// Omega_0 (one byte per voxel) packed into row words, bit x % 64 of word x / 64
hipError_t imf_launch_om_bits(const uint8_t* om, int nx, long long rows, uint64_t* out,
                              hipStream_t s);
// candidates of the maximum, their exact f (cmin: cand_cap words of scratch),
// and F_max = the largest of those
hipError_t imf_launch_exact_fmax(const imf_exact_args& a, unsigned long long* cmin,
                                 hipStream_t s);
hipError_t imf_launch_fq_from_fmax(const unsigned int* fmax_bits, double inv_scale,
                                   unsigned long long* Fq, hipStream_t s);
hipError_t imf_launch_band_scan(const imf_exact_args& a, long long max_vol, hipStream_t s);
// after the exact F_max: the listed bracket (blo, bhi] holds the band of lambda
// F_max (and did not overflow) -> *ok = 1; otherwise *ok = 0 and the list is
// emptied for the scan
hipError_t imf_launch_bracket_check(const imf_exact_args& a, double blo, double bhi,
                                    unsigned int* ok, hipStream_t s);
hipError_t imf_launch_band_exact(const imf_exact_args& a, hipStream_t s);
hipError_t imf_launch_finalize_exact(const imf_exact_args& a, const void* design, int density,
                                     double tau, double Efin, float* imf_out, float* imf_norm,
                                     uint8_t* secluded, hipStream_t s);

// finalize
hipError_t imf_launch_fill_f(float* f, long long n, float v, hipStream_t s);
hipError_t imf_launch_fill_u32(unsigned int* p, long long n, unsigned int v, hipStream_t s);
hipError_t imf_launch_omega0(const uint8_t* fixture, const uint8_t* domain, uint8_t* omega0,
                             long long n, hipStream_t s);
hipError_t imf_launch_or_u8(const uint8_t* a, const uint8_t* b, uint8_t* out, long long n,
                            hipStream_t s);
hipError_t imf_launch_fmax(const float* f, const uint8_t* omega0, long long n,
                           unsigned int* fmax_bits, hipStream_t s);
hipError_t imf_launch_masks_from_gamma(const float* gamma_stack, int nq, const uint8_t* omega0,
                                       int nx, int ny, int nz, const unsigned long long* Fq,
                                       double scale, double lambda, double E, uint64_t* masks,
                                       const unsigned long long* keep, int shape,
                                       long long kstride, const long long* gbase,
                                       const int* koff, hipStream_t s);

// coupling to the TO loop (Sec. 2.2)
hipError_t imf_launch_heaviside(const float* xi, long long n, double beta, float* rho,
                                hipStream_t s);
struct imf_couple_args {
  long long n;
  const void* design; int density;       // rho_Omega (uint8 {0,1} or float32)
  const uint8_t* fixture; const uint8_t* domain;  // Omega_0 as in a request
  const float* imf_norm; const uint8_t* secluded; double tau;
  float* filt;                           // out: Sbar_IMF
  const float* sens; double w; float* sens_out;   // optional: S_phi in, S out
  unsigned int* smax;                    // device scratch: max |S_phi| over Omega_0
};
hipError_t imf_launch_access_filter(const imf_couple_args& a, hipStream_t s);
// greedy machining plan (Sec. 3.4.1)
hipError_t imf_launch_negative_bits(const void* design, int density, double tau,
                                    const uint8_t* fixture, const uint8_t* domain, int nx,
                                    long long rows, uint64_t* R, hipStream_t s);
hipError_t imf_launch_cover_count(const uint64_t* masks, int nq, long long nw, const uint64_t* R,
                                  unsigned long long* counts, hipStream_t s);
hipError_t imf_launch_cover_remove(const uint64_t* A, long long nw, uint64_t* R, hipStream_t s);
hipError_t imf_launch_cover_best(const unsigned long long* counts, int nq, unsigned long long* out,
                                 hipStream_t s);
// fixed scratch of the allocation-free planner (64-bit words, per device)
#define IMF_PLAN_SCRATCH_WORDS (1 << 20)
#define IMF_MAX_DEVICES 64
// once per device, with that device current: take the device address of the
// scratch array (hipGetSymbolAddress); later calls return at once
hipError_t imf_plan_scratch_init(int device);
// that address, or NULL before imf_plan_scratch_init succeeded on the device
unsigned long long* imf_plan_scratch(int device);
