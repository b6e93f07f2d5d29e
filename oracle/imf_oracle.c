/*
 * imf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU oracle for the inaccessibility measure field (IMF) of
 * "Topology Optimization with Accessibility Constraint for Multi-Axis
 * Machining" (Mirzendehdel, Behandish, Nelaturi).  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never does.  It shares no code with the HIP library.
 *
 * Everything is exact integer arithmetic: binary designs count voxels, density
 * designs are fixed point with 24 fractional bits (every value k/2^24), so all
 * overlap sums are exact int64.  FP64 appears only in the rasterization
 * predicate and in the final normalization.
 *
 * Steps and where they come from:
 *   obstacle field   rho_O = max(rho_Omega, 1_F)       Sec. 2.1.5 (Eq. imf_4 and
 *                    the line defining rho_O); "implicit union" read as max.
 *   tool raster      T_R = raster(R(H u K)), S_R = raster(RK)   Sec. 2.1.5,
 *                    Rotate step of Algorithm 1; analytic rasterization at
 *                    voxel centres (the paper leaves the re-sampling open).
 *   overlap          g_R(t) = sum_{o in T_R} rho_O(t + o)      Eq. ident and
 *                    App. A Eq. conv_1 (vol[O n (R,t)T] as an inner product).
 *   sharp-point min  gamma_R(x) = min_{k in S_R} g_R(x - k)    Eq. imf_2.
 *   IMF              f(x) = min_tools min_R gamma_R(x)         Eqs. imf_3, imf_5.
 *   normalization    F_max = max_{x in Omega_0} f, fbar = f / F_max   Sec. 2.1.5.
 *   classification   B = Omega_0 and [f > lambda F_max], fbar <- fbar * 1_B,
 *                    Gamma = Omega_0 and not Omega and B        Algorithm 1, Eq. gamma.
 *   accessible mask  A_R = Omega_0 n {gamma_R <= theta}, and independently
 *                    A_R = Omega_0 n (D^c_R (+) S_R), D^c_R = {t : g_R(t) <= theta}
 *                                                              Eqs. sweep, A, conv_A.
 * Built with -ffp-contract=off so the FP64 predicate is evaluated exactly in
 * the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2

typedef struct {
  int kind; /* 0 flat end mill, 1 ball end mill, 2 2D rectangle, 3 voxel model */
  double cutter_r, cutter_len, holder_r, holder_len;
  /* voxel model (kind 3): labels [vdim z][y][x] in the tool frame, 0 empty,
   * 1 holder, 2 cutter; vorg = the tip voxel (tool-frame origin) */
  const uint8_t *vox;
  int vdim[3], vorg[3];
} or_tool;

typedef struct {
  int ndim, nx, ny, nz;
  int density; /* 0: uint8 {0,1}; 1: float32 on the 2^-24 grid */
  const void *design;
  const uint8_t *fixture; /* may be NULL */
  const uint8_t *domain;  /* may be NULL: Omega_0 = not fixture */
  int n_tools;
  const or_tool *tools;
  const int *n_dirs;
  int dir_kind; /* 0: float64 unit vectors, 1: int32 lattice vectors, 2: float64
                   rotation matrices (9 per orientation, row-major, tool frame to grid;
                   3D only; an axisymmetric tool uses the image of its +z axis) */
  const void *dirs;
  int sharp; /* 0 all cutter voxels, 1 boundary voxels, 2 tip voxel */
  double lambda, tau, mask_theta_abs;
  /* fixtures that change with the setup (Sec. 2.1.5: the fixture, hence O,
   * may differ per re-clamping, known beforehand): orientation R sees
   * F_R = fixture u fixture_sets[fixture_of[R]]; Omega_0 (without a domain)
   * excludes every fixture voxel of every setup */
  const uint8_t *fixture_sets; /* [n_fixture_sets][N], or NULL */
  int n_fixture_sets;
  const int *fixture_of;       /* [n_orient] */
} or_request;

typedef struct {
  double *imf;             /* [N] f in voxel-volume units, or NULL */
  float *imf_norm;         /* [N] fbar * 1_B, or NULL */
  uint8_t *secluded;       /* [N] Gamma, or NULL */
  uint64_t *masks;         /* [n_orient][nz][ny][words] threshold route, or NULL */
  uint64_t *masks_dil;     /* same, dilation route, or NULL */
  double *F_max;           /* scalar, or NULL */
  int64_t *g_debug;        /* overlap of one orientation over its query box */
  int debug_orient;
  int *debug_box;          /* lo[3], dims[3] of that box */
} or_outputs;

/* ------------------------------------------------------------------------ */
/* rasterization                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
  int ndim, lattice;
  double d[3];
  int64_t v[3], vn; /* lattice vector and |v|^2 */
  or_tool t;
  int64_t r2, L2, rh2, LH2; /* doubled parameters (lattice mode) */
  double R[9];              /* rotation (voxel tools), row-major */
} raster_ctx;

static int is_half_integer(double x) {
  double y = x * 2.0;
  return y == rint(y) && fabs(y) < 1e6;
}

static int raster_setup(raster_ctx *c, int ndim, const or_tool *t, int dir_kind,
                        const void *dirs, int index) {
  memset(c, 0, sizeof(*c));
  c->ndim = ndim;
  c->t = *t;
  if (t->kind < 0 || t->kind > 3) return OR_EINVAL;
  if (t->kind == 2 && ndim != 2) return OR_EINVAL;
  if (t->kind == 3) {
    if (ndim != 3 || dir_kind != 2 || !t->vox) return OR_EINVAL;
    for (int a = 0; a < 3; a++)
      if (t->vdim[a] < 1 || t->vorg[a] < 0 || t->vorg[a] >= t->vdim[a]) return OR_EINVAL;
  } else if (!(t->cutter_r > 0 && t->cutter_len > 0 && t->holder_r >= 0 &&
               t->holder_len >= 0)) {
    return OR_EINVAL;
  }
  if (dir_kind == 2) {
    /* rotation: orthonormal with determinant +1; d = image of the tool's +z */
    if (ndim != 3) return OR_EINVAL;
    const double *R = (const double *)dirs + (size_t)index * 9;
    for (int i = 0; i < 9; i++) c->R[i] = R[i];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        const double dot = R[3 * i] * R[3 * j] + R[3 * i + 1] * R[3 * j + 1] + R[3 * i + 2] * R[3 * j + 2];
        if (fabs(dot - (i == j ? 1.0 : 0.0)) > 1e-9) return OR_EINVAL;
      }
    const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                       R[2] * (R[3] * R[7] - R[4] * R[6]);
    if (det < 0) return OR_EINVAL;
    c->d[0] = R[2];
    c->d[1] = R[5];
    c->d[2] = R[8];
    return OR_OK;
  }
  if (dir_kind == 1) {
    const int32_t *iv = (const int32_t *)dirs + (size_t)index * ndim;
    c->lattice = 1;
    for (int a = 0; a < ndim; a++) c->v[a] = iv[a];
    c->vn = 0;
    for (int a = 0; a < ndim; a++) c->vn += c->v[a] * c->v[a];
    if (c->vn == 0) return OR_EINVAL;
    for (int a = 0; a < ndim; a++) c->d[a] = (double)c->v[a] / sqrt((double)c->vn);
    if (!is_half_integer(t->cutter_r) || !is_half_integer(t->cutter_len) ||
        !is_half_integer(t->holder_r) || !is_half_integer(t->holder_len))
      return OR_EINVAL;
    c->r2 = (int64_t)rint(2 * t->cutter_r);
    c->L2 = (int64_t)rint(2 * t->cutter_len);
    c->rh2 = (int64_t)rint(2 * t->holder_r);
    c->LH2 = (int64_t)rint(2 * (t->cutter_len + t->holder_len));
  } else {
    const double *dv = (const double *)dirs + (size_t)index * ndim;
    double n2 = 0;
    for (int a = 0; a < ndim; a++) {
      c->d[a] = dv[a];
      n2 += dv[a] * dv[a];
    }
    if (!(fabs(sqrt(n2) - 1.0) <= 1e-12)) return OR_EINVAL;
  }
  return OR_OK;
}

/* membership of integer offset o: returns bit0 = in tool T, bit1 = in cutter K */
static int raster_member(const raster_ctx *c, int64_t ox, int64_t oy, int64_t oz) {
  int cut = 0, hold = 0;
  if (c->t.kind == 3) {
    /* re-sampling: the tool-frame point R^T o, rounded to the nearest voxel
     * (halves to even), evaluated in this order */
    const double x = (double)ox, y = (double)oy, z = (double)oz;
    const double *R = c->R;
    int64_t idx[3];
    for (int a = 0; a < 3; a++) {
      const double u = (R[a] * x + R[3 + a] * y) + R[6 + a] * z;
      idx[a] = (int64_t)rint(u) + c->t.vorg[a];
      if (idx[a] < 0 || idx[a] >= c->t.vdim[a]) return 0;
    }
    const uint8_t lab =
        c->t.vox[(idx[2] * c->t.vdim[1] + idx[1]) * c->t.vdim[0] + idx[0]];
    cut = lab == 2;
    hold = lab == 1;
    return (cut || hold) | (cut << 1);
  }
  if (c->lattice) {
    int64_t dot, o2;
    if (c->ndim == 3) {
      dot = ox * c->v[0] + oy * c->v[1] + oz * c->v[2];
      o2 = ox * ox + oy * oy + oz * oz;
    } else {
      dot = ox * c->v[0] + oy * c->v[1];
      o2 = ox * ox + oy * oy;
    }
    const int64_t n = c->vn;
    const int64_t perp4 = 4 * (o2 * n - dot * dot); /* 4 q^2 |v|^2 */
    const int64_t dot4 = 4 * dot * dot;             /* 4 a^2 |v|^2 */
    const int in_r = perp4 <= c->r2 * c->r2 * n;
    const int a_ge0 = dot >= 0;
    const int a_ltL = a_ge0 && dot4 < c->L2 * c->L2 * n;
    if (c->t.kind == 1) {
      const int in_ball = a_ge0 && o2 * o2 * n <= c->r2 * c->r2 * dot * dot;
      const int a_ger = a_ge0 && dot4 >= c->r2 * c->r2 * n;
      cut = in_ball || (a_ger && a_ltL && in_r);
    } else {
      cut = a_ltL && in_r;
    }
    hold = a_ge0 && dot4 >= c->L2 * c->L2 * n && dot4 < c->LH2 * c->LH2 * n &&
           perp4 <= c->rh2 * c->rh2 * n;
  } else {
    const double dx = c->d[0], dy = c->d[1], dz = c->d[2];
    const double x = (double)ox, y = (double)oy, z = (double)oz;
    double a, q2;
    if (c->ndim == 3) {
      a = (x * dx + y * dy) + z * dz;
      const double px = x - a * dx, py = y - a * dy, pz = z - a * dz;
      q2 = (px * px + py * py) + pz * pz;
    } else {
      a = x * dx + y * dy;
      const double px = x - a * dx, py = y - a * dy;
      q2 = px * px + py * py;
    }
    const double r = c->t.cutter_r, L = c->t.cutter_len;
    const double rh = c->t.holder_r, LH = c->t.cutter_len + c->t.holder_len;
    const int in_cyl = a < L && q2 <= r * r;
    if (c->t.kind == 1) {
      double b2;
      const double bx = x - r * dx, by = y - r * dy;
      if (c->ndim == 3) {
        const double bz = z - r * dz;
        b2 = (bx * bx + by * by) + bz * bz;
      } else {
        b2 = bx * bx + by * by;
      }
      cut = b2 <= r * r || (a >= r && in_cyl);
    } else {
      cut = a >= 0 && in_cyl;
    }
    hold = a >= L && a < LH && q2 <= rh * rh;
  }
  return (cut || hold) | (cut << 1);
}

static void raster_bbox(const raster_ctx *c, int lo[3], int hi[3]) {
  if (c->t.kind == 3) {
    /* image of the label box (widened by half a voxel) under R, plus one */
    for (int a = 0; a < 3; a++) {
      double mn = 1e300, mx = -1e300;
      for (int k = 0; k < 8; k++) {
        double p = 0;
        for (int b = 0; b < 3; b++) {
          const double e = (k >> b) & 1 ? (double)(c->t.vdim[b] - 1 - c->t.vorg[b]) + 0.5
                                        : -(double)c->t.vorg[b] - 0.5;
          p += c->R[3 * a + b] * e;
        }
        if (p < mn) mn = p;
        if (p > mx) mx = p;
      }
      lo[a] = (int)floor(mn) - 1;
      hi[a] = (int)ceil(mx) + 1;
    }
    return;
  }
  double len = c->t.cutter_len + c->t.holder_len;
  if (2 * c->t.cutter_r > len) len = 2 * c->t.cutter_r;
  const double rmax = c->t.cutter_r > c->t.holder_r ? c->t.cutter_r : c->t.holder_r;
  for (int a = 0; a < 3; a++) {
    if (a >= c->ndim) {
      lo[a] = hi[a] = 0;
      continue;
    }
    const double e = len * c->d[a];
    lo[a] = (int)floor((e < 0 ? e : 0) - rmax) - 1;
    hi[a] = (int)ceil((e > 0 ? e : 0) + rmax) + 1;
  }
}

/* Enumerate the raster of one oriented tool in z, y, x order.  offs receives
 * (x, y, z) triples, is_cutter a 0/1 flag per offset.  Returns the count, or
 * -1 on invalid input, or -(needed) - 2 when cap is too small. */
long long or_raster(int ndim, const or_tool *t, int dir_kind, const void *dirs, int index,
                    int32_t *offs, uint8_t *is_cutter, long long cap) {
  raster_ctx c;
  if (raster_setup(&c, ndim, t, dir_kind, dirs, index) != OR_OK) return -1;
  int lo[3], hi[3];
  raster_bbox(&c, lo, hi);
  long long n = 0;
  for (int z = lo[2]; z <= hi[2]; z++)
    for (int y = lo[1]; y <= hi[1]; y++)
      for (int x = lo[0]; x <= hi[0]; x++) {
        const int m = raster_member(&c, x, y, z);
        if (!(m & 1)) continue;
        if (n < cap) {
          if (offs) {
            offs[3 * n] = x;
            offs[3 * n + 1] = y;
            offs[3 * n + 2] = z;
          }
          if (is_cutter) is_cutter[n] = (uint8_t)(m >> 1);
        }
        n++;
      }
  if (n > cap) return -n - 2;
  return n;
}

/* ------------------------------------------------------------------------ */
/* one oriented tool as offset lists                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t *T; /* tool offsets, xyz triples */
  long long nT;
  int32_t *S; /* sharp points in use, xyz triples */
  long long nS;
  int kmin[3], kmax[3]; /* extent of S */
} oriented_tool;

static void otool_free(oriented_tool *o) {
  free(o->T);
  free(o->S);
  memset(o, 0, sizeof(*o));
}

static int otool_build(oriented_tool *o, int ndim, const or_tool *t, int dir_kind,
                       const void *dirs, int index, int sharp) {
  memset(o, 0, sizeof(*o));
  raster_ctx c;
  if (raster_setup(&c, ndim, t, dir_kind, dirs, index) != OR_OK) return OR_EINVAL;
  long long n = or_raster(ndim, t, dir_kind, dirs, index, NULL, NULL, 0);
  if (n >= 0) return OR_EINVAL;
  n = -n - 2;
  o->T = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(n + 1));
  uint8_t *cut = (uint8_t *)malloc((size_t)n + 1);
  o->S = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(n + 1));
  if (!o->T || !cut || !o->S) {
    free(cut);
    otool_free(o);
    return OR_ENOMEM;
  }
  o->nT = or_raster(ndim, t, dir_kind, dirs, index, o->T, cut, n);
  o->nS = 0;
  if (sharp == 2) {
    /* the tip alone: the origin, which a ball cutter's raster may miss by
     * rounding because it lies exactly on the sphere */
    o->S[0] = o->S[1] = o->S[2] = 0;
    o->nS = 1;
  }
  for (long long i = 0; i < o->nT && sharp != 2; i++) {
    if (!cut[i]) continue;
    const int x = o->T[3 * i], y = o->T[3 * i + 1], z = o->T[3 * i + 2];
    int keep = 1;
    if (sharp == 1) {
      /* boundary voxel of the cutter raster: some axis neighbour is not cutter */
      keep = 0;
      for (int a = 0; a < ndim && !keep; a++)
        for (int s = -1; s <= 1; s += 2) {
          int64_t p[3] = {x, y, z};
          p[a] += s;
          if (!(raster_member(&c, p[0], p[1], p[2]) & 2)) keep = 1;
        }
    }
    if (!keep) continue;
    o->S[3 * o->nS] = x;
    o->S[3 * o->nS + 1] = y;
    o->S[3 * o->nS + 2] = z;
    o->nS++;
  }
  free(cut);
  if (o->nS == 0) {
    otool_free(o);
    return OR_EINVAL;
  }
  for (int a = 0; a < 3; a++) {
    o->kmin[a] = o->S[a];
    o->kmax[a] = o->S[a];
  }
  for (long long i = 0; i < o->nS; i++)
    for (int a = 0; a < 3; a++) {
      if (o->S[3 * i + a] < o->kmin[a]) o->kmin[a] = o->S[3 * i + a];
      if (o->S[3 * i + a] > o->kmax[a]) o->kmax[a] = o->S[3 * i + a];
    }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* fields                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nx, ny, nz;
  long long N;
  int64_t scale; /* 1 for binary, 2^24 for density */
  int64_t *rhoO; /* obstacle field of the current orientation, fixed point */
  int64_t *rhoD; /* design field in fixed point */
  uint8_t *omega0;
  int64_t *rhoO_base; /* with the common fixture only */
  int64_t **rhoO_sets; /* per fixture set, or NULL */
  int nsets;
} fields;

static void fields_free(fields *F) {
  free(F->rhoO_base);
  for (int s = 0; s < F->nsets; s++) free(F->rhoO_sets[s]);
  free(F->rhoO_sets);
  free(F->rhoD);
  free(F->omega0);
  memset(F, 0, sizeof(*F));
}

/* the obstacle field rho_O seen by orientation `orient` */
static void fields_select(fields *F, const or_request *q, int orient) {
  F->rhoO = F->nsets ? F->rhoO_sets[q->fixture_of[orient]] : F->rhoO_base;
}

static int count_orient_req(const or_request *q) {
  int n = 0;
  for (int i = 0; i < q->n_tools; i++) n += q->n_dirs[i];
  return n;
}

static int fields_build(fields *F, const or_request *q) {
  memset(F, 0, sizeof(*F));
  if (q->ndim != 2 && q->ndim != 3) return OR_EINVAL;
  if (q->nx <= 0 || q->ny <= 0 || q->nz <= 0) return OR_EINVAL;
  if (q->ndim == 2 && q->nz != 1) return OR_EINVAL;
  F->nx = q->nx;
  F->ny = q->ny;
  F->nz = q->nz;
  F->N = (long long)q->nx * q->ny * q->nz;
  F->scale = q->density ? ((int64_t)1 << 24) : 1;
  F->rhoO_base = (int64_t *)malloc(sizeof(int64_t) * (size_t)F->N);
  F->rhoO = F->rhoO_base;
  F->rhoD = (int64_t *)malloc(sizeof(int64_t) * (size_t)F->N);
  F->omega0 = (uint8_t *)malloc((size_t)F->N);
  if (!F->rhoO_base || !F->rhoD || !F->omega0) {
    fields_free(F);
    return OR_ENOMEM;
  }
  for (long long i = 0; i < F->N; i++) {
    int64_t v;
    if (q->density) {
      const double r = (double)((const float *)q->design)[i];
      const double s = r * 16777216.0;
      if (!(r >= 0.0 && r <= 1.0) || s != floor(s)) {
        fields_free(F);
        return OR_EINVAL;
      }
      v = (int64_t)s;
    } else {
      const uint8_t b = ((const uint8_t *)q->design)[i];
      if (b > 1) {
        fields_free(F);
        return OR_EINVAL;
      }
      v = b;
    }
    F->rhoD[i] = v;
    const int fix = q->fixture ? (q->fixture[i] != 0) : 0;
    F->rhoO_base[i] = fix ? F->scale : v; /* max(rho_Omega, 1_F) */
    F->omega0[i] = q->domain ? (q->domain[i] != 0) : (uint8_t)!fix;
  }
  if (q->n_fixture_sets > 0) {
    if (!q->fixture_sets || !q->fixture_of) {
      fields_free(F);
      return OR_EINVAL;
    }
    F->nsets = q->n_fixture_sets;
    F->rhoO_sets = (int64_t **)calloc((size_t)F->nsets, sizeof(int64_t *));
    if (!F->rhoO_sets) {
      fields_free(F);
      return OR_ENOMEM;
    }
    for (int s = 0; s < F->nsets; s++) {
      F->rhoO_sets[s] = (int64_t *)malloc(sizeof(int64_t) * (size_t)F->N);
      if (!F->rhoO_sets[s]) {
        fields_free(F);
        return OR_ENOMEM;
      }
      const uint8_t *fs = q->fixture_sets + (size_t)s * F->N;
      for (long long i = 0; i < F->N; i++) {
        F->rhoO_sets[s][i] = fs[i] ? F->scale : F->rhoO_base[i];
        if (fs[i] && !q->domain) F->omega0[i] = 0;
      }
    }
    const int nO = count_orient_req(q);
    for (int r = 0; r < nO; r++)
      if (q->fixture_of[r] < 0 || q->fixture_of[r] >= F->nsets) {
        fields_free(F);
        return OR_EINVAL;
      }
  }
  return OR_OK;
}

static inline int64_t field_at(const fields *F, long long x, long long y, long long z) {
  if (x < 0 || y < 0 || z < 0 || x >= F->nx || y >= F->ny || z >= F->nz) return 0;
  return F->rhoO[(z * F->ny + y) * F->nx + x];
}

/* g(t) = sum over tool offsets o of rho_O(t + o)  (Eq. ident) */
static int64_t overlap_at(const fields *F, const oriented_tool *o, long long tx, long long ty,
                          long long tz) {
  int64_t s = 0;
  for (long long i = 0; i < o->nT; i++)
    s += field_at(F, tx + o->T[3 * i], ty + o->T[3 * i + 1], tz + o->T[3 * i + 2]);
  return s;
}

static int count_orient(const or_request *q) {
  int n = 0;
  for (int i = 0; i < q->n_tools; i++) n += q->n_dirs[i];
  return n;
}

/* map a global orientation index to (tool, index into the dirs array) */
static int orient_lookup(const or_request *q, int orient, int *tool) {
  int base = 0;
  for (int i = 0; i < q->n_tools; i++) {
    if (orient < base + q->n_dirs[i]) {
      *tool = i;
      return orient;
    }
    base += q->n_dirs[i];
  }
  return -1;
}

static int build_orient(const or_request *q, int orient, oriented_tool *o) {
  int ti;
  if (orient_lookup(q, orient, &ti) < 0) return OR_EINVAL;
  return otool_build(o, q->ndim, &q->tools[ti], q->dir_kind, q->dirs, orient, q->sharp);
}

/* ------------------------------------------------------------------------ */
/* full IMF (Algorithm 1)                                                    */
/* ------------------------------------------------------------------------ */

int or_imf(const or_request *q, const or_outputs *out) {
  if (!q || !out || q->n_tools < 1 || !q->tools || !q->n_dirs || !q->dirs) return OR_EINVAL;
  const int nO = count_orient(q);
  if (nO < 1) return OR_EINVAL;
  fields F;
  int st = fields_build(&F, q);
  if (st) return st;
  const long long N = F.N;
  const int nx = F.nx, ny = F.ny, nz = F.nz;
  const int words = (nx + 63) / 64;
  int64_t *f = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  int64_t *gam = (int64_t *)malloc(sizeof(int64_t) * (size_t)N * nO);
  if (!f || !gam) {
    free(f);
    free(gam);
    fields_free(&F);
    return OR_ENOMEM;
  }
  for (long long i = 0; i < N; i++) f[i] = INT64_MAX; /* +infinity before the first min */

  for (int r = 0; r < nO && st == OR_OK; r++) {
    oriented_tool o;
    fields_select(&F, q, r);
    st = build_orient(q, r, &o);
    if (st) break;
    /* query box of translations: t = x - k, x in grid, k in S_R */
    long long lo[3], dim[3];
    const int n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; a++) {
      lo[a] = -(long long)o.kmax[a];
      dim[a] = n[a] + o.kmax[a] - o.kmin[a];
    }
    const long long M = dim[0] * dim[1] * dim[2];
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    if (!g) {
      otool_free(&o);
      st = OR_ENOMEM;
      break;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (long long tz = 0; tz < dim[2]; tz++)
      for (long long ty = 0; ty < dim[1]; ty++)
        for (long long tx = 0; tx < dim[0]; tx++)
          g[(tz * dim[1] + ty) * dim[0] + tx] =
              overlap_at(&F, &o, tx + lo[0], ty + lo[1], tz + lo[2]);
    if (out->g_debug && out->debug_orient == r) {
      memcpy(out->g_debug, g, sizeof(int64_t) * (size_t)M);
      if (out->debug_box)
        for (int a = 0; a < 3; a++) {
          out->debug_box[a] = (int)lo[a];
          out->debug_box[3 + a] = (int)dim[a];
        }
    }
    int64_t *gr = gam + (size_t)r * N;
    /* gamma_R(x) = min over sharp points k of g(x - k)  (Eq. imf_2) */
#pragma omp parallel for schedule(dynamic, 1)
    for (long long z = 0; z < nz; z++)
      for (long long y = 0; y < ny; y++)
        for (long long x = 0; x < nx; x++) {
          int64_t m = INT64_MAX;
          for (long long i = 0; i < o.nS; i++) {
            const long long tx = x - o.S[3 * i] - lo[0];
            const long long ty = y - o.S[3 * i + 1] - lo[1];
            const long long tz = z - o.S[3 * i + 2] - lo[2];
            const int64_t v = g[(tz * dim[1] + ty) * dim[0] + tx];
            if (v < m) m = v;
          }
          const long long xi = (z * ny + y) * nx + x;
          gr[xi] = m;
          if (m < f[xi]) f[xi] = m;
        }
    free(g);
    otool_free(&o);
  }
  if (st) {
    free(f);
    free(gam);
    fields_free(&F);
    return st;
  }

  /* F_max over the design domain Omega_0 */
  int64_t fmax = 0;
  for (long long i = 0; i < N; i++)
    if (F.omega0[i] && f[i] > fmax) fmax = f[i];
  const double fmax_d = (double)fmax;
  const double scale = (double)F.scale;
  const double thB = q->lambda * fmax_d; /* B: f > lambda * F_max */
  const double theta = q->mask_theta_abs >= 0 ? q->mask_theta_abs * scale : thB;
  if (out->F_max) *out->F_max = fmax_d / scale;
  for (long long i = 0; i < N; i++) {
    const int inB = F.omega0[i] && (double)f[i] > thB;
    if (out->imf) out->imf[i] = (double)f[i] / scale;
    if (out->imf_norm) out->imf_norm[i] = inB ? (float)((double)f[i] / fmax_d) : 0.0f;
    if (out->secluded) {
      const int solid = (double)F.rhoD[i] > q->tau * scale;
      out->secluded[i] = (uint8_t)(inB && !solid);
    }
  }

  /* accessible masks, route 1: threshold of gamma_R */
  if (out->masks) {
    memset(out->masks, 0, sizeof(uint64_t) * (size_t)nO * nz * ny * words);
    for (int r = 0; r < nO; r++) {
      const int64_t *gr = gam + (size_t)r * N;
      for (long long z = 0; z < nz; z++)
        for (long long y = 0; y < ny; y++)
          for (long long x = 0; x < nx; x++) {
            const long long xi = (z * ny + y) * nx + x;
            if (F.omega0[xi] && (double)gr[xi] <= theta)
              out->masks[(((size_t)r * nz + z) * ny + y) * words + x / 64] |=
                  (uint64_t)1 << (x % 64);
          }
    }
  }

  /* accessible masks, route 2: sweep the free translations by the cutter */
  if (out->masks_dil) {
    memset(out->masks_dil, 0, sizeof(uint64_t) * (size_t)nO * nz * ny * words);
    for (int r = 0; r < nO && st == OR_OK; r++) {
      oriented_tool o;
      fields_select(&F, q, r);
      st = build_orient(q, r, &o);
      if (st) break;
      long long lo[3], dim[3];
      const int n[3] = {nx, ny, nz};
      for (int a = 0; a < 3; a++) {
        lo[a] = -(long long)o.kmax[a];
        dim[a] = n[a] + o.kmax[a] - o.kmin[a];
      }
      const long long M = dim[0] * dim[1] * dim[2];
      uint8_t *freeset = (uint8_t *)malloc((size_t)M);
      if (!freeset) {
        otool_free(&o);
        st = OR_ENOMEM;
        break;
      }
#pragma omp parallel for schedule(dynamic, 1)
      for (long long tz = 0; tz < dim[2]; tz++)
        for (long long ty = 0; ty < dim[1]; ty++)
          for (long long tx = 0; tx < dim[0]; tx++)
            freeset[(tz * dim[1] + ty) * dim[0] + tx] =
                (double)overlap_at(&F, &o, tx + lo[0], ty + lo[1], tz + lo[2]) <= theta;
      /* x is swept iff x = t + k for a free t and a sharp point k */
      for (long long tz = 0; tz < dim[2]; tz++)
        for (long long ty = 0; ty < dim[1]; ty++)
          for (long long tx = 0; tx < dim[0]; tx++) {
            if (!freeset[(tz * dim[1] + ty) * dim[0] + tx]) continue;
            for (long long i = 0; i < o.nS; i++) {
              const long long x = tx + lo[0] + o.S[3 * i];
              const long long y = ty + lo[1] + o.S[3 * i + 1];
              const long long z = tz + lo[2] + o.S[3 * i + 2];
              if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) continue;
              if (!F.omega0[(z * ny + y) * nx + x]) continue;
              out->masks_dil[(((size_t)r * nz + z) * ny + y) * words + x / 64] |=
                  (uint64_t)1 << (x % 64);
            }
          }
      free(freeset);
      otool_free(&o);
    }
  }
  free(f);
  free(gam);
  fields_free(&F);
  return st;
}

/* ------------------------------------------------------------------------ */
/* sampled evaluation (for grids too large for the full oracle)              */
/* ------------------------------------------------------------------------ */

/* g_R(t) for n translations t (xyz triples), fixed point units */
int or_overlap_at(const or_request *q, int orient, const int32_t *t, long long n, int64_t *out) {
  fields F;
  int st = fields_build(&F, q);
  if (st) return st;
  oriented_tool o;
  fields_select(&F, q, orient);
  st = build_orient(q, orient, &o);
  if (st) {
    fields_free(&F);
    return st;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (long long i = 0; i < n; i++)
    out[i] = overlap_at(&F, &o, t[3 * i], t[3 * i + 1], t[3 * i + 2]);
  otool_free(&o);
  fields_free(&F);
  return OR_OK;
}

/* gamma_R(x) for n voxels x (xyz triples), fixed point units */
int or_gamma_at(const or_request *q, int orient, const int32_t *xs, long long n, int64_t *out) {
  fields F;
  int st = fields_build(&F, q);
  if (st) return st;
  oriented_tool o;
  fields_select(&F, q, orient);
  st = build_orient(q, orient, &o);
  if (st) {
    fields_free(&F);
    return st;
  }
  for (long long j = 0; j < n; j++) {
    int64_t m = INT64_MAX;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : m)
    for (long long i = 0; i < o.nS; i++) {
      const int64_t v = overlap_at(&F, &o, xs[3 * j] - o.S[3 * i], xs[3 * j + 1] - o.S[3 * i + 1],
                                   xs[3 * j + 2] - o.S[3 * i + 2]);
      if (v < m) m = v;
    }
    out[j] = m;
  }
  otool_free(&o);
  fields_free(&F);
  return OR_OK;
}

/* gamma_R(x) for n voxels x and every orientation R of the request:
 * out[R * n + j], fixed point units (the same sums as or_gamma_at, with the
 * obstacle field built once) */
int or_gamma_at_all(const or_request *q, const int32_t *xs, long long n, int64_t *out) {
  fields F;
  int st = fields_build(&F, q);
  if (st) return st;
  const int nO = count_orient(q);
  for (int r = 0; r < nO; r++) {
    oriented_tool o;
    fields_select(&F, q, r);
    st = build_orient(q, r, &o);
    if (st) {
      fields_free(&F);
      return st;
    }
    for (long long j = 0; j < n; j++) {
      int64_t m = INT64_MAX;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : m)
      for (long long i = 0; i < o.nS; i++) {
        const int64_t v = overlap_at(&F, &o, xs[3 * j] - o.S[3 * i], xs[3 * j + 1] - o.S[3 * i + 1],
                                     xs[3 * j + 2] - o.S[3 * i + 2]);
        if (v < m) m = v;
      }
      out[(long long)r * n + j] = m;
    }
    otool_free(&o);
  }
  fields_free(&F);
  return OR_OK;
}

/* Overlap of one orientation over the whole translation range where it can be
 * nonzero: t in [-o_max, n - 1 - o_min] per axis.  box receives lo[3], dims[3].
 * Call with out == NULL to get the box only. */
int or_overlap_full(const or_request *q, int orient, int64_t *out, int *box) {
  fields F;
  int st = fields_build(&F, q);
  if (st) return st;
  oriented_tool o;
  fields_select(&F, q, orient);
  st = build_orient(q, orient, &o);
  if (st) {
    fields_free(&F);
    return st;
  }
  int omin[3], omax[3];
  for (int a = 0; a < 3; a++) omin[a] = omax[a] = o.T[a];
  for (long long i = 0; i < o.nT; i++)
    for (int a = 0; a < 3; a++) {
      if (o.T[3 * i + a] < omin[a]) omin[a] = o.T[3 * i + a];
      if (o.T[3 * i + a] > omax[a]) omax[a] = o.T[3 * i + a];
    }
  const int n[3] = {F.nx, F.ny, F.nz};
  long long lo[3], dim[3];
  for (int a = 0; a < 3; a++) {
    lo[a] = -(long long)omax[a];
    dim[a] = n[a] + omax[a] - omin[a];
    box[a] = (int)lo[a];
    box[3 + a] = (int)dim[a];
  }
  if (out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (long long tz = 0; tz < dim[2]; tz++)
      for (long long ty = 0; ty < dim[1]; ty++)
        for (long long tx = 0; tx < dim[0]; tx++)
          out[(tz * dim[1] + ty) * dim[0] + tx] =
              overlap_at(&F, &o, tx + lo[0], ty + lo[1], tz + lo[2]);
  }
  otool_free(&o);
  fields_free(&F);
  return OR_OK;
}

/* sharp-point extent of one orientation: kmin[3], kmax[3], and |T|, |S| */
int or_orient_info(const or_request *q, int orient, int *kminmax, long long *counts) {
  oriented_tool o;
  int st = build_orient(q, orient, &o);
  if (st) return st;
  for (int a = 0; a < 3; a++) {
    kminmax[a] = o.kmin[a];
    kminmax[3 + a] = o.kmax[a];
  }
  counts[0] = o.nT;
  counts[1] = o.nS;
  otool_free(&o);
  return OR_OK;
}
