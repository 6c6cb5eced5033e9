/*
 * Plain CPU FP64 oracle for Gaussian-based volume ray marching (RayGaussX,
 * arXiv 2509.07782).  TEST INFRASTRUCTURE ONLY: it exists to check the GPU
 * library and is never part of the product path.  It shares no code with the
 * GPU path.
 *
 * Everything here is the definition written out, slowly and in double
 * precision, with no acceleration structure: every ray is tested against every
 * Gaussian.
 *
 *  - Density / radiance field: Sec. 3.1, Eq. 1.  Truncated unnormalised
 *    Gaussians: sigma~ * exp(-q/2), q = (x-mu)^T Sigma^-1 (x-mu),
 *    Sigma = R S S^T R^T, contributing only inside the sigma_eps level-set
 *    ellipsoid q <= k^2, k^2 = 2 ln(sigma~/sigma_eps) (Supp. B, ellipsoid
 *    definition).  Radiance is the density-weighted mean of the per-Gaussian
 *    SH colours c_l(d) at the ray direction.
 *  - Discrete ray marching: Sec. 3.1, Eq. 3.
 *  - Segment loop with closest-hit empty-space skipping: Sec. 3.2, Alg. 1
 *    and Eq. 4.  Adaptive segment size: Sec. 3.2, Eq. 5.
 *  - Backward: reverse-mode derivative of the above with the sample schedule
 *    and the truncation boundary held fixed.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *  - samples sit at segment midpoints t = a + (k + 1/2) dt;
 *  - a sample counts Gaussian l iff q_l(t) <= k_l^2 (truncation per sample);
 *  - a Gaussian belongs to a segment [a,b] iff its ellipsoid interval
 *    [t_in,t_out] meets [a,b] (closed intervals; containment counts);
 *  - termination (T > T_eps) is tested at segment starts only;
 *  - ess = 1 snaps the restart point to the fixed segment grid
 *    a = t_n + i * dS (fixed step only), ess = 2 restarts at the closest hit;
 *  - samples with t >= t_f are dropped;
 *  - a sample with sigma = 0 leaves colour and transmittance unchanged.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int64_t n;
  int32_t sh_degree;
  const double *means;      /* [n,3] */
  const double *log_scales; /* [n,3] */
  const double *quats;      /* [n,4] (w,x,y,z), unnormalised */
  const double *density;    /* [n]   raw sigma~ */
  const double *sh;         /* [n,K,3] */
  int32_t n_sg;             /* spherical-Gaussian lobes per Gaussian (0 = SH colour only) */
  const double *sg;         /* [n, n_sg, 7]: amplitude rgb, axis xyz (any norm > 0), sharpness */
} orc_scene;

typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
  double c2w[12]; /* 3x4 row-major: columns right, down, forward, centre */
  double t_near, t_far;
} orc_camera;

typedef struct {
  int32_t adaptive;
  double dt, dt_min, dt_max, beta;
  int32_t n_s;
  double t_eps;
  int32_t ess; /* 0 off, 1 snapped to the segment grid, 2 restart at closest hit */
  double bg[3];
  double sigma_eps;
} orc_opts;

/* per-ray statistics written by orc_render */
enum { ST_Q = 0, ST_P, ST_SAMPLES, ST_SEGMENTS, ST_CLOSEST, ST_NSTAT };

/* ------------------------------------------------------------------------ */
/* Per-Gaussian quantities (Eq. 1; Supp. B).                                 */

typedef struct {
  double mu[3], s[3], qhat[4], qnorm, R[9], M[9], k2, sig;
  int active;
} gauss;

/* Rotation matrix of a unit quaternion (w,x,y,z): the standard formula
   v -> q v q*, written out. */
static void quat_to_rot(const double q[4], double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void make_gauss(const orc_scene *sc, double sigma_eps, int64_t l, gauss *g) {
  const double *q = sc->quats + 4 * l;
  int finite = 1;
  for (int i = 0; i < 3; i++) {
    g->mu[i] = sc->means[3 * l + i];
    g->s[i] = exp(sc->log_scales[3 * l + i]);
    finite &= isfinite(g->mu[i]) && isfinite(sc->log_scales[3 * l + i]);
  }
  g->sig = sc->density[l];
  finite &= isfinite(g->sig);
  double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  finite &= isfinite(qn);
  g->qnorm = qn;
  g->active = finite && qn > 0 && g->sig > sigma_eps && g->s[0] > 0 && g->s[1] > 0 && g->s[2] > 0;
  if (!g->active) return;
  for (int i = 0; i < 4; i++) g->qhat[i] = q[i] / qn;
  quat_to_rot(g->qhat, g->R);
  /* M = S^-1 R^T, so that z = M (x - mu) has |z|^2 = q */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) g->M[3 * i + j] = g->R[3 * j + i] / g->s[i];
  g->k2 = 2.0 * log(g->sig / sigma_eps);
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics from the associated Legendre functions
   P_l^m (Condon-Shortley phase included), polar axis +z:
     m = 0 : K_l^0 P_l^0(cos th)
     m > 0 : sqrt2 K_l^m cos(m ph) P_l^m(cos th)
     m < 0 : sqrt2 K_l^|m| sin(|m| ph) P_l^|m|(cos th)
   K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), basis index l^2 + l + m. */

static double fact(int n) { double r = 1; for (int i = 2; i <= n; i++) r *= i; return r; }

static double assoc_legendre(int l, int m, double x) {
  /* P_m^m = (-1)^m (2m-1)!! (1-x^2)^(m/2), then the three-term recurrence in l */
  double pmm = 1.0, somx2 = sqrt(fmax(0.0, (1 - x) * (1 + x)));
  for (int i = 1; i <= m; i++) pmm *= -(2.0 * i - 1.0) * somx2;
  if (l == m) return pmm;
  double pmmp1 = x * (2.0 * m + 1.0) * pmm;
  if (l == m + 1) return pmmp1;
  double pll = 0;
  for (int ll = m + 2; ll <= l; ll++) {
    pll = ((2.0 * ll - 1.0) * x * pmmp1 - (ll + m - 1.0) * pmm) / (ll - m);
    pmm = pmmp1;
    pmmp1 = pll;
  }
  return pll;
}

void orc_sh_basis(int32_t deg, const double d[3], double *Y) {
  double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double ct = d[2] / r, ph = atan2(d[1], d[0]);
  for (int l = 0; l <= deg; l++) {
    for (int m = -l; m <= l; m++) {
      int am = m < 0 ? -m : m;
      double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * fact(l - am) / fact(l + am));
      double P = assoc_legendre(l, am, ct);
      double v;
      if (m == 0) v = K * P;
      else if (m > 0) v = sqrt(2.0) * K * cos(m * ph) * P;
      else v = sqrt(2.0) * K * sin(am * ph) * P;
      Y[l * l + l + m] = v;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Rays: pinhole through the pixel centre, unit direction (so t is metric).  */

/* Colour of Gaussian l at the unit direction d: the SH sum (Eq. 1's c_l(d))
   plus, when the scene has spherical-Gaussian lobes (the 9 SH + 7 SG
   appearance model of the supplement's comparison), the lobes
   a_j exp(lambda_j (xi_j.d / |xi_j| - 1)).  Used as is (no offset or clamp).
   A lobe with a zero axis contributes nothing. */
static void gaussian_colour(const orc_scene *sc, int K, int64_t l, const double *Y, const double d[3],
                            double col[3]) {
  for (int ch = 0; ch < 3; ch++) {
    double c = 0;
    for (int m = 0; m < K; m++) c += sc->sh[(l * K + m) * 3 + ch] * Y[m];
    col[ch] = c;
  }
  for (int j = 0; j < sc->n_sg; j++) {
    const double *p = sc->sg + (l * sc->n_sg + j) * 7;
    const double xn = sqrt(p[3] * p[3] + p[4] * p[4] + p[5] * p[5]);
    if (!(xn > 0)) continue;
    const double cosang = (p[3] * d[0] + p[4] * d[1] + p[5] * d[2]) / xn;
    const double g = exp(p[6] * (cosang - 1.0));
    for (int ch = 0; ch < 3; ch++) col[ch] += p[ch] * g;
  }
}

/* Adds dL/d(lobe parameters of Gaussian l) for dL/dc = dc[3] at direction d:
   da_j = g_j dc, dlambda_j = (a_j.dc) g_j (cos_j - 1), and through the unit
   axis u_j = xi_j / |xi_j|: dxi_j = (a_j.dc) g_j lambda_j (d - cos_j u_j) / |xi_j|. */
static void sg_backward(const orc_scene *sc, int64_t l, const double d[3], const double dc[3],
                        double *g_sg) {
  for (int j = 0; j < sc->n_sg; j++) {
    const double *p = sc->sg + (l * sc->n_sg + j) * 7;
    double *gp = g_sg + (l * sc->n_sg + j) * 7;
    const double xn = sqrt(p[3] * p[3] + p[4] * p[4] + p[5] * p[5]);
    if (!(xn > 0)) continue;
    const double u[3] = {p[3] / xn, p[4] / xn, p[5] / xn};
    const double cosang = u[0] * d[0] + u[1] * d[1] + u[2] * d[2];
    const double g = exp(p[6] * (cosang - 1.0));
    const double ad = p[0] * dc[0] + p[1] * dc[1] + p[2] * dc[2];
    double add[7];
    for (int ch = 0; ch < 3; ch++) add[ch] = g * dc[ch];
    for (int i = 0; i < 3; i++) add[3 + i] = ad * g * p[6] * (d[i] - cosang * u[i]) / xn;
    add[6] = ad * g * (cosang - 1.0);
    for (int i = 0; i < 7; i++) {
#pragma omp atomic
      gp[i] += add[i];
    }
  }
}

static void make_ray(const orc_camera *c, int64_t pix, double o[3], double d[3]) {
  int64_t u = pix % c->width, v = pix / c->width;
  double dc[3] = {((double)u + 0.5 - c->cx) / c->fx, ((double)v + 0.5 - c->cy) / c->fy, 1.0};
  double n = 0;
  for (int i = 0; i < 3; i++) {
    o[i] = c->c2w[4 * i + 3];
    d[i] = c->c2w[4 * i + 0] * dc[0] + c->c2w[4 * i + 1] * dc[1] + c->c2w[4 * i + 2] * dc[2];
    n += d[i] * d[i];
  }
  n = sqrt(n);
  for (int i = 0; i < 3; i++) d[i] /= n;
}

void orc_rays(const orc_camera *c, const int64_t *pix, int64_t n, double *o, double *d) {
  for (int64_t r = 0; r < n; r++) make_ray(c, pix[r], o + 3 * r, d + 3 * r);
}

/* q(x) = |M (x - mu)|^2, the plain definition */
static double qform(const gauss *g, const double x[3], double z[3]) {
  double e[3] = {x[0] - g->mu[0], x[1] - g->mu[1], x[2] - g->mu[2]};
  double q = 0;
  for (int i = 0; i < 3; i++) {
    z[i] = g->M[3 * i] * e[0] + g->M[3 * i + 1] * e[1] + g->M[3 * i + 2] * e[2];
    q += z[i] * z[i];
  }
  return q;
}

/* Ray / ellipsoid {q <= k^2} interval.  Along the ray q(t) = A t^2 + 2 B t + C;
   it is solved about the point of closest approach t* = -B/A, where
   q(t*) = h^2, so the roots are t* -/+ sqrt((k^2 - h^2)/A).  Returns 0 on a miss. */
static int ellipsoid_interval(const gauss *g, const double o[3], const double d[3], double *t0,
                              double *t1, double *h2_out) {
  double op[3], dp[3];
  double e[3] = {o[0] - g->mu[0], o[1] - g->mu[1], o[2] - g->mu[2]};
  for (int i = 0; i < 3; i++) {
    op[i] = g->M[3 * i] * e[0] + g->M[3 * i + 1] * e[1] + g->M[3 * i + 2] * e[2];
    dp[i] = g->M[3 * i] * d[0] + g->M[3 * i + 1] * d[1] + g->M[3 * i + 2] * d[2];
  }
  double A = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
  double ts = -(op[0] * dp[0] + op[1] * dp[1] + op[2] * dp[2]) / A;
  double h2 = 0;
  for (int i = 0; i < 3; i++) {
    double p = op[i] + ts * dp[i];
    h2 += p * p;
  }
  if (h2_out) *h2_out = h2;
  if (h2 > g->k2) return 0;
  double w = sqrt((g->k2 - h2) / A);
  *t0 = ts - w;
  *t1 = ts + w;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* One ray through Algorithm 1.                                             */

typedef struct { int64_t id; double t0, t1; } cand; /* Gaussians the ray's line meets */

typedef struct { int64_t g; double w, q; double z[3]; } contrib; /* one (sample, Gaussian) */

typedef struct {
  double t, dt, sigma, W[3];
  int64_t c_begin, c_end; /* range in the contrib list */
} sample_rec;

typedef struct {
  contrib *c; int64_t nc, cap_c;
  sample_rec *s; int64_t ns, cap_s;
} trace;

static void trace_push_contrib(trace *tr, contrib c) {
  if (tr->nc == tr->cap_c) {
    tr->cap_c = tr->cap_c ? 2 * tr->cap_c : 256;
    tr->c = (contrib *)realloc(tr->c, sizeof(contrib) * tr->cap_c);
  }
  tr->c[tr->nc++] = c;
}
static void trace_push_sample(trace *tr, sample_rec s) {
  if (tr->ns == tr->cap_s) {
    tr->cap_s = tr->cap_s ? 2 * tr->cap_s : 64;
    tr->s = (sample_rec *)realloc(tr->s, sizeof(sample_rec) * tr->cap_s);
  }
  tr->s[tr->ns++] = s;
}

typedef struct {
  const orc_scene *sc;
  const gauss *G;
  int K;
} prep;

/* closest(t_lo,t_hi) = min over Gaussians whose interval meets [t_lo,t_hi] of
   max(t_in, t_lo); +inf if none (Alg. 1 ClosestHit, Eq. 4). */
static double closest_hit(const cand *cd, int64_t nc, double lo, double hi) {
  double best = INFINITY;
  for (int64_t i = 0; i < nc; i++)
    if (cd[i].t0 <= hi && cd[i].t1 >= lo) {
      double t = cd[i].t0 > lo ? cd[i].t0 : lo;
      if (t < best) best = t;
    }
  return best;
}

typedef struct {
  /* outputs */
  double C[3], T;
  int64_t stats[ST_NSTAT];
  /* smallest relative distance to its threshold of any discrete decision that
     can change the pixel: sample inclusion q <= k^2, termination T > T_eps and,
     where the restart point is not snapped, segment emptiness */
  double margin;
  /* optional per-segment hit lists */
  int64_t *seg_off; double *seg_a; double *seg_dt; int64_t *ids; int64_t cap_ids, cap_segs;
  int64_t n_segs, n_ids, overflow;
  /* where the march ended: the segment start at which T <= T_eps stopped it,
     else t_f (the loop ran past t_f or nothing further was hit) */
  double t_end;
} ray_out;

static void note_margin(ray_out *ro, double m) { if (m < ro->margin) ro->margin = m; }

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

static void march_ray(const prep *P, const orc_camera *cam, const orc_opts *op, const double o[3],
                      const double d[3], ray_out *ro, trace *tr) {
  const gauss *G = P->G;
  const int64_t N = P->sc->n;
  const int K = P->K, deg = P->sc->sh_degree;
  const double tn = cam->t_near, tf = cam->t_far;

  /* every Gaussian against the ray (no acceleration structure) */
  cand *cd = (cand *)malloc(sizeof(cand) * (N > 0 ? N : 1));
  int64_t nc = 0;
  for (int64_t l = 0; l < N; l++) {
    if (!G[l].active) continue;
    double t0, t1;
    int hit = ellipsoid_interval(&G[l], o, d, &t0, &t1, NULL);
    if (hit) { cd[nc].id = l; cd[nc].t0 = t0; cd[nc].t1 = t1; nc++; }
  }
  /* colour of each candidate at this ray direction */
  double Y[16];
  orc_sh_basis(deg, d, Y);
  double *col = (double *)malloc(sizeof(double) * 3 * (nc > 0 ? nc : 1));
  for (int64_t i = 0; i < nc; i++) gaussian_colour(P->sc, K, cd[i].id, Y, d, col + 3 * i);
  unsigned char *seen = (unsigned char *)calloc(nc > 0 ? nc : 1, 1);
  int64_t *hl = (int64_t *)malloc(sizeof(int64_t) * (nc > 0 ? nc : 1));

  double T = 1.0, C[3] = {0, 0, 0};
  ro->t_end = tf;
  const int fixed = !op->adaptive;
  const double dS_fixed = op->dt * op->n_s;
  int64_t seg_i = 0;   /* fixed mode: segment index on the grid a = tn + i dS */
  double a = tn;
  int ess_snap = (op->ess == 1) && fixed;

  int done = 0;
  if (op->ess) {
    ro->stats[ST_CLOSEST]++;
    double tc = closest_hit(cd, nc, tn, tf);
    if (!(tc < INFINITY)) done = 1; /* nothing along the ray */
    else if (ess_snap) {
      seg_i = (int64_t)floor((tc - tn) / dS_fixed);
      if (seg_i < 0) seg_i = 0;
      a = tn + (double)seg_i * dS_fixed;
    } else a = tc;
  }

  while (!done) {
    if (fixed && op->ess != 2) a = tn + (double)seg_i * dS_fixed;
    if (!(a < tf)) break;
    if (op->t_eps > 0) note_margin(ro, fabs(T - op->t_eps) / op->t_eps);
    if (!(T > op->t_eps)) { ro->t_end = a; break; }
    double dt;
    if (fixed) dt = op->dt;
    else {
      /* Eq. 5 with d_i = |s_i - o| = a (unit direction) */
      double base = a / op->beta > op->dt_min ? a / op->beta : op->dt_min;
      dt = base * pow(T, -1.0 / 3.0);
      if (!(dt < op->dt_max)) dt = op->dt_max;
    }
    double b = (fixed && op->ess != 2) ? tn + (double)(seg_i + 1) * dS_fixed : a + op->n_s * dt;

    /* the segment's hit set H = {l : [t_in,t_out] meets [a,b]} */
    int64_t nh = 0;
    double depth = -INFINITY; /* how far the most-overlapping interval reaches into [a,b] */
    for (int64_t i = 0; i < nc; i++) {
      double dep = fmin(b - cd[i].t0, cd[i].t1 - a);
      if (dep > depth) depth = dep;
      if (cd[i].t0 <= b && cd[i].t1 >= a) hl[nh++] = i;
    }
    /* Where the restart point is not snapped to the grid, whether a segment is
       empty changes the schedule; record how close that decision was. */
    if (op->ess && !ess_snap && nc > 0) note_margin(ro, fabs(depth) / fmax(1.0, fabs(b)));
    if (nh == 0) {
      if (op->ess) {
        ro->stats[ST_CLOSEST]++;
        double tc = closest_hit(cd, nc, b, tf);
        if (!(tc < INFINITY)) break;
        if (ess_snap) {
          int64_t j = (int64_t)floor((tc - tn) / dS_fixed);
          seg_i = j > seg_i + 1 ? j : seg_i + 1;
        } else a = tc;
      } else {
        if (fixed && op->ess != 2) seg_i++;
        else a = b;
      }
      continue;
    }
    ro->stats[ST_SEGMENTS]++;
    ro->stats[ST_P] += nh;
    for (int64_t j = 0; j < nh; j++)
      if (!seen[hl[j]]) { seen[hl[j]] = 1; ro->stats[ST_Q]++; }
    if (ro->seg_off) {
      if (ro->n_segs < ro->cap_segs && ro->n_ids + nh <= ro->cap_ids) {
        ro->seg_a[ro->n_segs] = a;
        ro->seg_dt[ro->n_segs] = dt;
        for (int64_t j = 0; j < nh; j++) ro->ids[ro->n_ids + j] = cd[hl[j]].id;
        qsort(ro->ids + ro->n_ids, nh, sizeof(int64_t), cmp_i64);
        ro->n_ids += nh;
        ro->seg_off[++ro->n_segs] = ro->n_ids;
      } else ro->overflow = 1;
    }

    /* RayUpdate: N_s midpoint samples, density-weighted colour, Eq. 3 */
    for (int k = 0; k < op->n_s; k++) {
      double t;
      if (fixed && op->ess != 2) t = tn + ((double)seg_i * op->n_s + k + 0.5) * dt;
      else t = a + (k + 0.5) * dt;
      if (!(t < tf)) continue;
      ro->stats[ST_SAMPLES]++;
      double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
      double sigma = 0, W[3] = {0, 0, 0};
      sample_rec sr;
      sr.c_begin = tr ? tr->nc : 0;
      for (int64_t j = 0; j < nh; j++) {
        const gauss *g = &G[cd[hl[j]].id];
        double z[3];
        double q = qform(g, x, z);
        note_margin(ro, fabs(q - g->k2) / g->k2);
        if (!(q <= g->k2)) continue;
        double w = g->sig * exp(-0.5 * q);
        sigma += w;
        for (int ch = 0; ch < 3; ch++) W[ch] += w * col[3 * hl[j] + ch];
        if (tr) {
          contrib c;
          c.g = cd[hl[j]].id; c.w = w; c.q = q;
          c.z[0] = z[0]; c.z[1] = z[1]; c.z[2] = z[2];
          trace_push_contrib(tr, c);
        }
      }
      if (tr) {
        sr.c_end = tr->nc;
        sr.t = t; sr.dt = dt; sr.sigma = sigma;
        sr.W[0] = W[0]; sr.W[1] = W[1]; sr.W[2] = W[2];
        trace_push_sample(tr, sr);
      }
      if (sigma > 0) {
        double alpha = -expm1(-sigma * dt);
        for (int ch = 0; ch < 3; ch++) C[ch] += T * (alpha / sigma) * W[ch];
        T *= exp(-sigma * dt);
      }
    }
    if (fixed && op->ess != 2) seg_i++;
    else a = b;
  }
  for (int ch = 0; ch < 3; ch++) ro->C[ch] = C[ch] + T * op->bg[ch];
  ro->T = T;
  free(cd); free(col); free(seen); free(hl);
}

/* ------------------------------------------------------------------------ */
/* C ABI for the Python wrapper                                               */

typedef struct { gauss *G; } orc_prep_handle;

static gauss *prepare_all(const orc_scene *sc, double sigma_eps) {
  gauss *G = (gauss *)malloc(sizeof(gauss) * (sc->n > 0 ? sc->n : 1));
  for (int64_t l = 0; l < sc->n; l++) make_gauss(sc, sigma_eps, l, &G[l]);
  return G;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Forward: colour and transmittance of the listed pixels of one view.
   stats: [n_rays, ST_NSTAT] int64 (may be NULL); margin: [n_rays] (may be NULL). */
int orc_render(const orc_scene *sc, const orc_camera *cam, const orc_opts *op, const int64_t *pix,
               int64_t n_rays, double *out_rgb, double *out_T, int64_t *stats, double *margin) {
  if (sc->sh_degree < 0 || sc->sh_degree > 3) return -1;
  gauss *G = prepare_all(sc, op->sigma_eps);
  prep P = {sc, G, (sc->sh_degree + 1) * (sc->sh_degree + 1)};
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < n_rays; r++) {
    double o[3], d[3];
    make_ray(cam, pix[r], o, d);
    ray_out ro;
    memset(&ro, 0, sizeof ro);
    ro.margin = INFINITY;
    march_ray(&P, cam, op, o, d, &ro, NULL);
    for (int ch = 0; ch < 3; ch++) out_rgb[3 * r + ch] = ro.C[ch];
    out_T[r] = ro.T;
    if (stats) for (int s = 0; s < ST_NSTAT; s++) stats[r * ST_NSTAT + s] = ro.stats[s];
    if (margin) margin[r] = ro.margin;
  }
  free(G);
  return 0;
}

/* Per-segment hit lists of one ray (original Gaussian ids, ascending within a
   segment).  seg_off has room for cap_segs+1 entries.  Returns the number of
   processed segments, or -1 when a capacity was too small. */
int64_t orc_hits(const orc_scene *sc, const orc_camera *cam, const orc_opts *op, int64_t pix,
                 int64_t *seg_off, double *seg_a, double *seg_dt, int64_t cap_segs, int64_t *ids,
                 int64_t cap_ids) {
  gauss *G = prepare_all(sc, op->sigma_eps);
  prep P = {sc, G, (sc->sh_degree + 1) * (sc->sh_degree + 1)};
  double o[3], d[3];
  make_ray(cam, pix, o, d);
  ray_out ro;
  memset(&ro, 0, sizeof ro);
  ro.margin = INFINITY;
  ro.seg_off = seg_off; ro.seg_a = seg_a; ro.seg_dt = seg_dt; ro.ids = ids;
  ro.cap_ids = cap_ids; ro.cap_segs = cap_segs;
  seg_off[0] = 0;
  march_ray(&P, cam, op, o, d, &ro, NULL);
  free(G);
  return ro.overflow ? -1 : ro.n_segs;
}

/* Derivative of the rotation matrix entries with respect to the unit
   quaternion components, from quat_to_rot differentiated by hand. */
static void drot_dq(const double q[4], const double dR[9], double dq[4]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  /* R0=1-2(y2+z2) R1=2(xy-wz) R2=2(xz+wy) R3=2(xy+wz) R4=1-2(x2+z2) R5=2(yz-wx)
     R6=2(xz-wy) R7=2(yz+wx) R8=1-2(x2+y2) */
  dq[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dq[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] +
               w * dR[7] - 2 * x * dR[8]);
  dq[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
               z * dR[7] - 2 * y * dR[8]);
  dq[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] +
               x * dR[6] + y * dR[7]);
}

/* Backward: accumulates dL/d(parameters) into the gradient arrays (caller
   zeroes them) for the loss whose derivatives with respect to the listed
   pixels' colour and final transmittance are grad_rgb and grad_T (grad_T may
   be NULL).  Reverse sweep over each ray's recorded samples. */
int orc_backward(const orc_scene *sc, const orc_camera *cam, const orc_opts *op, const int64_t *pix,
                 int64_t n_rays, const double *grad_rgb, const double *grad_T, double *g_means,
                 double *g_log_scales, double *g_quats, double *g_density, double *g_sh,
                 double *g_sg) {
  if (sc->n_sg < 0 || (sc->n_sg > 0 && (!sc->sg || !g_sg))) return -1;
  if (sc->sh_degree < 0 || sc->sh_degree > 3) return -1;
  gauss *G = prepare_all(sc, op->sigma_eps);
  const int K = (sc->sh_degree + 1) * (sc->sh_degree + 1);
  prep P = {sc, G, K};
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < n_rays; r++) {
    double o[3], d[3];
    make_ray(cam, pix[r], o, d);
    ray_out ro;
    memset(&ro, 0, sizeof ro);
    ro.margin = INFINITY;
    trace tr;
    memset(&tr, 0, sizeof tr);
    march_ray(&P, cam, op, o, d, &ro, &tr);
    double Y[16];
    orc_sh_basis(sc->sh_degree, d, Y);
    const double *Gc = grad_rgb + 3 * r;
    double gT = grad_T ? grad_T[r] : 0.0;
    double Tfin = ro.T;

    /* transmittance before each sample, front to back */
    double *Tk = (double *)malloc(sizeof(double) * (tr.ns > 0 ? tr.ns : 1));
    double T = 1.0;
    for (int64_t k = 0; k < tr.ns; k++) {
      Tk[k] = T;
      if (tr.s[k].sigma > 0) T *= exp(-tr.s[k].sigma * tr.s[k].dt);
    }
    /* reverse sweep; S = radiance arriving from behind sample k (later samples + background) */
    double S[3] = {Tfin * op->bg[0], Tfin * op->bg[1], Tfin * op->bg[2]};
    for (int64_t k = tr.ns - 1; k >= 0; k--) {
      const sample_rec *s = &tr.s[k];
      if (!(s->sigma > 0)) continue;
      double sg = s->sigma, dt = s->dt;
      double E = exp(-sg * dt), alpha = -expm1(-sg * dt);
      double phi = alpha / sg;
      double dphi = (sg * dt * E - alpha) / (sg * sg); /* d(alpha/sigma)/dsigma */
      double GW = Gc[0] * s->W[0] + Gc[1] * s->W[1] + Gc[2] * s->W[2];
      double GS = Gc[0] * S[0] + Gc[1] * S[1] + Gc[2] * S[2];
      /* C = sum_k T_k phi_k W_k + T_fin bg ; T_{j>k} and T_fin carry exp(-sigma_k dt_k) */
      double dsig = Tk[k] * dphi * GW - dt * GS - dt * gT * Tfin;
      double dW[3] = {Tk[k] * phi * Gc[0], Tk[k] * phi * Gc[1], Tk[k] * phi * Gc[2]};
      for (int64_t c = s->c_begin; c < s->c_end; c++) {
        const contrib *cb = &tr.c[c];
        const gauss *g = &G[cb->g];
        const int64_t l = cb->g;
        double col[3];
        gaussian_colour(sc, K, l, Y, d, col);
        double dw = dsig + dW[0] * col[0] + dW[1] * col[1] + dW[2] * col[2];
        double dq = -0.5 * cb->w * dw; /* w = sig exp(-q/2) */
        double xm[3] = {o[0] + s->t * d[0] - g->mu[0], o[1] + s->t * d[1] - g->mu[1],
                        o[2] + s->t * d[2] - g->mu[2]};
        double gmu[3], gls[3], dR[9], dqh[4], gq[4];
        /* dq/dmu = -2 M^T z */
        for (int j = 0; j < 3; j++)
          gmu[j] = dq * -2.0 * (g->M[j] * cb->z[0] + g->M[3 + j] * cb->z[1] + g->M[6 + j] * cb->z[2]);
        /* z_i = (1/s_i) sum_j R_ji xm_j, s_i = exp(l_i): dq/dl_i = -2 z_i^2 */
        for (int i = 0; i < 3; i++) gls[i] = dq * -2.0 * cb->z[i] * cb->z[i];
        /* dq/dR_ji = 2 z_i xm_j / s_i */
        for (int j = 0; j < 3; j++)
          for (int i = 0; i < 3; i++) dR[3 * j + i] = dq * 2.0 * cb->z[i] * xm[j] / g->s[i];
        drot_dq(g->qhat, dR, dqh);
        /* through qhat = q/|q| */
        double pr = dqh[0] * g->qhat[0] + dqh[1] * g->qhat[1] + dqh[2] * g->qhat[2] + dqh[3] * g->qhat[3];
        for (int i = 0; i < 4; i++) gq[i] = (dqh[i] - pr * g->qhat[i]) / g->qnorm;
        double gd = dw * exp(-0.5 * cb->q);
        for (int j = 0; j < 3; j++) {
#pragma omp atomic
          g_means[3 * l + j] += gmu[j];
#pragma omp atomic
          g_log_scales[3 * l + j] += gls[j];
        }
        for (int i = 0; i < 4; i++) {
#pragma omp atomic
          g_quats[4 * l + i] += gq[i];
        }
#pragma omp atomic
        g_density[l] += gd;
        for (int m = 0; m < K; m++)
          for (int ch = 0; ch < 3; ch++) {
#pragma omp atomic
            g_sh[(l * K + m) * 3 + ch] += Y[m] * cb->w * dW[ch];
          }
        if (sc->n_sg) {
          const double dc[3] = {cb->w * dW[0], cb->w * dW[1], cb->w * dW[2]};
          sg_backward(sc, l, d, dc, g_sg);
        }
      }
      for (int ch = 0; ch < 3; ch++) S[ch] += Tk[k] * phi * s->W[ch];
    }
    free(Tk);
    free(tr.c);
    free(tr.s);
  }
  free(G);
  return 0;
}

/* Per-Gaussian ellipsoid data for the geometry checks: k^2, active flag, the
   rotation R and the world-axis half-lengths of the ellipsoid's minimal AABB,
   L_i = k sqrt(sum_j r_ij^2 s_j^2) (Supp. B, minimal AABB). */
void orc_gaussians(const orc_scene *sc, double sigma_eps, double *k2, int32_t *active, double *R,
                   double *half) {
  for (int64_t l = 0; l < sc->n; l++) {
    gauss g;
    make_gauss(sc, sigma_eps, l, &g);
    active[l] = g.active;
    k2[l] = g.active ? g.k2 : 0;
    for (int i = 0; i < 9; i++) R[9 * l + i] = g.active ? g.R[i] : 0;
    for (int i = 0; i < 3; i++) {
      double acc = 0;
      for (int j = 0; j < 3; j++) acc += g.R[3 * i + j] * g.R[3 * i + j] * g.s[j] * g.s[j];
      half[3 * l + i] = g.active ? sqrt(g.k2) * sqrt(acc) : 0;
    }
  }
}

/* False positives of the AABB test along a whole ray (Sec. 3.4, Eq. 6;
   minimal AABB of Supp. B): the number of active Gaussians whose minimal AABB
   mu +/- L, L_i = k sqrt(sum_j r_ij^2 s_j^2), meets the ray over [t_n, t_end]
   while the ellipsoid's chord does not, t_end being where the ray's march
   ended (Algorithm 1).  Also per ray: t_end, and how many Gaussians had one of
   the two decisions within a relative 1e-5 of flipping (a near tie: the slab
   interval's overlap, |h^2 - k^2| / k^2, or a chord end against t_n / t_end).
   The AABB test is the slab method: the ray meets the box over [lo, hi]
   iff max(lo, max_i min(t0_i, t1_i)) <= min(hi, min_i max(t0_i, t1_i)),
   t0_i, t1_i the parameters of the two planes of axis i. */
int orc_false_positives(const orc_scene *sc, const orc_camera *cam, const orc_opts *op,
                        const int64_t *pix, int64_t n_rays, int64_t *count, int64_t *ties,
                        double *t_end) {
  if (sc->sh_degree < 0 || sc->sh_degree > 3) return -1;
  gauss *G = prepare_all(sc, op->sigma_eps);
  prep P = {sc, G, (sc->sh_degree + 1) * (sc->sh_degree + 1)};
  const double tol = 1e-5;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < n_rays; r++) {
    double o[3], d[3];
    make_ray(cam, pix[r], o, d);
    ray_out ro;
    memset(&ro, 0, sizeof ro);
    ro.margin = INFINITY;
    march_ray(&P, cam, op, o, d, &ro, NULL);
    const double lo = cam->t_near, hi = ro.t_end;
    int64_t fp = 0, nt = 0;
    for (int64_t l = 0; l < sc->n; l++) {
      const gauss *g = &G[l];
      if (!g->active) continue;
      double enter = lo, leave = hi;
      for (int i = 0; i < 3; i++) {
        double acc = 0;
        for (int j = 0; j < 3; j++) acc += g->R[3 * i + j] * g->R[3 * i + j] * g->s[j] * g->s[j];
        const double L = sqrt(g->k2) * sqrt(acc);
        const double ta = (g->mu[i] - L - o[i]) / d[i], tb = (g->mu[i] + L - o[i]) / d[i];
        enter = fmax(enter, fmin(ta, tb));
        leave = fmin(leave, fmax(ta, tb));
      }
      const int box = enter <= leave;
      double t0, t1, h2;
      const int chord = ellipsoid_interval(g, o, d, &t0, &t1, &h2);
      const int ell = chord && t0 <= hi && t1 >= lo;
      if (box && !ell) fp++;
      int tie = fabs(leave - enter) <= tol * fmax(1.0, fabs(enter));
      tie |= fabs(h2 - g->k2) <= tol * g->k2;
      tie |= chord && (fabs(t0 - hi) <= tol * fmax(1.0, fabs(hi)) ||
                       fabs(t1 - lo) <= tol * fmax(1.0, fabs(lo)));
      nt += tie;
    }
    count[r] = fp;
    ties[r] = nt;
    t_end[r] = ro.t_end;
  }
  free(G);
  return 0;
}

/* Ray / ellipsoid data of listed Gaussians for one pixel's ray (for tests that
   classify near ties): k^2, the squared local distance h^2 of the point of
   closest approach and the chord [t0, t1] (NaN for a miss or an inactive
   Gaussian). */
void orc_chords(const orc_scene *sc, const orc_camera *cam, double sigma_eps, int64_t pix,
                const int64_t *ids, int64_t n, double *k2, double *h2, double *t0, double *t1) {
  double o[3], d[3];
  make_ray(cam, pix, o, d);
  for (int64_t i = 0; i < n; i++) {
    gauss g;
    make_gauss(sc, sigma_eps, ids[i], &g);
    k2[i] = h2[i] = t0[i] = t1[i] = NAN;
    if (!g.active) continue;
    double a, b, hh;
    int hit = ellipsoid_interval(&g, o, d, &a, &b, &hh);
    k2[i] = g.k2;
    h2[i] = hh;
    if (hit) { t0[i] = a; t1[i] = b; }
  }
}

/* Colour of Gaussian l at listed unit directions (for tests of the colour model). */
void orc_colour(const orc_scene *sc, int64_t l, const double *dirs, int64_t n, double *out) {
  const int K = (sc->sh_degree + 1) * (sc->sh_degree + 1);
  for (int64_t i = 0; i < n; i++) {
    double Y[16];
    orc_sh_basis(sc->sh_degree, dirs + 3 * i, Y);
    gaussian_colour(sc, K, l, Y, dirs + 3 * i, out + 3 * i);
  }
}

/* Evaluate q and the truncated density of one Gaussian at points (for tests). */
void orc_density_at(const orc_scene *sc, double sigma_eps, int64_t l, const double *x, int64_t n,
                    double *out) {
  gauss g;
  make_gauss(sc, sigma_eps, l, &g);
  for (int64_t i = 0; i < n; i++) {
    double z[3];
    if (!g.active) { out[i] = 0; continue; }
    double q = qform(&g, x + 3 * i, z);
    out[i] = q <= g.k2 ? g.sig * exp(-0.5 * q) : 0.0;
  }
}
