/*
 * mrpop_oracle.c -- plain FP64 CPU oracle for the MR. POP hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code with the HIP library: both sides read the same seeded inputs and
 * nothing else.
 *
 * What it computes (paper sections cited per function):
 *   - forward kinematics of serial arms to world collision spheres
 *     (Sec. "Multi-Thread Reassignment for Collision Checking": robots are
 *     approximated by spheres attached to their links);
 *   - the composite edge check "(q, q') in C^f": discretise the edge into
 *     states, and test every robot sphere against environment spheres and
 *     axis-aligned boxes and against every other robot's spheres (Sec.
 *     "Problem Setup": composite free space excludes robot-robot contact);
 *     reported as the minimum signed margin (distance minus radius sum);
 *   - a coarse-to-fine checker with early exit (same section: one
 *     conservative sphere per link, then the fine spheres of flagged links),
 *     which also counts the pair tests it performs;
 *   - NEAREST(V, q, c) of Alg. 2: argmin of ||q - q_v|| over vertices with
 *     g_v + ||q - q_v|| < c, ties toward lower cost, then lower index;
 *   - the counter-based random stream and the informed sample of Alg. 2
 *     (prolate hyperspheroid with foci q_start, q_goal and transverse
 *     diameter c_best).
 *
 * Precision: all geometry in double.  The number of states of an edge is an
 * integer decided from single-precision inputs; it is evaluated with one
 * stated single-precision formula so that both sides get the same count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LINKS 16

typedef struct {
  int32_t n_robots;
  const int32_t *nj;      /* [R] joints of robot r                              */
  const int32_t *q_off;   /* [R] offset of robot r's joints in a composite q    */
  const float *dh;        /* [sum nj][4] a_{j-1}, d_j, alpha_{j-1}, theta_off_j */
  const float *base;      /* [R][12] row-major world-from-base 3x4              */
  const int32_t *ns;      /* [R] spheres of robot r                             */
  const int32_t *s_off;   /* [R] offset of robot r's spheres                    */
  const int32_t *s_link;  /* [sum ns] link index 0..nj                          */
  const float *s_xyzr;    /* [sum ns][4] link-local centre, radius              */
  int32_t n_env_spheres;
  const float *env_s;     /* [n][4] centre, radius                              */
  int32_t n_env_boxes;
  const float *env_b;     /* [n][6] lo xyz, hi xyz                              */
} orc_scene;

/* ------------------------------------------------------------------------ */
/* 4x4 homogeneous matrices                                                  */
/* ------------------------------------------------------------------------ */

typedef struct { double m[4][4]; } mat4;

static mat4 mat4_identity(void) {
  mat4 r;
  memset(&r, 0, sizeof r);
  for (int i = 0; i < 4; ++i) r.m[i][i] = 1.0;
  return r;
}

static mat4 mat4_mul(const mat4 *a, const mat4 *b) {
  mat4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += a->m[i][k] * b->m[k][j];
      r.m[i][j] = s;
    }
  return r;
}

static mat4 rot_x(double a) {
  mat4 r = mat4_identity();
  r.m[1][1] = cos(a); r.m[1][2] = -sin(a);
  r.m[2][1] = sin(a); r.m[2][2] = cos(a);
  return r;
}
static mat4 rot_z(double a) {
  mat4 r = mat4_identity();
  r.m[0][0] = cos(a); r.m[0][1] = -sin(a);
  r.m[1][0] = sin(a); r.m[1][1] = cos(a);
  return r;
}
static mat4 trans(double x, double y, double z) {
  mat4 r = mat4_identity();
  r.m[0][3] = x; r.m[1][3] = y; r.m[2][3] = z;
  return r;
}

static void apply(const mat4 *t, const double p[3], double out[3]) {
  for (int i = 0; i < 3; ++i)
    out[i] = t->m[i][0] * p[0] + t->m[i][1] * p[1] + t->m[i][2] * p[2] + t->m[i][3];
}

/* Frames T_0..T_nj of robot r at joint vector q (nj values).  T_0 is the
 * base; T_j = T_{j-1} RotX(alpha_{j-1}) TransX(a_{j-1}) RotZ(q_j + theta_off_j)
 * TransZ(d_j)  (Craig's modified Denavit-Hartenberg convention). */
static void robot_frames(const orc_scene *s, int r, const double *q, mat4 *frames) {
  mat4 t = mat4_identity();
  const float *b = s->base + 12 * r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 4; ++j) t.m[i][j] = b[4 * i + j];
  frames[0] = t;
  int row0 = 0;
  for (int k = 0; k < r; ++k) row0 += s->nj[k];
  for (int j = 1; j <= s->nj[r]; ++j) {
    const float *d = s->dh + 4 * (row0 + j - 1);
    double a = d[0], dd = d[1], alpha = d[2], th = q[j - 1] + (double)d[3];
    mat4 x1 = rot_x(alpha), x2 = trans(a, 0, 0), x3 = rot_z(th), x4 = trans(0, 0, dd);
    mat4 m = mat4_mul(&frames[j - 1], &x1);
    m = mat4_mul(&m, &x2);
    m = mat4_mul(&m, &x3);
    frames[j] = mat4_mul(&m, &x4);
  }
}

/* World sphere centres (and radii) of every robot at composite q (D doubles).
 * out: [sum ns][4]. */
static void all_world_spheres(const orc_scene *s, const double *q, double *out) {
  mat4 frames[ORC_MAX_LINKS];
  for (int r = 0; r < s->n_robots; ++r) {
    robot_frames(s, r, q + s->q_off[r], frames);
    for (int i = 0; i < s->ns[r]; ++i) {
      int g = s->s_off[r] + i;
      double p[3] = {s->s_xyzr[4 * g], s->s_xyzr[4 * g + 1], s->s_xyzr[4 * g + 2]};
      apply(&frames[s->s_link[g]], p, out + 4 * g);
      out[4 * g + 3] = s->s_xyzr[4 * g + 3];
    }
  }
}

int orc_total_spheres(const orc_scene *s) {
  int n = 0;
  for (int r = 0; r < s->n_robots; ++r) n += s->ns[r];
  return n;
}
int orc_dof(const orc_scene *s) {
  int n = 0;
  for (int r = 0; r < s->n_robots; ++r) n += s->nj[r];
  return n;
}

/* FK to world spheres for n_cfg composite configurations (float inputs).
 * out: [n_cfg][sum ns][4] doubles. */
void orc_fk_spheres(const orc_scene *s, const float *q, int64_t n_cfg, double *out) {
  int D = orc_dof(s), S = orc_total_spheres(s);
  double *qd = (double *)malloc(sizeof(double) * D);
  for (int64_t c = 0; c < n_cfg; ++c) {
    for (int j = 0; j < D; ++j) qd[j] = q[c * D + j];
    all_world_spheres(s, qd, out + c * (int64_t)S * 4);
  }
  free(qd);
}

/* ------------------------------------------------------------------------ */
/* Margins: distance minus radius sum (negative = penetration)               */
/* ------------------------------------------------------------------------ */

static double margin_sphere_sphere(const double *c, double r, const double *o, double ro) {
  double dx = c[0] - o[0], dy = c[1] - o[1], dz = c[2] - o[2];
  return sqrt(dx * dx + dy * dy + dz * dz) - (r + ro);
}

/* Distance from a point to an axis-aligned box is the norm of the per-axis
 * excess max(lo - c, 0, c - hi) (Arvo, Graphics Gems, 1990). */
static double margin_sphere_box(const double *c, double r, const float *b) {
  double e2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double lo = b[a], hi = b[3 + a];
    double e = 0.0;
    if (lo - c[a] > e) e = lo - c[a];
    if (c[a] - hi > e) e = c[a] - hi;
    e2 += e * e;
  }
  return sqrt(e2) - r;
}

/* Minimum margin over every pair at one composite state; world: [S][4]. */
static double state_min_margin(const orc_scene *s, const double *world) {
  double m = INFINITY;
  int S = orc_total_spheres(s);
  for (int g = 0; g < S; ++g) {
    const double *c = world + 4 * g;
    for (int k = 0; k < s->n_env_spheres; ++k) {
      double o[3] = {s->env_s[4 * k], s->env_s[4 * k + 1], s->env_s[4 * k + 2]};
      double v = margin_sphere_sphere(c, c[3], o, s->env_s[4 * k + 3]);
      if (v < m) m = v;
    }
    for (int k = 0; k < s->n_env_boxes; ++k) {
      double v = margin_sphere_box(c, c[3], s->env_b + 6 * k);
      if (v < m) m = v;
    }
  }
  for (int i = 0; i < s->n_robots; ++i)
    for (int j = i + 1; j < s->n_robots; ++j)
      for (int a = 0; a < s->ns[i]; ++a)
        for (int b = 0; b < s->ns[j]; ++b) {
          const double *ca = world + 4 * (s->s_off[i] + a), *cb = world + 4 * (s->s_off[j] + b);
          double v = margin_sphere_sphere(ca, ca[3], cb, cb[3]);
          if (v < m) m = v;
        }
  return m;
}

/* ------------------------------------------------------------------------ */
/* Edge discretisation                                                       */
/* ------------------------------------------------------------------------ */

/* Number of states of an edge: n = 1 + ceil(Linf / res), Linf the largest
 * per-joint change, everything in single precision with correctly rounded
 * division.  The paper only says the edge is discretised into motions
 * (collision-checking section); this count rule is the stated reading. */
int32_t orc_edge_nstates(const float *qa, const float *qb, int D, float res) {
  float linf = 0.0f;
  for (int j = 0; j < D; ++j) {
    float d = fabsf(qb[j] - qa[j]);
    if (d > linf) linf = d;
  }
  if (linf == 0.0f) return 1;
  float ratio = linf / res;
  return 1 + (int32_t)ceilf(ratio);
}

/* State k of n along the edge: q_a + (k/(n-1)) (q_b - q_a), last one exactly q_b. */
static void edge_state(const float *qa, const float *qb, int D, int n, int k, double *q) {
  if (n <= 1 || k == n - 1) {
    for (int j = 0; j < D; ++j) q[j] = (n <= 1) ? qa[j] : qb[j];
    return;
  }
  double t = (double)k / (double)(n - 1);
  for (int j = 0; j < D; ++j) q[j] = (double)qa[j] + t * ((double)qb[j] - (double)qa[j]);
}

/* ------------------------------------------------------------------------ */
/* Brute-force classification (minimum margin over all pairs and states)     */
/* ------------------------------------------------------------------------ */

typedef struct {
  const orc_scene *s;
  const float *qa, *qb;
  int64_t e0, e1;
  float res;
  const int32_t *nstates_opt;
  int32_t *out_n;
  double *out_m;
  uint8_t *out_valid;
  int64_t *counts;
  int early_exit;
  int mode; /* 0 = classify, 1 = fast */
} job_t;

static void classify_range(job_t *J) {
  const orc_scene *s = J->s;
  int D = orc_dof(s), S = orc_total_spheres(s);
  double *q = (double *)malloc(sizeof(double) * D);
  double *w = (double *)malloc(sizeof(double) * 4 * (S > 0 ? S : 1));
  for (int64_t e = J->e0; e < J->e1; ++e) {
    const float *qa = J->qa + e * D, *qb = J->qb + e * D;
    int n = J->nstates_opt ? J->nstates_opt[e] : orc_edge_nstates(qa, qb, D, J->res);
    double m = INFINITY;
    for (int k = 0; k < n; ++k) {
      edge_state(qa, qb, D, n, k, q);
      all_world_spheres(s, q, w);
      double v = state_min_margin(s, w);
      if (v < m) m = v;
    }
    J->out_n[e] = n;
    J->out_m[e] = m;
  }
  free(q);
  free(w);
}

/* ------------------------------------------------------------------------ */
/* Coarse-to-fine checker with early exit and pair-test counters             */
/* ------------------------------------------------------------------------ */

/* counts[]: 0 states checked, 1 robot FK evaluations, 2 coarse sphere-sphere
 * (env), 3 coarse sphere-box, 4 coarse robot-robot, 5 fine sphere-sphere
 * (env), 6 fine sphere-box, 7 fine robot-robot, 8 edges found invalid. */
#define ORC_NCOUNT 9

/* One conservative sphere per link: centre at the middle of the bounding
 * box of the link's sphere centres, radius reaching past every fine sphere,
 * plus 1e-5 m.  Links without spheres get radius -1 (never flagged). */
static void coarse_spheres(const orc_scene *s, int r, double (*cs)[4]) {
  int nl = s->nj[r] + 1;
  for (int l = 0; l < nl; ++l) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int any = 0;
    for (int i = 0; i < s->ns[r]; ++i) {
      int g = s->s_off[r] + i;
      if (s->s_link[g] != l) continue;
      any = 1;
      for (int a = 0; a < 3; ++a) {
        double v = s->s_xyzr[4 * g + a];
        if (v < lo[a]) lo[a] = v;
        if (v > hi[a]) hi[a] = v;
      }
    }
    if (!any) { cs[l][0] = cs[l][1] = cs[l][2] = 0.0; cs[l][3] = -1.0; continue; }
    double c[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
    double rad = 0.0;
    for (int i = 0; i < s->ns[r]; ++i) {
      int g = s->s_off[r] + i;
      if (s->s_link[g] != l) continue;
      double dx = s->s_xyzr[4 * g] - c[0], dy = s->s_xyzr[4 * g + 1] - c[1], dz = s->s_xyzr[4 * g + 2] - c[2];
      double v = sqrt(dx * dx + dy * dy + dz * dz) + s->s_xyzr[4 * g + 3];
      if (v > rad) rad = v;
    }
    cs[l][0] = c[0]; cs[l][1] = c[1]; cs[l][2] = c[2]; cs[l][3] = rad + 1e-5;
  }
}

/* Collision test of one composite state, coarse link spheres first, fine
 * spheres only for flagged (link, obstacle) and (link, link) pairs.  Returns 1
 * if the state collides.  With stop_at_hit == 0 every flagged pair is still
 * refined, so the counters give the full hierarchical work of the state. */
static int state_collides_fast(const orc_scene *s, const double *q, double (*coarse)[ORC_MAX_LINKS][4],
                               mat4 (*frames)[ORC_MAX_LINKS], double (*cw)[ORC_MAX_LINKS][4],
                               int64_t *cnt, int stop_at_hit) {
  int hit = 0;
  int R = s->n_robots;
  for (int r = 0; r < R; ++r) {
    robot_frames(s, r, q + s->q_off[r], frames[r]);
    cnt[1]++;
    for (int l = 0; l <= s->nj[r]; ++l) {
      apply(&frames[r][l], coarse[r][l], cw[r][l]);
      cw[r][l][3] = coarse[r][l][3];
    }
  }
  for (int r = 0; r < R; ++r) {
    for (int l = 0; l <= s->nj[r]; ++l) {
      if (cw[r][l][3] < 0) continue;
      for (int k = 0; k < s->n_env_spheres; ++k) {
        const float *o = s->env_s + 4 * k;
        double od[3] = {o[0], o[1], o[2]};
        cnt[2]++;
        if (margin_sphere_sphere(cw[r][l], cw[r][l][3], od, o[3]) >= 0) continue;
        for (int i = 0; i < s->ns[r]; ++i) {
          int g = s->s_off[r] + i;
          if (s->s_link[g] != l) continue;
          double p[3] = {s->s_xyzr[4 * g], s->s_xyzr[4 * g + 1], s->s_xyzr[4 * g + 2]}, c[3];
          apply(&frames[r][l], p, c);
          cnt[5]++;
          if (margin_sphere_sphere(c, s->s_xyzr[4 * g + 3], od, o[3]) < 0) {
            hit = 1;
            if (stop_at_hit) return 1;
          }
        }
      }
      for (int k = 0; k < s->n_env_boxes; ++k) {
        const float *b = s->env_b + 6 * k;
        cnt[3]++;
        if (margin_sphere_box(cw[r][l], cw[r][l][3], b) >= 0) continue;
        for (int i = 0; i < s->ns[r]; ++i) {
          int g = s->s_off[r] + i;
          if (s->s_link[g] != l) continue;
          double p[3] = {s->s_xyzr[4 * g], s->s_xyzr[4 * g + 1], s->s_xyzr[4 * g + 2]}, c[3];
          apply(&frames[r][l], p, c);
          cnt[6]++;
          if (margin_sphere_box(c, s->s_xyzr[4 * g + 3], b) < 0) {
            hit = 1;
            if (stop_at_hit) return 1;
          }
        }
      }
    }
  }
  for (int i = 0; i < R; ++i)
    for (int j = i + 1; j < R; ++j)
      for (int la = 0; la <= s->nj[i]; ++la) {
        if (cw[i][la][3] < 0) continue;
        for (int lb = 0; lb <= s->nj[j]; ++lb) {
          if (cw[j][lb][3] < 0) continue;
          cnt[4]++;
          if (margin_sphere_sphere(cw[i][la], cw[i][la][3], cw[j][lb], cw[j][lb][3]) >= 0) continue;
          for (int a = 0; a < s->ns[i]; ++a) {
            int ga = s->s_off[i] + a;
            if (s->s_link[ga] != la) continue;
            double pa[3] = {s->s_xyzr[4 * ga], s->s_xyzr[4 * ga + 1], s->s_xyzr[4 * ga + 2]}, ca[3];
            apply(&frames[i][la], pa, ca);
            for (int b = 0; b < s->ns[j]; ++b) {
              int gb = s->s_off[j] + b;
              if (s->s_link[gb] != lb) continue;
              double pb[3] = {s->s_xyzr[4 * gb], s->s_xyzr[4 * gb + 1], s->s_xyzr[4 * gb + 2]}, cb[3];
              apply(&frames[j][lb], pb, cb);
              cnt[7]++;
              if (margin_sphere_sphere(ca, s->s_xyzr[4 * ga + 3], cb, s->s_xyzr[4 * gb + 3]) < 0) {
                hit = 1;
                if (stop_at_hit) return 1;
              }
            }
          }
        }
      }
  return hit;
}

static void fast_range(job_t *J) {
  const orc_scene *s = J->s;
  int D = orc_dof(s), R = s->n_robots;
  double *q = (double *)malloc(sizeof(double) * D);
  double (*coarse)[ORC_MAX_LINKS][4] = malloc(sizeof(*coarse) * R);
  double (*cw)[ORC_MAX_LINKS][4] = malloc(sizeof(*cw) * R);
  mat4 (*frames)[ORC_MAX_LINKS] = malloc(sizeof(*frames) * R);
  for (int r = 0; r < R; ++r) coarse_spheres(s, r, coarse[r]);
  for (int64_t e = J->e0; e < J->e1; ++e) {
    const float *qa = J->qa + e * D, *qb = J->qb + e * D;
    int n = J->nstates_opt ? J->nstates_opt[e] : orc_edge_nstates(qa, qb, D, J->res);
    int valid = 1;
    for (int k = 0; k < n; ++k) {
      edge_state(qa, qb, D, n, k, q);
      J->counts[0]++;
      if (state_collides_fast(s, q, coarse, frames, cw, J->counts, J->early_exit)) {
        valid = 0;
        if (J->early_exit) break;
      }
    }
    if (!valid) J->counts[8]++;
    if (J->out_n) J->out_n[e] = n;
    J->out_valid[e] = (uint8_t)valid;
  }
  free(q);
  free(coarse);
  free(cw);
  free(frames);
}

static void *job_main(void *p) {
  job_t *J = (job_t *)p;
  if (J->mode == 0) classify_range(J); else fast_range(J);
  return NULL;
}

static void run_jobs(job_t proto, int64_t n_edges, int nthreads, int64_t *counts_out) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > n_edges) nthreads = (int)(n_edges > 0 ? n_edges : 1);
  job_t *jobs = (job_t *)calloc(nthreads, sizeof(job_t));
  int64_t *cnts = (int64_t *)calloc((size_t)nthreads * ORC_NCOUNT, sizeof(int64_t));
  pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
  for (int t = 0; t < nthreads; ++t) {
    jobs[t] = proto;
    jobs[t].e0 = n_edges * t / nthreads;
    jobs[t].e1 = n_edges * (t + 1) / nthreads;
    jobs[t].counts = cnts + (size_t)t * ORC_NCOUNT;
    if (nthreads > 1) pthread_create(&th[t], NULL, job_main, &jobs[t]);
  }
  if (nthreads == 1) job_main(&jobs[0]);
  else for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  if (counts_out)
    for (int t = 0; t < nthreads; ++t)
      for (int c = 0; c < ORC_NCOUNT; ++c) counts_out[c] += cnts[(size_t)t * ORC_NCOUNT + c];
  free(jobs);
  free(cnts);
  free(th);
}

/* Per edge: number of states and minimum margin over all pairs and states. */
void orc_classify_edges(const orc_scene *s, const float *qa, const float *qb, int64_t n_edges, float res,
                        const int32_t *nstates_opt, int32_t *out_n, double *out_m, int nthreads) {
  job_t J;
  memset(&J, 0, sizeof J);
  J.s = s; J.qa = qa; J.qb = qb; J.res = res; J.nstates_opt = nstates_opt;
  J.out_n = out_n; J.out_m = out_m; J.mode = 0;
  run_jobs(J, n_edges, nthreads, NULL);
}

/* Per edge valid bit (1 = free) from the coarse-to-fine checker; counts
 * (ORC_NCOUNT int64, accumulated) give the work done. */
void orc_validate_fast(const orc_scene *s, const float *qa, const float *qb, int64_t n_edges, float res,
                       const int32_t *nstates_opt, uint8_t *out_valid, int32_t *out_n, int64_t *counts,
                       int early_exit, int nthreads) {
  job_t J;
  memset(&J, 0, sizeof J);
  J.s = s; J.qa = qa; J.qb = qb; J.res = res; J.nstates_opt = nstates_opt;
  J.out_valid = out_valid; J.out_n = out_n; J.early_exit = early_exit; J.mode = 1;
  run_jobs(J, n_edges, nthreads, counts);
}

/* Minimum margin of single composite states (n_cfg x D floats). */
void orc_state_margins(const orc_scene *s, const float *q, int64_t n_cfg, double *out_m) {
  int D = orc_dof(s), S = orc_total_spheres(s);
  double *qd = (double *)malloc(sizeof(double) * D);
  double *w = (double *)malloc(sizeof(double) * 4 * (S > 0 ? S : 1));
  for (int64_t c = 0; c < n_cfg; ++c) {
    for (int j = 0; j < D; ++j) qd[j] = q[c * D + j];
    all_world_spheres(s, qd, w);
    out_m[c] = state_min_margin(s, w);
  }
  free(qd);
  free(w);
}

/* ------------------------------------------------------------------------ */
/* NEAREST (Alg. 2): cost-bounded nearest vertex                             */
/* ------------------------------------------------------------------------ */

/* V: [N][D] vertex configurations, g: [N] cost-to-come.  Among vertices with
 * g_v + ||q - q_v|| < c, return the one of least distance; equal distances go
 * to the lower cost (the paper's rule for vertices at one configuration), then
 * to the lower index.  Returns -1 when no vertex is admissible. */
int64_t orc_nearest(const float *V, const float *g, int64_t N, int D, const float *q, double c,
                    double *out_dist) {
  int64_t best = -1;
  double bd = INFINITY, bg = INFINITY;
  for (int64_t v = 0; v < N; ++v) {
    double d2 = 0.0;
    for (int j = 0; j < D; ++j) {
      double t = (double)q[j] - (double)V[v * D + j];
      d2 += t * t;
    }
    double d = sqrt(d2);
    if (!((double)g[v] + d < c)) continue;
    if (d < bd || (d == bd && ((double)g[v] < bg || ((double)g[v] == bg && v < best)))) {
      best = v; bd = d; bg = g[v];
    }
  }
  if (out_dist) *out_dist = bd;
  return best;
}

void orc_nearest_batch(const float *V, const float *g, int64_t N, int D, const float *Q, const double *c,
                       int64_t M, int64_t *out_idx) {
  for (int64_t i = 0; i < M; ++i) out_idx[i] = orc_nearest(V, g, N, D, Q + i * D, c[i], NULL);
}

/* ------------------------------------------------------------------------ */
/* Counter-based random stream (SplitMix64, Steele, Lea and Flood 2014)      */
/* ------------------------------------------------------------------------ */

#define ORC_GAMMA 0x9E3779B97F4A7C15ULL

uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Stream key from a seed and three 64-bit labels. */
uint64_t orc_key(uint64_t seed, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t k = orc_mix64(seed + ORC_GAMMA * (a + 1));
  k = orc_mix64(k + ORC_GAMMA * (b + 1));
  return orc_mix64(k + ORC_GAMMA * (c + 1));
}

/* i-th uniform of a stream: top 24 bits of the i-th SplitMix64 output,
 * scaled to [0, 1) (exact in single precision). */
double orc_u01(uint64_t key, uint64_t i) {
  uint64_t z = orc_mix64(key + ORC_GAMMA * (i + 1));
  return (double)(z >> 40) * (1.0 / 16777216.0);
}

void orc_u01_batch(uint64_t key, int64_t n, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = orc_u01(key, (uint64_t)i);
}

/* ------------------------------------------------------------------------ */
/* Informed sample (Alg. 2, INFORMED_SAMPLE; Gammell et al. 2014)            */
/* ------------------------------------------------------------------------ */

/* Uniform point in the unit D-ball from stream `key`: D standard normals by
 * the Box-Muller transform of uniform pairs (2i, 2i+1), normalised, scaled by
 * u^(1/D) with u the stream's uniform number 2*ceil(D/2). */
void orc_unit_ball(uint64_t key, int D, double *x) {
  int pairs = (D + 1) / 2;
  double n2 = 0.0;
  for (int p = 0; p < pairs; ++p) {
    double u1 = 1.0 - orc_u01(key, 2 * p), u2 = orc_u01(key, 2 * p + 1);
    double rad = sqrt(-2.0 * log(u1)), ang = 2.0 * M_PI * u2;
    x[2 * p] = rad * cos(ang);
    if (2 * p + 1 < D) x[2 * p + 1] = rad * sin(ang);
  }
  for (int j = 0; j < D; ++j) n2 += x[j] * x[j];
  double u = orc_u01(key, 2 * pairs);
  double scale = pow(u, 1.0 / D) / sqrt(n2);
  for (int j = 0; j < D; ++j) x[j] *= scale;
}

/* Map a unit-ball point x into the prolate hyperspheroid with foci qs, qg and
 * transverse diameter c_best: q = centre + H L x, where L scales axis 1 by
 * c_best/2 and the rest by sqrt(c_best^2 - c_min^2)/2, and H is the
 * reflection taking e_1 to (qg - qs)/c_min (any orthogonal map with that
 * property gives the same set, since the other semi-axes are equal). */
void orc_ellipsoid_map(int D, const float *qs, const float *qg, double c_best, const double *x, double *q) {
  double cmin2 = 0.0;
  for (int j = 0; j < D; ++j) {
    double d = (double)qg[j] - (double)qs[j];
    cmin2 += d * d;
  }
  double cmin = sqrt(cmin2);
  double r1 = 0.5 * c_best;
  double rr = c_best * c_best - cmin2;
  double r2 = rr > 0 ? 0.5 * sqrt(rr) : 0.0;
  double *y = (double *)malloc(sizeof(double) * D);
  for (int j = 0; j < D; ++j) y[j] = x[j] * (j == 0 ? r1 : r2);
  /* reflection H = I - 2 v v^T / (v^T v), v = e_1 - a_1 */
  double *v = (double *)malloc(sizeof(double) * D);
  double vv = 0.0, vy = 0.0;
  for (int j = 0; j < D; ++j) {
    double a = cmin > 0 ? ((double)qg[j] - (double)qs[j]) / cmin : (j == 0 ? 1.0 : 0.0);
    v[j] = (j == 0 ? 1.0 : 0.0) - a;
    vv += v[j] * v[j];
    vy += v[j] * y[j];
  }
  for (int j = 0; j < D; ++j) {
    double hy = vv > 1e-300 ? y[j] - 2.0 * v[j] * vy / vv : y[j];
    q[j] = 0.5 * ((double)qs[j] + (double)qg[j]) + hy;
  }
  free(y);
  free(v);
}
