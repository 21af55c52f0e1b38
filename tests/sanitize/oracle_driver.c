/*
 * Drives every entry point of the oracle on small random inputs, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitize.py).
 * Two seven-joint arms with one sphere per link, spheres and boxes around
 * them, random edges, trees and queries; single- and multi-threaded checkers.
 * Exits non-zero on a failed sanity condition; the sanitizers abort on any
 * finding.
 */
#include "../../oracle/mrpop_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x1234567ULL;
static double urand(void) { /* xorshift64*, uniform in [0, 1) */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 2685821657736338717ULL) >> 11) * (1.0 / 9007199254740992.0);
}

#define R 2
#define NJ 7
#define NS 8
#define D (R * NJ)

int main(void) {
  static const float dh_row[NJ][4] = {{0, 0.333f, 0, 0},       {0, 0, -1.5708f, 0},       {0, 0.316f, 1.5708f, 0},
                                      {0.0825f, 0, 1.5708f, 0}, {-0.0825f, 0.384f, -1.5708f, 0}, {0, 0, 1.5708f, 0},
                                      {0.088f, 0, 1.5708f, 0}};
  int32_t nj[R] = {NJ, NJ}, q_off[R] = {0, NJ}, ns[R] = {NS, NS}, s_off[R] = {0, NS};
  float dh[R * NJ * 4], base[R * 12], s_xyzr[R * NS * 4];
  int32_t s_link[R * NS];
  for (int r = 0; r < R; ++r) {
    for (int j = 0; j < NJ; ++j)
      for (int k = 0; k < 4; ++k) dh[(r * NJ + j) * 4 + k] = dh_row[j][k];
    for (int k = 0; k < 12; ++k) base[r * 12 + k] = 0.f;
    base[r * 12 + 0] = base[r * 12 + 5] = base[r * 12 + 10] = 1.f;
    base[r * 12 + 3] = r == 0 ? -0.5f : 0.5f;
    for (int i = 0; i < NS; ++i) {
      s_link[r * NS + i] = i;
      s_xyzr[(r * NS + i) * 4 + 0] = 0.f;
      s_xyzr[(r * NS + i) * 4 + 1] = 0.f;
      s_xyzr[(r * NS + i) * 4 + 2] = 0.02f * i;
      s_xyzr[(r * NS + i) * 4 + 3] = 0.08f - 0.005f * i;
    }
  }
  float env_s[4 * 4] = {0.0f, 0.4f, 0.5f, 0.1f, 0.3f, -0.3f, 0.8f, 0.12f,
                        -0.4f, 0.2f, 1.0f, 0.08f, 0.0f, 0.0f, 1.4f, 0.1f};
  float env_b[3 * 6] = {-0.2f, 0.5f, 0.0f, 0.2f, 0.7f, 0.3f, 0.4f, 0.4f, 0.2f, 0.6f, 0.6f, 0.5f,
                        -0.1f, -0.8f, 0.9f, 0.1f, -0.6f, 1.1f};
  orc_scene s = {R, nj, q_off, dh, base, ns, s_off, s_link, s_xyzr, 4, env_s, 3, env_b};
  if (orc_dof(&s) != D || orc_total_spheres(&s) != R * NS) return 2;

  enum { E = 96 };
  float qa[E * D], qb[E * D];
  for (int e = 0; e < E; ++e)
    for (int j = 0; j < D; ++j) {
      qa[e * D + j] = (float)(urand() * 5.0 - 2.5);
      qb[e * D + j] = e % 7 == 0 ? qa[e * D + j] : (float)(qa[e * D + j] + urand() * 0.8 - 0.4);
    }
  double *fk = (double *)malloc(sizeof(double) * E * R * NS * 4);
  orc_fk_spheres(&s, qa, E, fk);
  int32_t n[E], n2[E], nexp[E];
  double m[E], sm[E];
  orc_classify_edges(&s, qa, qb, E, 0.05f, NULL, n, m, 3);
  for (int e = 0; e < E; ++e) nexp[e] = 1 + e % 5;
  orc_classify_edges(&s, qa, qb, E, 0.05f, nexp, n2, m, 2);
  for (int e = 0; e < E; ++e)
    if (n2[e] != nexp[e] || n[e] != orc_edge_nstates(qa + e * D, qb + e * D, D, 0.05f)) return 3;
  uint8_t v1[E], v2[E];
  int64_t counts[16] = {0};
  orc_validate_fast(&s, qa, qb, E, 0.05f, NULL, v1, n2, counts, 1, 1);
  orc_validate_fast(&s, qa, qb, E, 0.05f, NULL, v2, n2, counts, 0, 4);
  orc_classify_edges(&s, qa, qb, E, 0.05f, NULL, n, m, 1);
  for (int e = 0; e < E; ++e) {
    if (v1[e] != v2[e]) return 4;
    if (m[e] > 1e-9 && !v1[e]) return 5;
    if (m[e] < -1e-9 && v1[e]) return 6;
  }
  orc_validate_fast(&s, qa, qb, 0, 0.05f, NULL, v1, n2, counts, 1, 2); /* empty batch */
  orc_state_margins(&s, qa, E, sm);

  enum { N = 200, M = 40 };
  float V[N * D], g[N], Q[M * D];
  double c[M];
  int64_t idx[M];
  for (int i = 0; i < N * D; ++i) V[i] = (float)(urand() * 4 - 2);
  for (int i = 0; i < N; ++i) g[i] = (float)(urand() * 3);
  for (int i = 0; i < M * D; ++i) Q[i] = (float)(urand() * 4 - 2);
  for (int i = 0; i < M; ++i) c[i] = i % 4 == 0 ? INFINITY : urand() * 12;
  orc_nearest_batch(V, g, N, D, Q, c, M, idx);
  for (int i = 0; i < M; ++i)
    if (idx[i] < -1 || idx[i] >= N) return 7;
  if (orc_nearest(V, g, 0, D, Q, INFINITY, NULL) != -1) return 8;

  double u[64], x[D], q[D];
  orc_u01_batch(orc_key(1, 2, 3, 4), 64, u);
  for (int i = 0; i < 64; ++i)
    if (!(u[i] >= 0 && u[i] < 1)) return 9;
  float qs[D], qg[D];
  for (int j = 0; j < D; ++j) {
    qs[j] = (float)(urand() - 0.5);
    qg[j] = (float)(urand() - 0.5);
  }
  for (int t = 0; t < 20; ++t) {
    orc_unit_ball(orc_key(5, 6, t, 7), D, x);
    orc_ellipsoid_map(D, qs, qg, 3.0, x, q);
  }
  orc_ellipsoid_map(D, qs, qs, 1.0, x, q); /* coincident foci */
  free(fk);
  printf("oracle driver ok: %d edges, %d free\n", E, (int)(v1[0] + v1[1]));
  return 0;
}
