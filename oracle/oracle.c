/*
 * FP64 CPU oracle of the coupled immersed-boundary lattice-Boltzmann timestep
 * of Tan, Sinno & Diamond, "A parallel fluid solid coupling model using LAMMPS
 * and Palabos based on the immersed boundary method" (arXiv:1704.04551).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no source with the GPU library: every table, constant and formula
 * below is written out here on its own.
 *
 * What it computes (all in double precision, plain loops):
 *   Sec. 2.1  D3Q19 lattice-BGK with the forcing term of Eq. (4):
 *             Eq. (1) evolution, Eq. (2) equilibrium, Eq. (3) moments with the
 *             half-force shift, Eq. (5) tau-viscosity relation.
 *   Sec. 2.2  membrane forces: linear springs 1/2 ks (l - l0)^2 per edge and the
 *             dihedral bending energy of Eq. (8), F = -dE/dX; optionally the
 *             rest of the paper's membrane energy, Eq. (6): the WLC-POW
 *             stretching energy of Eq. (7), the global and local area
 *             constraints of Eq. (9) and the volume constraint of Eq. (10).
 *   Sec. 2.3  Eq. (14) velocity interpolation, Eq. (15) force spreading, with
 *             the cosine kernel of Eq. (16) or Peskin's 4-point kernel.
 *
 * Readings taken where the paper is silent (each is also listed in the design
 * notes of the repository):
 *   - step order: forces at X^n -> spread -> moments (u^n includes g^n/2) ->
 *     interpolate u^n at X^n -> X^{n+1} = X^n + U -> collide -> stream;
 *   - walls: a wall axis has solid layers at index 0 and n-1; halfway
 *     bounce-back with the moving-wall term -6 w_i rho_w (c_i . u_w), rho_w = 1;
 *   - spreading drops shares that land on solid cells; interpolation reads the
 *     wall velocity at solid cells;
 *   - node positions are kept unwrapped; stencil cells wrap on periodic axes;
 *   - bending angle: signed angle between the outward normals of the two
 *     triangles sharing an edge, positive where the surface is convex.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Loops over cells (nodes) run in parallel only above these sizes: a small
 * case gains nothing from threads and loses much when a core is busy. */
#define OMP_MIN_CELLS 32768
#define OMP_MIN_NODES 2048

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the parallel loops from now on (n >= 1); returns the number
 * the loops will use (1 without OpenMP). */
int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* D3Q19 velocity set: one rest velocity, 6 face and 12 edge neighbours.     */
/* Weights 1/3, 1/18, 1/36 (textbook D3Q19, the lattice named in Sec. 2.1).  */
/* ------------------------------------------------------------------------ */
static const int OC[19][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double ow(int i) {
  int s = abs(OC[i][0]) + abs(OC[i][1]) + abs(OC[i][2]);
  if (s == 0) return 1.0 / 3.0;
  if (s == 1) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

static int oopp(int i) {
  for (int j = 0; j < 19; ++j)
    if (OC[j][0] == -OC[i][0] && OC[j][1] == -OC[i][1] && OC[j][2] == -OC[i][2])
      return j;
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Discrete delta kernels, Sec. 2.3.                                         */
/* ------------------------------------------------------------------------ */
enum { ODELTA_COS = 0, ODELTA_PESKIN4 = 1 };

/* One-dimensional kernel phi(r). kind 0: Eq. (16), 1/4 (1 + cos(pi r / 2)) for
 * |r| <= 2.  kind 1: Peskin's 4-point kernel (Peskin 2002, cited in Sec. 2.3):
 * (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8 for |r| <= 1,
 * (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8 for 1 <= |r| <= 2. */
double oracle_phi(int kind, double r) {
  double a = fabs(r);
  if (a > 2.0) return 0.0;
  if (kind == ODELTA_COS) return 0.25 * (1.0 + cos(M_PI * r / 2.0));
  if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
  {
    double q = -7.0 + 12.0 * a - 4.0 * a * a;
    if (q < 0.0) q = 0.0; /* a == 2 exactly gives q = 0; guard rounding */
    return (5.0 - 2.0 * a - sqrt(q)) / 8.0;
  }
}

/* ------------------------------------------------------------------------ */
/* Membrane template: topology from outward (counter-clockwise) triangles.   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int nn, nt, ne;
  int *tri;      /* [nt][3] */
  int *ev;       /* [ne][4]: v0, v1, v2, v3 ; shared edge v1-v2,
                    v0 opposite in the triangle holding v1->v2,
                    v3 opposite in the triangle holding v2->v1 */
  double *l0;    /* [ne] rest length */
  double *th0;   /* [ne] rest bending angle */
  double *a0;    /* [nt] rest triangle area (A_j0 of Eq. (9)) */
  double A0, V0; /* rest total area and enclosed volume (Eqs. (9), (10)) */
} otmpl;

static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Build the edge list.  Every directed edge of a closed, consistently
 * oriented manifold appears in exactly one triangle, and its reverse in
 * exactly one other.  Returns 0, or -1 for a mesh that is not such a surface. */
static int tmpl_build(otmpl *T, int nn, int nt, const int *tri) {
  T->nn = nn;
  T->nt = nt;
  T->tri = (int *)malloc(sizeof(int) * 3 * (size_t)nt);
  memcpy(T->tri, tri, sizeof(int) * 3 * (size_t)nt);
  /* directed-edge table: for each triangle side (p->q), the opposite vertex */
  int nd = 3 * nt;
  int *dp = (int *)malloc(sizeof(int) * nd), *dq = (int *)malloc(sizeof(int) * nd),
      *dr = (int *)malloc(sizeof(int) * nd);
  for (int t = 0; t < nt; ++t)
    for (int s = 0; s < 3; ++s) {
      int p = tri[3 * t + s], q = tri[3 * t + (s + 1) % 3], r = tri[3 * t + (s + 2) % 3];
      if (p < 0 || p >= nn || q < 0 || q >= nn || r < 0 || r >= nn || p == q || q == r || p == r) {
        free(dp); free(dq); free(dr);
        return -1;
      }
      dp[3 * t + s] = p; dq[3 * t + s] = q; dr[3 * t + s] = r;
    }
  /* each undirected edge once, taken from its directed copy with p < q */
  T->ne = 0;
  T->ev = (int *)malloc(sizeof(int) * 4 * (size_t)nd);
  int ok = 0;
  for (int a = 0; a < nd; ++a) {
    /* count copies of a's direction and of its reverse */
    int same = 0, rev = -1, nrev = 0;
    for (int b = 0; b < nd; ++b) {
      if (dp[b] == dp[a] && dq[b] == dq[a]) ++same;
      if (dp[b] == dq[a] && dq[b] == dp[a]) { rev = b; ++nrev; }
    }
    if (same != 1 || nrev != 1) { ok = -1; break; }
    if (dp[a] < dq[a]) {
      int *e = T->ev + 4 * T->ne;
      e[0] = dr[a];    /* v0: opposite vertex of the triangle with v1->v2 */
      e[1] = dp[a];    /* v1 */
      e[2] = dq[a];    /* v2 */
      e[3] = dr[rev];  /* v3: opposite vertex of the triangle with v2->v1 */
      T->ne++;
    }
  }
  free(dp); free(dq); free(dr);
  if (ok != 0) return -1;
  T->l0 = (double *)calloc((size_t)T->ne, sizeof(double));
  T->th0 = (double *)calloc((size_t)T->ne, sizeof(double));
  T->a0 = (double *)calloc((size_t)T->nt, sizeof(double));
  return 0;
}

/* Signed angle between the outward normals of the two triangles of an edge
 * (Eq. (8) uses the angle formed by the two outward surface normals).
 * nA = (v2 - v1) x (v0 - v1), nB = (v1 - v2) x (v3 - v2); the sign is that of
 * (nA x nB) . (v2 - v1): positive where the surface bends outward (convex). */
static double dihedral_angle(const double *v0, const double *v1, const double *v2,
                             const double *v3) {
  double e[3], a[3], b[3], nA[3], nB[3], m[3];
  for (int k = 0; k < 3; ++k) {
    e[k] = v2[k] - v1[k];
    a[k] = v0[k] - v1[k];
    b[k] = v3[k] - v2[k];
  }
  double me[3] = {-e[0], -e[1], -e[2]};
  cross3(e, a, nA);
  cross3(me, b, nB);
  cross3(nA, nB, m);
  double le = sqrt(dot3(e, e));
  double s = dot3(m, e) / le;  /* |nA||nB| sin(theta) */
  double c = dot3(nA, nB);     /* |nA||nB| cos(theta) */
  return atan2(s, c);
}

/* ------------------------------------------------------------------------ */
/* Membrane energy and force, Sec. 2.2.                                      */
/*   E = sum_edges 1/2 ks (l - l0)^2 + sum_edges kb (1 - cos(theta - theta0)) */
/*   F_k = -dE/dX_k.                                                          */
/* The bending gradient uses the closed form of the dihedral-angle gradient:  */
/* with e = v2 - v1, L = |e|, nA, nB as above:                                */
/*   dtheta/dv0 = -L nA / |nA|^2,  dtheta/dv3 = -L nB / |nB|^2,               */
/*   dtheta/dv1 = -(1 - t0) dtheta/dv0 - (1 - t3) dtheta/dv3,                 */
/*   dtheta/dv2 = -t0 dtheta/dv0 - t3 dtheta/dv3,                             */
/* where t0 = (v0 - v1).e / L^2 and t3 = (v3 - v1).e / L^2.                   */
/* ------------------------------------------------------------------------ */
static double tri_area(const double *p1, const double *p2, const double *p3);
static double tri_volume(const double *p1, const double *p2, const double *p3, const double *c);

static void tmpl_rest(otmpl *T, const double *xr) {
  for (int j = 0; j < T->ne; ++j) {
    const int *e = T->ev + 4 * j;
    const double *v0 = xr + 3 * e[0], *v1 = xr + 3 * e[1], *v2 = xr + 3 * e[2],
                 *v3 = xr + 3 * e[3];
    double d[3] = {v2[0] - v1[0], v2[1] - v1[1], v2[2] - v1[2]};
    T->l0[j] = sqrt(dot3(d, d));
    T->th0[j] = dihedral_angle(v0, v1, v2, v3);
  }
  T->A0 = 0.0;
  T->V0 = 0.0;
  for (int t = 0; t < T->nt; ++t) {
    const int *q = T->tri + 3 * t;
    T->a0[t] = tri_area(xr + 3 * q[0], xr + 3 * q[1], xr + 3 * q[2]);
    T->A0 += T->a0[t];
    T->V0 += tri_volume(xr + 3 * q[0], xr + 3 * q[1], xr + 3 * q[2], xr);
  }
}

/* Adds the membrane force of one mesh to F (both [nn][3]); returns energy. */
static double membrane_force(const otmpl *T, const double *x, double ks, double kb, double *F) {
  double E = 0.0;
  for (int j = 0; j < T->ne; ++j) {
    const int *ev = T->ev + 4 * j;
    const double *v0 = x + 3 * ev[0], *v1 = x + 3 * ev[1], *v2 = x + 3 * ev[2],
                 *v3 = x + 3 * ev[3];
    /* spring on edge v1-v2 */
    double d[3] = {v2[0] - v1[0], v2[1] - v1[1], v2[2] - v1[2]};
    double l = sqrt(dot3(d, d));
    double dl = l - T->l0[j];
    E += 0.5 * ks * dl * dl;
    for (int k = 0; k < 3; ++k) {
      double fk = ks * dl * d[k] / l;  /* dE/dv2 = ks dl d/l ; force on v2 = -that */
      F[3 * ev[1] + k] += fk;
      F[3 * ev[2] + k] -= fk;
    }
    /* dihedral bending on the same edge */
    if (kb != 0.0) {
      double th = dihedral_angle(v0, v1, v2, v3);
      E += kb * (1.0 - cos(th - T->th0[j]));
      double dEdth = kb * sin(th - T->th0[j]);
      double e[3], a[3], b[3], nA[3], nB[3];
      for (int k = 0; k < 3; ++k) {
        e[k] = v2[k] - v1[k];
        a[k] = v0[k] - v1[k];
        b[k] = v3[k] - v2[k];
      }
      double me[3] = {-e[0], -e[1], -e[2]};
      cross3(e, a, nA);
      cross3(me, b, nB);
      double L2 = dot3(e, e), L = sqrt(L2);
      double nA2 = dot3(nA, nA), nB2 = dot3(nB, nB);
      double t0 = dot3(a, e) / L2;
      double v3v1[3] = {v3[0] - v1[0], v3[1] - v1[1], v3[2] - v1[2]};
      double t3 = dot3(v3v1, e) / L2;
      for (int k = 0; k < 3; ++k) {
        double g0 = -L * nA[k] / nA2;
        double g3 = -L * nB[k] / nB2;
        double g1 = -(1.0 - t0) * g0 - (1.0 - t3) * g3;
        double g2 = -t0 * g0 - t3 * g3;
        F[3 * ev[0] + k] -= dEdth * g0;
        F[3 * ev[1] + k] -= dEdth * g1;
        F[3 * ev[2] + k] -= dEdth * g2;
        F[3 * ev[3] + k] -= dEdth * g3;
      }
    }
  }
  return E;
}

/* ------------------------------------------------------------------------ */
/* The rest of the membrane energy of Eq. (6), Sec. 2.2.                     */
/*                                                                            */
/* Stretching, Eq. (7), per edge with x = l / l_m, l_m = 2 l0 (the maximum     */
/* bond length is twice the equilibrium one), C = kBT / p:                    */
/*   U = C l_m / 4 (3 x^2 - 2 x^3) / (1 - x) + k_p / l,                       */
/*   dU/dl = C (1 / (4 (1 - x)^2) - 1/4 + x) - k_p / l^2.                     */
/* k_p makes each bond force-free at its rest length (x = 1/2), the paper's   */
/* rule for fixing it: C (1 - 1/4 + 1/2) = k_p / l0^2, k_p = 5/4 C l0^2.       */
/*                                                                            */
/* Area, Eq. (9): U = kg (A - A0)^2 / (2 A0) + sum_j kl (A_j - A_j0)^2 /      */
/* (2 A_j0), A_j = |(p2 - p1) x (p3 - p1)| / 2, A = sum_j A_j; with n the      */
/* unit normal of a counter-clockwise triangle, dA_j/dp1 = n x (p3 - p2) / 2   */
/* and cyclically.                                                            */
/*                                                                            */
/* Volume, Eq. (10): U = kv (V - V0)^2 / (2 V0), V = sum_j (p1 - c) .          */
/* ((p2 - c) x (p3 - c)) / 6 over the outward triangles, for any fixed point   */
/* c (the closed surface makes the sum independent of it; c = the mesh's       */
/* first node keeps the terms small); dV/dp1 = (p2 - c) x (p3 - c) / 6 and     */
/* cyclically.                                                                */
/* ------------------------------------------------------------------------ */
static double tri_area(const double *p1, const double *p2, const double *p3) {
  double a[3], b[3], n[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = p2[k] - p1[k];
    b[k] = p3[k] - p1[k];
  }
  cross3(a, b, n);
  return 0.5 * sqrt(dot3(n, n));
}

static double tri_volume(const double *p1, const double *p2, const double *p3, const double *c) {
  double a[3], b[3], d[3], n[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = p1[k] - c[k];
    b[k] = p2[k] - c[k];
    d[k] = p3[k] - c[k];
  }
  cross3(b, d, n);
  return dot3(a, n) / 6.0;
}

/* Adds the force of the terms above to F; returns their energy.  A bond at or
 * beyond its maximum length has no finite energy: returns NAN. */
static double membrane_extra(const otmpl *T, const double *x, double kbtp, double kg, double kl,
                             double kv, double *F) {
  double E = 0.0;
  if (kbtp != 0.0) {
    for (int j = 0; j < T->ne; ++j) {
      const int *ev = T->ev + 4 * j;
      const double *v1 = x + 3 * ev[1], *v2 = x + 3 * ev[2];
      double d[3] = {v2[0] - v1[0], v2[1] - v1[1], v2[2] - v1[2]};
      double l = sqrt(dot3(d, d));
      double lm = 2.0 * T->l0[j];
      double xr = l / lm;
      if (!(xr < 1.0)) return NAN;
      double kp = 1.25 * kbtp * T->l0[j] * T->l0[j];
      E += kbtp * lm / 4.0 * (3.0 * xr * xr - 2.0 * xr * xr * xr) / (1.0 - xr) + kp / l;
      double dUdl = kbtp * (1.0 / (4.0 * (1.0 - xr) * (1.0 - xr)) - 0.25 + xr) - kp / (l * l);
      for (int k = 0; k < 3; ++k) {
        double fk = dUdl * d[k] / l;  /* dU/dv2; the force on v2 is minus that */
        F[3 * ev[1] + k] += fk;
        F[3 * ev[2] + k] -= fk;
      }
    }
  }
  if (kg != 0.0 || kl != 0.0 || kv != 0.0) {
    double A = 0.0, V = 0.0;
    for (int t = 0; t < T->nt; ++t) {
      const int *q = T->tri + 3 * t;
      A += tri_area(x + 3 * q[0], x + 3 * q[1], x + 3 * q[2]);
      V += tri_volume(x + 3 * q[0], x + 3 * q[1], x + 3 * q[2], x);
    }
    E += kg * (A - T->A0) * (A - T->A0) / (2.0 * T->A0) + kv * (V - T->V0) * (V - T->V0) / (2.0 * T->V0);
    double cg = kg * (A - T->A0) / T->A0, cv = kv * (V - T->V0) / T->V0;
    for (int t = 0; t < T->nt; ++t) {
      const int *q = T->tri + 3 * t;
      const double *p[3] = {x + 3 * q[0], x + 3 * q[1], x + 3 * q[2]};
      double At = tri_area(p[0], p[1], p[2]);
      E += kl * (At - T->a0[t]) * (At - T->a0[t]) / (2.0 * T->a0[t]);
      double ca = cg + kl * (At - T->a0[t]) / T->a0[t];
      double a[3], b[3], nrm[3];
      for (int k = 0; k < 3; ++k) {
        a[k] = p[1][k] - p[0][k];
        b[k] = p[2][k] - p[0][k];
      }
      cross3(a, b, nrm);
      double nl = sqrt(dot3(nrm, nrm));
      for (int k = 0; k < 3; ++k) nrm[k] /= nl;
      for (int i = 0; i < 3; ++i) {
        const double *pn = p[(i + 1) % 3], *pp = p[(i + 2) % 3];
        double opp[3] = {pp[0] - pn[0], pp[1] - pn[1], pp[2] - pn[2]}, gA[3];
        cross3(nrm, opp, gA);  /* 2 dA_t/dp_i */
        double r1[3], r2[3], gV[3];
        for (int k = 0; k < 3; ++k) {
          r1[k] = pn[k] - x[k];
          r2[k] = pp[k] - x[k];
        }
        cross3(r1, r2, gV);  /* 6 dV_t/dp_i */
        for (int k = 0; k < 3; ++k) F[3 * q[i] + k] -= ca * 0.5 * gA[k] + cv * gV[k] / 6.0;
      }
    }
  }
  return E;
}

static void tmpl_free(otmpl *T) {
  free(T->tri); free(T->ev); free(T->l0); free(T->th0); free(T->a0);
  memset(T, 0, sizeof(*T));
}

/* Stand-alone membrane force for pinning tests: topology from tris, rest
 * state from xref, force and energy at x.  Returns #edges, or -1 on a bad mesh. */
int oracle_membrane(int nn, int nt, const int *tri, const double *xref, const double *x,
                    double ks, double kb, double *F, double *E) {
  otmpl T;
  memset(&T, 0, sizeof(T));
  if (tmpl_build(&T, nn, nt, tri) != 0) { tmpl_free(&T); return -1; }
  tmpl_rest(&T, xref);
  memset(F, 0, sizeof(double) * 3 * (size_t)nn);
  double e = membrane_force(&T, x, ks, kb, F);
  if (E) *E = e;
  int ne = T.ne;
  tmpl_free(&T);
  return ne;
}

/* The same with the rest of Eq. (6): WLC-POW stretching (kbtp = kBT / p),
 * global / local area (kg, kl) and volume (kv) constraints.  Returns #edges,
 * -1 on a bad mesh, -2 where a bond reaches its maximum length. */
int oracle_membrane_full(int nn, int nt, const int *tri, const double *xref, const double *x,
                         double ks, double kb, double kbtp, double kg, double kl, double kv,
                         double *F, double *E) {
  otmpl T;
  memset(&T, 0, sizeof(T));
  if (tmpl_build(&T, nn, nt, tri) != 0) { tmpl_free(&T); return -1; }
  tmpl_rest(&T, xref);
  memset(F, 0, sizeof(double) * 3 * (size_t)nn);
  double e = membrane_force(&T, x, ks, kb, F);
  double e2 = membrane_extra(&T, x, kbtp, kg, kl, kv, F);
  if (E) *E = e + e2;
  int ne = T.ne;
  tmpl_free(&T);
  return isnan(e2) ? -2 : ne;
}

/* Rest area, per-triangle rest areas and rest volume of a template (tests). */
int oracle_template_rest(int nn, int nt, const int *tri, const double *xref, double *a0,
                         double *A0, double *V0) {
  otmpl T;
  memset(&T, 0, sizeof(T));
  if (tmpl_build(&T, nn, nt, tri) != 0) { tmpl_free(&T); return -1; }
  tmpl_rest(&T, xref);
  if (a0) memcpy(a0, T.a0, sizeof(double) * (size_t)nt);
  *A0 = T.A0;
  *V0 = T.V0;
  tmpl_free(&T);
  return 0;
}

/* Edge list and rest data (v0,v1,v2,v3 per edge, l0, theta0) for tests. */
int oracle_mesh_edges(int nn, int nt, const int *tri, const double *xref, int *ev_out,
                      double *l0_out, double *th0_out) {
  otmpl T;
  memset(&T, 0, sizeof(T));
  if (tmpl_build(&T, nn, nt, tri) != 0) { tmpl_free(&T); return -1; }
  tmpl_rest(&T, xref);
  if (ev_out) memcpy(ev_out, T.ev, sizeof(int) * 4 * (size_t)T.ne);
  if (l0_out) memcpy(l0_out, T.l0, sizeof(double) * (size_t)T.ne);
  if (th0_out) memcpy(th0_out, T.th0, sizeof(double) * (size_t)T.ne);
  int ne = T.ne;
  tmpl_free(&T);
  return ne;
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry.                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n[3];
  int wall[3];           /* 1: solid layers at 0 and n-1 on this axis */
  double ulo[3][3];      /* velocity of the wall layer at index 0, per axis */
  double uhi[3][3];      /* velocity of the wall layer at index n-1, per axis */
} ogeom;

static long cidx(const ogeom *G, int x, int y, int z) {
  return (long)x + (long)G->n[0] * ((long)y + (long)G->n[1] * (long)z);
}

static int wrapi(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

/* Is cell (x,y,z) (already inside the array) solid?  If so, its velocity. */
static int solid_at(const ogeom *G, const int c[3], double uw[3]) {
  for (int a = 0; a < 3; ++a) {
    if (!G->wall[a]) continue;
    if (c[a] == 0 || c[a] == G->n[a] - 1) {
      const double *v = (c[a] == 0) ? G->ulo[a] : G->uhi[a];
      if (uw) { uw[0] = v[0]; uw[1] = v[1]; uw[2] = v[2]; }
      return 1;
    }
  }
  return 0;
}

/* Stencil of a node on one axis: base floor(X) - 1 ... floor(X) + 2 (four
 * points; the kernel vanishes at distance 2).  On a wall axis a node must lie
 * in [1, n-2) so that every stencil cell is inside the array.  Returns 0, or
 * -1 for a node outside that range. */
static int stencil_axis(const ogeom *G, int a, double X, int cell[4], double r[4]) {
  double fb = floor(X);
  long b = (long)fb;
  if (G->wall[a]) {
    if (!(X >= 1.0 && X < (double)(G->n[a] - 2))) return -1;
  }
  for (int s = 0; s < 4; ++s) {
    long c = b - 1 + s;
    r[s] = (double)c - X;
    cell[s] = G->wall[a] ? (int)c : wrapi((int)(c % G->n[a]), G->n[a]);
  }
  return 0;
}

/* Eq. (15): g(x) += sum_k F_k delta(x - X_k), delta = phi phi phi (Eq. (16)).
 * Nodes are visited in ascending order; shares on solid cells are dropped.
 * g is [3][ncell].  Returns 0, or -1 if a node is outside the admissible range.
 * (The four one-dimensional kernel values of each axis are evaluated once per
 * node; the product for a stencil point is formed as phi_x phi_y phi_z.) */
static int spread(const ogeom *G, int kind, int nn, const double *X, const double *F, double *g) {
  long nc = (long)G->n[0] * G->n[1] * G->n[2];
  for (int k = 0; k < nn; ++k) {
    int cx[4], cy[4], cz[4];
    double rx[4], ry[4], rz[4], px[4], py[4], pz[4];
    if (stencil_axis(G, 0, X[3 * k + 0], cx, rx) || stencil_axis(G, 1, X[3 * k + 1], cy, ry) ||
        stencil_axis(G, 2, X[3 * k + 2], cz, rz))
      return -1;
    for (int i = 0; i < 4; ++i) {
      px[i] = oracle_phi(kind, rx[i]);
      py[i] = oracle_phi(kind, ry[i]);
      pz[i] = oracle_phi(kind, rz[i]);
    }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        for (int l = 0; l < 4; ++l) {
          int c[3] = {cx[i], cy[j], cz[l]};
          if (solid_at(G, c, NULL)) continue;
          double w = px[i] * py[j] * pz[l];
          long id = cidx(G, c[0], c[1], c[2]);
          for (int a = 0; a < 3; ++a) g[a * nc + id] += w * F[3 * k + a];
        }
  }
  return 0;
}

/* Eq. (14): U_k = sum_x u(x) delta(x - X_k); a solid stencil cell contributes
 * its wall velocity.  u is [3][ncell]; U is [nn][3].  Each node's sum is
 * formed by one thread in a fixed order, so the node loop runs in parallel. */
static int interp(const ogeom *G, int kind, int nn, const double *X, const double *u, double *U) {
  long nc = (long)G->n[0] * G->n[1] * G->n[2];
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad) if (nn >= OMP_MIN_NODES)
  for (int k = 0; k < nn; ++k) {
    int cx[4], cy[4], cz[4];
    double rx[4], ry[4], rz[4], px[4], py[4], pz[4];
    if (stencil_axis(G, 0, X[3 * k + 0], cx, rx) || stencil_axis(G, 1, X[3 * k + 1], cy, ry) ||
        stencil_axis(G, 2, X[3 * k + 2], cz, rz)) {
      bad = 1;
      continue;
    }
    for (int i = 0; i < 4; ++i) {
      px[i] = oracle_phi(kind, rx[i]);
      py[i] = oracle_phi(kind, ry[i]);
      pz[i] = oracle_phi(kind, rz[i]);
    }
    double s[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        for (int l = 0; l < 4; ++l) {
          int c[3] = {cx[i], cy[j], cz[l]};
          double w = px[i] * py[j] * pz[l];
          double uw[3];
          if (solid_at(G, c, uw)) {
            for (int a = 0; a < 3; ++a) s[a] += w * uw[a];
          } else {
            long id = cidx(G, c[0], c[1], c[2]);
            for (int a = 0; a < 3; ++a) s[a] += w * u[a * nc + id];
          }
        }
    for (int a = 0; a < 3; ++a) U[3 * k + a] = s[a];
  }
  return bad ? -1 : 0;
}

static void geom_set(ogeom *G, const int n[3], const int wall[3], const double *ulo,
                     const double *uhi) {
  for (int a = 0; a < 3; ++a) {
    G->n[a] = n[a];
    G->wall[a] = wall ? wall[a] : 0;
    for (int b = 0; b < 3; ++b) {
      G->ulo[a][b] = ulo ? ulo[3 * a + b] : 0.0;
      G->uhi[a][b] = uhi ? uhi[3 * a + b] : 0.0;
    }
  }
}

/* Stand-alone spreading onto a box (for adjointness and brute-force pins). */
int oracle_spread_field(const int n[3], const int wall[3], int kind, int nn, const double *X,
                        const double *F, double *g) {
  ogeom G;
  geom_set(&G, n, wall, NULL, NULL);
  memset(g, 0, sizeof(double) * 3 * (size_t)n[0] * n[1] * n[2]);
  return spread(&G, kind, nn, X, F, g);
}

/* Stand-alone interpolation from a given velocity field. */
int oracle_interp_field(const int n[3], const int wall[3], const double *ulo, const double *uhi,
                        int kind, int nn, const double *X, const double *u, double *U) {
  ogeom G;
  geom_set(&G, n, wall, ulo, uhi);
  return interp(&G, kind, nn, X, u, U);
}

/* ------------------------------------------------------------------------ */
/* The coupled simulation.                                                   */
/* ------------------------------------------------------------------------ */
typedef struct { int tmpl, off, nn; double ks, kb, kbtp, kg, kl, kv; } omesh;

/* A rigid body (Sec. 2.3, Eq. (17)): a closed surface moved rigidly.  Node k
 * sits at X_k = xc + R(q) r_k.  State: centre of mass xc, orientation q (unit
 * quaternion w, x, y, z), velocity v, angular momentum L (lab frame). */
typedef struct {
  int tmpl, off, nn;
  double *r;           /* [nn][3] node positions about the centre of mass, body frame */
  double *dv;          /* [nn] node weights: a third of the incident triangles' areas
                          times one lattice spacing */
  double M, Ib[9], Ibinv[9];  /* mass, body-frame inertia tensor and its inverse */
  double xc[3], q[4], v[3], L[3];
  double force[3], torque[3];  /* hydrodynamic force and torque of the last evaluation */
} obody;

typedef struct osim {
  ogeom G;
  long nc;
  double tau, gb[3];
  int kind;
  double *f, *fn;       /* [19][nc] populations (post-streaming, pre-collision) */
  double *g;            /* [3][nc] spread IB force density */
  double *rho, *u;      /* moments of the current step */
  unsigned char *solid; /* [nc] */
  int ntm, nme, nnode, cap_nodes;
  otmpl *tm;
  omesh *me;
  int nbo;
  obody *bo;
  double *ustar;        /* [nnode][3] fluid velocity without the IB force at the nodes (bodies) */
  double *ufree;        /* [3][nc] that velocity field */
  double morse[4];      /* D0, alpha, r0, rc of the inter-object Morse potential (D0 = 0: off) */
  double *X, *F, *U;    /* [nnode][3] */
  long step;
  int err;
  int obs_valid;        /* F, g, rho, u, U hold the observables of the current state */
} osim;

static double feq(int i, double rho, const double u[3]) {
  double cu = OC[i][0] * u[0] + OC[i][1] * u[1] + OC[i][2] * u[2];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  /* Eq. (2) with cs^2 = 1/3 */
  return ow(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

/* init_profile 0: fluid at rest; 1: the linear (Couette) profile between the
 * walls of the single wall axis, wall layers at 0 and n-1, effective walls at
 * 0.5 and n-1.5.  f = f_eq(rho = 1, u0), Sec. 2.1. */
osim *oracle_sim_create(const int n[3], double tau, const double gb[3], const int wall[3],
                        const double *ulo, const double *uhi, int kind, int init_profile) {
  if (tau <= 0.5) return NULL;
  for (int a = 0; a < 3; ++a)
    if (n[a] < 4) return NULL;
  osim *S = (osim *)calloc(1, sizeof(osim));
  geom_set(&S->G, n, wall, ulo, uhi);
  S->nc = (long)n[0] * n[1] * n[2];
  S->tau = tau;
  for (int a = 0; a < 3; ++a) S->gb[a] = gb ? gb[a] : 0.0;
  S->kind = kind;
  S->f = (double *)calloc(19 * (size_t)S->nc, sizeof(double));
  S->fn = (double *)calloc(19 * (size_t)S->nc, sizeof(double));
  S->g = (double *)calloc(3 * (size_t)S->nc, sizeof(double));
  S->rho = (double *)calloc((size_t)S->nc, sizeof(double));
  S->u = (double *)calloc(3 * (size_t)S->nc, sizeof(double));
  S->solid = (unsigned char *)calloc((size_t)S->nc, 1);
  int pa = -1;
  for (int a = 0; a < 3; ++a)
    if (S->G.wall[a]) pa = a;
  for (int z = 0; z < n[2]; ++z)
    for (int y = 0; y < n[1]; ++y)
      for (int x = 0; x < n[0]; ++x) {
        int c[3] = {x, y, z};
        long id = cidx(&S->G, x, y, z);
        S->solid[id] = (unsigned char)solid_at(&S->G, c, NULL);
        double u0[3] = {0.0, 0.0, 0.0};
        if (init_profile == 1 && pa >= 0) {
          double H = (double)(n[pa] - 2);
          double s = ((double)c[pa] - 0.5) / H;
          for (int b = 0; b < 3; ++b) u0[b] = S->G.ulo[pa][b] + (S->G.uhi[pa][b] - S->G.ulo[pa][b]) * s;
        }
        for (int i = 0; i < 19; ++i) S->f[i * S->nc + id] = S->solid[id] ? 0.0 : feq(i, 1.0, u0);
      }
  return S;
}

void oracle_sim_destroy(osim *S) {
  if (!S) return;
  for (int t = 0; t < S->ntm; ++t) tmpl_free(&S->tm[t]);
  free(S->tm); free(S->me);
  free(S->f); free(S->fn); free(S->g); free(S->rho); free(S->u); free(S->solid);
  free(S->X); free(S->F); free(S->U);
  for (int b = 0; b < S->nbo; ++b) { free(S->bo[b].r); free(S->bo[b].dv); }
  free(S->bo); free(S->ustar); free(S->ufree);
  free(S);
}

int oracle_template_add(osim *S, int nn, int nt, const int *tri, const double *xref) {
  S->tm = (otmpl *)realloc(S->tm, sizeof(otmpl) * (size_t)(S->ntm + 1));
  otmpl *T = &S->tm[S->ntm];
  memset(T, 0, sizeof(*T));
  if (tmpl_build(T, nn, nt, tri) != 0) { tmpl_free(T); return -1; }
  tmpl_rest(T, xref);
  S->obs_valid = 0;
  return S->ntm++;
}

int oracle_mesh_add(osim *S, int tmpl, const double *x, double ks, double kb) {
  if (tmpl < 0 || tmpl >= S->ntm) return -1;
  int nn = S->tm[tmpl].nn;
  S->me = (omesh *)realloc(S->me, sizeof(omesh) * (size_t)(S->nme + 1));
  omesh *M = &S->me[S->nme];
  M->tmpl = tmpl; M->off = S->nnode; M->nn = nn; M->ks = ks; M->kb = kb;
  M->kbtp = M->kg = M->kl = M->kv = 0.0;
  S->X = (double *)realloc(S->X, sizeof(double) * 3 * (size_t)(S->nnode + nn));
  S->F = (double *)realloc(S->F, sizeof(double) * 3 * (size_t)(S->nnode + nn));
  S->U = (double *)realloc(S->U, sizeof(double) * 3 * (size_t)(S->nnode + nn));
  S->ustar = (double *)realloc(S->ustar, sizeof(double) * 3 * (size_t)(S->nnode + nn));
  memcpy(S->X + 3 * (size_t)S->nnode, x, sizeof(double) * 3 * (size_t)nn);
  memset(S->F + 3 * (size_t)S->nnode, 0, sizeof(double) * 3 * (size_t)nn);
  memset(S->U + 3 * (size_t)S->nnode, 0, sizeof(double) * 3 * (size_t)nn);
  S->nnode += nn;
  S->obs_valid = 0;
  return S->nme++;
}

/* The rest of the paper's membrane energy on one mesh (zero: absent). */
int oracle_mesh_membrane(osim *S, int mesh, double kbtp, double kg, double kl, double kv) {
  if (mesh < 0 || mesh >= S->nme) return -1;
  omesh *M = &S->me[mesh];
  M->kbtp = kbtp; M->kg = kg; M->kl = kl; M->kv = kv;
  S->obs_valid = 0;
  return 0;
}

static int observe(osim *S);

/* ------------------------------------------------------------------------ */
/* Inter-object repulsion, Eq. (13) (Sec. 2.2): a Morse potential between    */
/* nodes of different capsules,                                              */
/*   U(r) = D0 [exp(-2 alpha (r - r0)) - 2 exp(-alpha (r - r0))],  r < rc,   */
/* F on node i from node j = -dU/dr (X_i - X_j) / r                          */
/*                         = 2 alpha D0 [exp(-2 alpha (r - r0))              */
/*                                       - exp(-alpha (r - r0))] (X_i - X_j) / r. */
/* The distance is the minimum image on periodic axes.  Every pair i < j of  */
/* nodes of different meshes is visited once, in ascending (i, j), and its   */
/* force added to both nodes with opposite signs.  Returns the energy.       */
/* ------------------------------------------------------------------------ */
static double morse_pairs(const ogeom *G, int np, const double *X, const int *obj, const double prm[4],
                          double *F) {
  const double D0 = prm[0], al = prm[1], r0 = prm[2], rc = prm[3];
  double E = 0.0;
  for (int i = 0; i < np; ++i)
    for (int j = i + 1; j < np; ++j) {
      if (obj[i] == obj[j]) continue;
      double d[3];
      for (int a = 0; a < 3; ++a) {
        d[a] = X[3 * i + a] - X[3 * j + a];
        if (!G->wall[a]) d[a] -= G->n[a] * floor(d[a] / G->n[a] + 0.5);
      }
      double r = sqrt(dot3(d, d));
      if (!(r < rc) || r == 0.0) continue;
      double e1 = exp(-al * (r - r0)), e2 = e1 * e1;
      E += D0 * (e2 - 2.0 * e1);
      double f = 2.0 * al * D0 * (e2 - e1) / r;
      for (int a = 0; a < 3; ++a) {
        F[3 * i + a] += f * d[a];
        F[3 * j + a] -= f * d[a];
      }
    }
  return E;
}

/* Stand-alone Morse forces and energy of np nodes (object index per node) in
 * a box n with the given walls: F [np][3] (overwritten). */
double oracle_morse(const int n[3], const int wall[3], int np, const double *X, const int *obj,
                    const double prm[4], double *F) {
  ogeom G;
  geom_set(&G, n, wall, NULL, NULL);
  memset(F, 0, sizeof(double) * 3 * (size_t)np);
  return morse_pairs(&G, np, X, obj, prm, F);
}

/* Set the Morse parameters of a simulation (D0 = 0 turns it off).  It acts
 * between the nodes of different capsules; rigid bodies do not take part. */
void oracle_sim_morse(osim *S, double D0, double alpha, double r0, double rc) {
  S->morse[0] = D0; S->morse[1] = alpha; S->morse[2] = r0; S->morse[3] = rc;
  S->obs_valid = 0;
}

/* Add the Morse forces between capsules to S->F (mesh nodes only). */
static void morse_forces(osim *S) {
  int np = 0;
  for (int m = 0; m < S->nme; ++m) np += S->me[m].nn;
  double *X = (double *)calloc(3 * (size_t)np + 3, sizeof(double)), *F = (double *)calloc(3 * (size_t)np + 3, sizeof(double));
  int *obj = (int *)calloc((size_t)np + 1, sizeof(int));
  int k = 0;
  for (int m = 0; m < S->nme; ++m)
    for (int i = 0; i < S->me[m].nn; ++i, ++k) {
      memcpy(X + 3 * k, S->X + 3 * ((size_t)S->me[m].off + i), sizeof(double) * 3);
      obj[k] = m;
    }
  morse_pairs(&S->G, np, X, obj, S->morse, F);
  k = 0;
  for (int m = 0; m < S->nme; ++m)
    for (int i = 0; i < S->me[m].nn; ++i, ++k)
      for (int a = 0; a < 3; ++a) S->F[3 * ((size_t)S->me[m].off + i) + a] += F[3 * k + a];
  free(X); free(F); free(obj);
}

/* ------------------------------------------------------------------------ */
/* Rigid bodies (Sec. 2.3, Eq. (17)).                                        */
/*                                                                            */
/* Mass properties of a uniform solid bounded by a closed, outward surface:   */
/* the solid is the union of the tetrahedra (o, p1, p2, p3) over the          */
/* triangles, o any fixed point (signed volumes cancel outside).  Per         */
/* tetrahedron with o at the origin: volume p1 . (p2 x p3) / 6, centroid      */
/* (p1 + p2 + p3) / 4 times that volume, and second moment                    */
/*   int x x^T dV = V_t / 20 (sum_i p_i p_i^T + (sum_i p_i)(sum_i p_i)^T)     */
/* (the canonical tetrahedron's covariance, mapped linearly).  The inertia    */
/* tensor about the centre of mass is density (tr(C) Id - C), C the second    */
/* moment about it.                                                           */
/* ------------------------------------------------------------------------ */
static int mass_props(int nn, int nt, const int *tri, const double *x, double dens, double *M,
                      double c[3], double I[9]) {
  const double *o = x;  /* first node */
  double V = 0.0, cm[3] = {0.0, 0.0, 0.0}, C[9];
  memset(C, 0, sizeof(C));
  for (int t = 0; t < nt; ++t) {
    double p[3][3];
    for (int i = 0; i < 3; ++i) {
      int v = tri[3 * t + i];
      if (v < 0 || v >= nn) return -1;
      for (int a = 0; a < 3; ++a) p[i][a] = x[3 * v + a] - o[a];
    }
    double n[3];
    cross3(p[1], p[2], n);
    double Vt = dot3(p[0], n) / 6.0;
    V += Vt;
    double sp[3];
    for (int a = 0; a < 3; ++a) {
      sp[a] = p[0][a] + p[1][a] + p[2][a];
      cm[a] += Vt * sp[a] / 4.0;
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double pp = p[0][a] * p[0][b] + p[1][a] * p[1][b] + p[2][a] * p[2][b];
        C[3 * a + b] += Vt / 20.0 * (pp + sp[a] * sp[b]);
      }
  }
  if (!(V > 0.0)) return -1;
  for (int a = 0; a < 3; ++a) cm[a] /= V;
  /* second moment about the centre of mass, then the inertia tensor */
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C[3 * a + b] -= V * cm[a] * cm[b];
  double tr = C[0] + C[4] + C[8];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) I[3 * a + b] = dens * ((a == b ? tr : 0.0) - C[3 * a + b]);
  *M = dens * V;
  for (int a = 0; a < 3; ++a) c[a] = o[a] + cm[a];
  return 0;
}

int oracle_mass_properties(int nn, int nt, const int *tri, const double *x, double dens, double *M,
                           double *c, double *I) {
  return mass_props(nn, nt, tri, x, dens, M, c, I);
}

static int inv3(const double *A, double *B) {
  double d = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
             A[2] * (A[3] * A[7] - A[4] * A[6]);
  if (!(fabs(d) > 0.0)) return -1;
  B[0] = (A[4] * A[8] - A[5] * A[7]) / d;
  B[1] = (A[2] * A[7] - A[1] * A[8]) / d;
  B[2] = (A[1] * A[5] - A[2] * A[4]) / d;
  B[3] = (A[5] * A[6] - A[3] * A[8]) / d;
  B[4] = (A[0] * A[8] - A[2] * A[6]) / d;
  B[5] = (A[2] * A[3] - A[0] * A[5]) / d;
  B[6] = (A[3] * A[7] - A[4] * A[6]) / d;
  B[7] = (A[1] * A[6] - A[0] * A[7]) / d;
  B[8] = (A[0] * A[4] - A[1] * A[3]) / d;
  return 0;
}

/* Rotation matrix of the unit quaternion q = (w, x, y, z). */
static void quat_R(const double *q, double *R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
  R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
  R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
}

static void matvec(const double *A, const double *v, double *o) {
  for (int a = 0; a < 3; ++a) o[a] = A[3 * a] * v[0] + A[3 * a + 1] * v[1] + A[3 * a + 2] * v[2];
}

/* Angular velocity from the angular momentum: Omega = R Ib^-1 R^T L. */
static void body_omega(const obody *B, double *w) {
  double R[9], t[3], t2[3];
  quat_R(B->q, R);
  for (int a = 0; a < 3; ++a) t[a] = R[a] * B->L[0] + R[3 + a] * B->L[1] + R[6 + a] * B->L[2];  /* R^T L */
  matvec(B->Ibinv, t, t2);
  matvec(R, t2, w);
}

/* Node positions X_k = xc + R r_k. */
static void body_place(obody *B, double *X) {
  double R[9];
  quat_R(B->q, R);
  for (int k = 0; k < B->nn; ++k) {
    double d[3];
    matvec(R, B->r + 3 * k, d);
    for (int a = 0; a < 3; ++a) X[3 * k + a] = B->xc[a] + d[a];
  }
}

/* Add a rigid body: the template's surface at node positions x (its shape
 * and initial placement), density dens, initial velocity v0 and angular
 * velocity w0.  Returns the body index, or -1. */
int oracle_body_add(osim *S, int tmpl, const double *x, double dens, const double *v0, const double *w0) {
  if (tmpl < 0 || tmpl >= S->ntm || !(dens > 0.0)) return -1;
  const otmpl *T = &S->tm[tmpl];
  int nn = T->nn;
  double M, c[3], I[9];
  if (mass_props(nn, T->nt, T->tri, x, dens, &M, c, I) != 0) return -1;
  S->bo = (obody *)realloc(S->bo, sizeof(obody) * (size_t)(S->nbo + 1));
  obody *B = &S->bo[S->nbo];
  memset(B, 0, sizeof(*B));
  B->tmpl = tmpl; B->off = S->nnode; B->nn = nn; B->M = M;
  memcpy(B->Ib, I, sizeof(I));
  if (inv3(I, B->Ibinv) != 0) return -1;
  B->r = (double *)malloc(sizeof(double) * 3 * (size_t)nn);
  B->dv = (double *)calloc((size_t)nn, sizeof(double));
  for (int k = 0; k < nn; ++k)
    for (int a = 0; a < 3; ++a) B->r[3 * k + a] = x[3 * k + a] - c[a];
  for (int t = 0; t < T->nt; ++t) {
    const int *q = T->tri + 3 * t;
    double At = tri_area(x + 3 * q[0], x + 3 * q[1], x + 3 * q[2]);
    for (int i = 0; i < 3; ++i) B->dv[q[i]] += At / 3.0;  /* times one lattice spacing */
  }
  for (int a = 0; a < 3; ++a) {
    B->xc[a] = c[a];
    B->v[a] = v0 ? v0[a] : 0.0;
  }
  B->q[0] = 1.0; B->q[1] = B->q[2] = B->q[3] = 0.0;
  double w[3] = {w0 ? w0[0] : 0.0, w0 ? w0[1] : 0.0, w0 ? w0[2] : 0.0};
  matvec(B->Ib, w, B->L);  /* R = identity */
  S->X = (double *)realloc(S->X, sizeof(double) * 3 * (size_t)(S->nnode + nn));
  S->F = (double *)realloc(S->F, sizeof(double) * 3 * (size_t)(S->nnode + nn));
  S->U = (double *)realloc(S->U, sizeof(double) * 3 * (size_t)(S->nnode + nn));
  S->ustar = (double *)realloc(S->ustar, sizeof(double) * 3 * (size_t)(S->nnode + nn));
  body_place(B, S->X + 3 * (size_t)S->nnode);
  memset(S->F + 3 * (size_t)S->nnode, 0, sizeof(double) * 3 * (size_t)nn);
  memset(S->U + 3 * (size_t)S->nnode, 0, sizeof(double) * 3 * (size_t)nn);
  S->nnode += nn;
  S->obs_valid = 0;
  return S->nbo++;
}

/* The FSI force of Eq. (17) at every node of every body, at the current
 * state: f_k = rho_f (u(X_k) - U_k) / dt per unit volume, with u the fluid
 * velocity before the immersed-boundary force (moments of the populations
 * with the body force's half shift only, Eq. (3)), interpolated by Eq. (14),
 * and U_k = v + Omega x (X_k - xc) the node's rigid-body velocity; rho_f = 1,
 * dt = 1.  The node carries f_k dv_k; the body receives it and the fluid
 * minus it (written to F, which the spreading takes).  Also the body's total
 * force and torque. */
static int body_forces(osim *S) {
  long nc = S->nc;
  if (!S->ufree) S->ufree = (double *)calloc(3 * (size_t)nc, sizeof(double));
#pragma omp parallel for schedule(static) if (nc >= OMP_MIN_CELLS)
  for (long id = 0; id < nc; ++id) {
    if (S->solid[id]) {
      S->ufree[id] = S->ufree[nc + id] = S->ufree[2 * nc + id] = 0.0;
      continue;
    }
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
      double fi = S->f[i * nc + id];
      rho += fi;
      for (int a = 0; a < 3; ++a) j[a] += fi * OC[i][a];
    }
    for (int a = 0; a < 3; ++a) S->ufree[a * nc + id] = (j[a] + 0.5 * S->gb[a]) / rho;
  }
  for (int b = 0; b < S->nbo; ++b) {
    obody *B = &S->bo[b];
    double *X = S->X + 3 * (size_t)B->off, *us = S->ustar + 3 * (size_t)B->off;
    if (interp(&S->G, S->kind, B->nn, X, S->ufree, us) != 0) return -1;
    double w[3];
    body_omega(B, w);
    for (int a = 0; a < 3; ++a) B->force[a] = B->torque[a] = 0.0;
    for (int k = 0; k < B->nn; ++k) {
      double r[3], wr[3], f[3];
      for (int a = 0; a < 3; ++a) r[a] = X[3 * k + a] - B->xc[a];
      cross3(w, r, wr);
      for (int a = 0; a < 3; ++a) {
        f[a] = B->dv[k] * (us[3 * k + a] - (B->v[a] + wr[a]));  /* on the body */
        S->F[3 * ((size_t)B->off + k) + a] = -f[a];              /* on the fluid */
        B->force[a] += f[a];
      }
      double rf[3];
      cross3(r, f, rf);
      for (int a = 0; a < 3; ++a) B->torque[a] += rf[a];
    }
  }
  return 0;
}

/* Newton's second law for each body, with the force and torque of this step
 * (semi-implicit Euler, dt = 1): v += F / M, L += T, xc += v; the orientation
 * turns by the angle |Omega| about Omega, Omega = R Ib^-1 R^T L at the start
 * of the step's orientation; the nodes are placed at the new pose. */
static void body_advance(osim *S) {
  for (int b = 0; b < S->nbo; ++b) {
    obody *B = &S->bo[b];
    for (int a = 0; a < 3; ++a) {
      B->v[a] += B->force[a] / B->M;
      B->L[a] += B->torque[a];
      B->xc[a] += B->v[a];
    }
    double w[3];
    body_omega(B, w);
    double th = sqrt(dot3(w, w));
    if (th > 0.0) {
      double s = sin(0.5 * th) / th, dq[4] = {cos(0.5 * th), w[0] * s, w[1] * s, w[2] * s}, q[4];
      const double *p = B->q;
      q[0] = dq[0] * p[0] - dq[1] * p[1] - dq[2] * p[2] - dq[3] * p[3];
      q[1] = dq[0] * p[1] + dq[1] * p[0] + dq[2] * p[3] - dq[3] * p[2];
      q[2] = dq[0] * p[2] - dq[1] * p[3] + dq[2] * p[0] + dq[3] * p[1];
      q[3] = dq[0] * p[3] + dq[1] * p[2] - dq[2] * p[1] + dq[3] * p[0];
      double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      for (int a = 0; a < 4; ++a) B->q[a] = q[a] / nq;
    }
    body_place(B, S->X + 3 * (size_t)B->off);
  }
}

/* Body state: centre of mass, orientation (w, x, y, z), velocity, angular
 * velocity, and the hydrodynamic force and torque at the current state. */
int oracle_body_state(osim *S, int body, double *xc, double *q, double *v, double *w, double *force,
                      double *torque) {
  if (body < 0 || body >= S->nbo) return -1;
  if (observe(S) != 0) return -1;
  obody *B = &S->bo[body];
  for (int a = 0; a < 3; ++a) {
    if (xc) xc[a] = B->xc[a];
    if (v) v[a] = B->v[a];
    if (force) force[a] = B->force[a];
    if (torque) torque[a] = B->torque[a];
  }
  if (q) memcpy(q, B->q, sizeof(B->q));
  if (w) body_omega(B, w);
  return 0;
}

/* Node positions, rigid-body velocities and FSI forces on the fluid of one
 * body, each [nn][3]. */
int oracle_body_nodes(osim *S, int body, double *X, double *U, double *F) {
  if (body < 0 || body >= S->nbo) return -1;
  if (observe(S) != 0) return -1;
  obody *B = &S->bo[body];
  double w[3];
  body_omega(B, w);
  for (int k = 0; k < B->nn; ++k) {
    const double *x = S->X + 3 * ((size_t)B->off + k);
    double r[3], wr[3];
    for (int a = 0; a < 3; ++a) r[a] = x[a] - B->xc[a];
    cross3(w, r, wr);
    for (int a = 0; a < 3; ++a) {
      if (X) X[3 * k + a] = x[a];
      if (U) U[3 * k + a] = B->v[a] + wr[a];
      if (F) F[3 * k + a] = S->F[3 * ((size_t)B->off + k) + a];
    }
  }
  return B->nn;
}

/* Steps 1-4 of a timestep at the current state (no mutation of f or X):
 * membrane forces F(X^n), spread g^n, moments rho^n, u^n (Eq. (3) with the
 * total force g_body + g^n), interpolated node velocities U^n. */
static int observe(osim *S) {
  if (S->obs_valid) return 0;  /* state unchanged since the last evaluation */
  long nc = S->nc;
  memset(S->F, 0, sizeof(double) * 3 * (size_t)S->nnode);
  int bad = 0;
  /* meshes are independent (each writes its own nodes' forces) */
#pragma omp parallel for schedule(dynamic) reduction(|| : bad) if (S->nme > 1)
  for (int m = 0; m < S->nme; ++m) {
    const omesh *M = &S->me[m];
    membrane_force(&S->tm[M->tmpl], S->X + 3 * (size_t)M->off, M->ks, M->kb, S->F + 3 * (size_t)M->off);
    if (isnan(membrane_extra(&S->tm[M->tmpl], S->X + 3 * (size_t)M->off, M->kbtp, M->kg, M->kl, M->kv,
                             S->F + 3 * (size_t)M->off)))
      bad = 1;
  }
  if (bad) return -1;
  if (S->morse[0] != 0.0) morse_forces(S);
  if (S->nbo && body_forces(S) != 0) return -1;
  memset(S->g, 0, sizeof(double) * 3 * (size_t)nc);
  if (spread(&S->G, S->kind, S->nnode, S->X, S->F, S->g) != 0) return -1;
#pragma omp parallel for schedule(static) if (nc >= OMP_MIN_CELLS)
  for (long id = 0; id < nc; ++id) {
    if (S->solid[id]) {
      S->rho[id] = 0.0;
      S->u[id] = S->u[nc + id] = S->u[2 * nc + id] = 0.0;
      continue;
    }
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
      double fi = S->f[i * nc + id];
      rho += fi;
      for (int a = 0; a < 3; ++a) j[a] += fi * OC[i][a];
    }
    S->rho[id] = rho;
    for (int a = 0; a < 3; ++a) S->u[a * nc + id] = (j[a] + 0.5 * (S->gb[a] + S->g[a * nc + id])) / rho;
  }
  if (interp(&S->G, S->kind, S->nnode, S->X, S->u, S->U) != 0) return -1;
  S->obs_valid = 1;
  return 0;
}

/* One timestep, in the order documented at the top of this file. */
static int step1(osim *S) {
  if (observe(S) != 0) return -1;
  long nc = S->nc;
  const int *n = S->G.n;
  /* node update X^{n+1} = X^n + U^n (unit time step) of the deformable
   * meshes; rigid bodies follow Newton's law with this step's force */
  for (int m = 0; m < S->nme; ++m) {
    const omesh *M = &S->me[m];
    for (long k = 3L * M->off; k < 3L * (M->off + M->nn); ++k) S->X[k] += S->U[k];
  }
  body_advance(S);
  S->obs_valid = 0;
  double om = 1.0 / S->tau, pre = 1.0 - 0.5 / S->tau;
#pragma omp parallel for schedule(static) if (nc >= OMP_MIN_CELLS)
  for (int z = 0; z < n[2]; ++z)
    for (int y = 0; y < n[1]; ++y)
      for (int x = 0; x < n[0]; ++x) {
        long id = cidx(&S->G, x, y, z);
        if (S->solid[id]) continue;
        double rho = S->rho[id];
        double u[3] = {S->u[id], S->u[nc + id], S->u[2 * nc + id]};
        double g[3];
        for (int a = 0; a < 3; ++a) g[a] = S->gb[a] + S->g[a * nc + id];
        double ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
        for (int i = 0; i < 19; ++i) {
          double fi = S->f[i * nc + id];
          double cu = OC[i][0] * u[0] + OC[i][1] * u[1] + OC[i][2] * u[2];
          double cg = OC[i][0] * g[0] + OC[i][1] * g[1] + OC[i][2] * g[2];
          /* Eq. (4): (1 - 1/(2 tau)) w_i [ (c_i - u)/cs^2 + (c_i.u) c_i / cs^4 ] . g */
          double Fi = pre * ow(i) * (3.0 * (cg - ug) + 9.0 * cu * cg);
          /* Eq. (1): BGK relaxation plus forcing */
          double fs = fi - om * (fi - feq(i, rho, u)) + Fi;
          /* streaming with periodic wrap and halfway bounce-back */
          int c[3] = {x + OC[i][0], y + OC[i][1], z + OC[i][2]};
          for (int a = 0; a < 3; ++a)
            if (!S->G.wall[a]) c[a] = wrapi(c[a], n[a]);
          double uw[3];
          if (solid_at(&S->G, c, uw)) {
            double cuw = OC[i][0] * uw[0] + OC[i][1] * uw[1] + OC[i][2] * uw[2];
            S->fn[oopp(i) * nc + id] = fs - 6.0 * ow(i) * 1.0 * cuw;
          } else {
            S->fn[i * nc + cidx(&S->G, c[0], c[1], c[2])] = fs;
          }
        }
      }
  double *t = S->f; S->f = S->fn; S->fn = t;
  S->step++;
  S->obs_valid = 0;
  return 0;
}

int oracle_sim_step(osim *S, long nsteps) {
  for (long s = 0; s < nsteps; ++s)
    if (step1(S) != 0) { S->err = 1; return -1; }
  return 0;
}

/* Observables at the current time N: rho, u (fluid cells; 0 at solid cells),
 * g = g_body + spread IB force (fluid cells), each [ncell] / [3][ncell]. */
int oracle_sim_observe(osim *S, double *rho, double *u, double *g) {
  if (observe(S) != 0) return -1;
  long nc = S->nc;
  if (rho) memcpy(rho, S->rho, sizeof(double) * (size_t)nc);
  if (u) memcpy(u, S->u, sizeof(double) * 3 * (size_t)nc);
  if (g)
    for (long id = 0; id < nc; ++id)
      for (int a = 0; a < 3; ++a) g[a * nc + id] = S->solid[id] ? 0.0 : S->gb[a] + S->g[a * nc + id];
  return 0;
}

/* Node state of one mesh at time N: X^N, U^N (interpolated with the force at
 * X^N) and F^N, each [nn][3]. */
int oracle_sim_nodes(osim *S, int mesh, double *X, double *U, double *F) {
  if (mesh < 0 || mesh >= S->nme) return -1;
  if (observe(S) != 0) return -1;
  const omesh *M = &S->me[mesh];
  size_t o = 3 * (size_t)M->off, c = sizeof(double) * 3 * (size_t)M->nn;
  if (X) memcpy(X, S->X + o, c);
  if (U) memcpy(U, S->U + o, c);
  if (F) memcpy(F, S->F + o, c);
  return M->nn;
}

/* Mass sum_fluid sum_i f_i and momentum sum_fluid sum_i f_i c_i of the
 * stored populations. */
void oracle_sim_conservation(osim *S, double *mass, double mom[3]) {
  double m = 0.0, p[3] = {0.0, 0.0, 0.0};
  for (long id = 0; id < S->nc; ++id) {
    if (S->solid[id]) continue;
    for (int i = 0; i < 19; ++i) {
      double fi = S->f[i * S->nc + id];
      m += fi;
      for (int a = 0; a < 3; ++a) p[a] += fi * OC[i][a];
    }
  }
  *mass = m;
  for (int a = 0; a < 3; ++a) mom[a] = p[a];
}

/* Raw populations [19][ncell] in this file's velocity order (tests only). */
void oracle_sim_populations(osim *S, double *f) {
  memcpy(f, S->f, sizeof(double) * 19 * (size_t)S->nc);
}

/* Velocity set as used here, for tests that pin it. */
void oracle_velocity_set(int *c, double *w) {
  for (int i = 0; i < 19; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = OC[i][a];
    w[i] = ow(i);
  }
}

long oracle_sim_stepcount(osim *S) { return S->step; }
int oracle_sim_nnodes(osim *S) { return S->nnode; }
