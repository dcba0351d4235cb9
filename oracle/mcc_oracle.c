/*
 * mcc_oracle.c -- CPU FP64 oracle for the weighted, moment-preserving
 * binary-pairing Monte-Carlo Coulomb collision step of
 *   J. R. Angus, Y. Fu, V. Geyko, D. Grote, D. Larson,
 *   "Moment-preserving Monte-Carlo Coulomb collision method for particle codes".
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, sequential, obviously-correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or helper with the GPU path.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never does.
 *
 * Precision: IEEE FP64 throughout, built with -ffp-contract=off, glibc libm.
 *
 * What it computes (one time step, cell by cell, collision by collision; the
 * paper's Algorithm 1 in the paper's order):
 *   1. snapshot of the before-scatter velocities (Alg. 1, first step);
 *   2. random binary pairs (Fig. 1; Sec. 3.2 pairing; odd intra-species rule);
 *   3. per pair: normalized scattering length s of Eq. (12), TA77 or N97
 *      centre-of-mass angle, rotation of the relative velocity, update of the
 *      lighter-weight particle and of the heavier one with probability
 *      w_min/w_max (Sec. 3.1-3.2);
 *   4. momentum restore, Eq. (17);
 *   5. energy violation, Eq. (18), inter-species partition, Eq. (24);
 *   6. optional descending-weight sort; zero-angle inelastic pair energy
 *      correction, Eqs. (19)-(23), until the violation is absorbed;
 *   7. failure policy of Sec. 6.2 (reset or keep).
 *  Relativistic variant (Appendix A): proper velocity u = gamma v is stored,
 *  the momentum shift acts on u, and the pair energy correction solves
 *  Eq. (A.5) for alpha of Eqs. (A.3)-(A.4).
 *
 * Readings where the paper is silent (each is listed, with its reason, in the
 * design notes of this repository):
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = {index, cell, step_lo, step_hi16<<16 | collision<<8 | purpose}.
 *   - Random pairs: each species list is ordered by (Philox word, local index).
 *   - N x N pairing (Sec. 3.1, optional): every pair of the collision once,
 *     s of Eq. (10) with w_max / dV.  The pairs are taken over the
 *     shuffled lists in rounds: intra-species, the circle schedule on N
 *     rounded up to even (round r: (r, pad) and ((r+m) mod R, (r-m) mod R),
 *     R = rounds), pairs with the pad skipped; inter-species, round r pairs
 *     list-a entry i with list-b entry (i + r) mod N_max.  Pair index
 *     r * P + slot (P = half the even N, or N_a).
 *   - Duplicity pairing (optional; the variant of Higginson et al. that the
 *     paper describes after Sec. 3.2): the order-N pairs, with an
 *     inter-species pair's s taken with N_max / D in place of N_min, D the
 *     number of pairs its fewer-population particle takes in the step.
 *     Intra-species pairs are unchanged (every particle is paired once).
 *   - Inter-species pair k is (big[k], small[k mod N_min]), written with the
 *     collision's first species first; odd intra-species triple
 *     (L0,L1),(L1,L2),(L2,L0) with s/2, then (L3,L4),(L5,L6),...
 *   - Per-pair uniforms u_m = (a_m + 1/2) 2^-32 from the four words of one
 *     Philox call: u0 -> angle, u1 -> Box-Muller phase (TA77), u2 -> azimuth,
 *     u3 -> acceptance of the heavier particle (accepted iff u3 <= w_min/w_max).
 *   - TA77: tan(Theta/2) ~ Normal(0, s/2).  N97: <cos chi> = exp(-s) with
 *     density proportional to exp(A cos chi); cos chi drawn by inverse CDF.
 *   - Relativistic scatter (paper silent): rotation of the centre-of-momentum
 *     momentum of the pair by the sampled angles, with s from the invariant
 *     collision rate (reduces to Eq. (12) as c -> infinity).
 *   - Hard-sphere process (optional; the non-Coulomb use of the same
 *     weighting and correction that the paper's summary names, with the
 *     collision integral of Sec. 2 for a total cross-section sigma and an
 *     isotropic differential one, I = sigma / 4 pi): the normalized path
 *     length is s = f sigma n_eff |u| dt, n_eff the density factor the
 *     pairing gives Eq. (12) or (10) (w_max N_min / dV, w_max / dV, or
 *     w_max (N_max / D) / dV).  The pair collides with probability
 *     1 - exp(-s) (u0 < 1 - exp(-s)), then 1 - cos chi = 2 u1 (isotropic),
 *     azimuth and acceptance as for the Coulomb methods.  Non-relativistic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_INVALID (-1)
#define ORC_ERR_OOM (-2)

#define ORC_TA77 0
#define ORC_N97 1
#define ORC_HARD_SPHERE 2
#define ORC_ORDER_N 0
#define ORC_NXN 1
#define ORC_DUPLICITY 2

#define PURPOSE_PAIR 0
#define PURPOSE_SHUFFLE0 1 /* + species slot (0: first species, 1: second) */

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11: ten rounds of two 32x32->64 multiplies with the  */
/* published multipliers and Weyl key increments.                            */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

static uint32_t ctr_word3(uint64_t step, int coll, int purpose) {
  return (uint32_t)(((step >> 32) & 0xFFFFu) << 16) |
         ((uint32_t)(coll & 0xFF) << 8) | (uint32_t)(purpose & 0xFF);
}

static void draw4(uint64_t seed, uint32_t c0, uint32_t cell, uint64_t step,
                  int coll, int purpose, uint32_t out[4]) {
  uint32_t ctr[4] = {c0, cell, (uint32_t)step, ctr_word3(step, coll, purpose)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  oracle_philox4x32_10(ctr, key, out);
}

/* uniform in (0,1): (a + 1/2) * 2^-32, exact in FP64 */
static double unif(uint32_t a) { return ((double)a + 0.5) * 0x1p-32; }

/* The FP32-kinematics form's uniform (reading of the design notes): the top
 * 23 bits of the word, (k + 1/2) * 2^-23, which FP32 holds exactly and which
 * never reaches 0 or 1.  The oracle takes it, on request, for the angle, the
 * Box-Muller phase and the azimuth (not for the acceptance, which both forms
 * draw at 32 bits), so that it samples the same angles as that form. */
static double unif23(uint32_t a) { return ((double)(a >> 9) + 0.5) * 0x1p-23; }

/* ------------------------------------------------------------------------ */
/* Random permutation of a species list ("random binary pairs", Fig. 1 and   */
/* Alg. 1): local indices ordered by (Philox word, index).                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t key;
  int32_t idx;
} keyidx;

static int cmp_keyidx(const void *pa, const void *pb) {
  const keyidx *a = (const keyidx *)pa, *b = (const keyidx *)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

static int shuffle_list(int32_t n, uint32_t cell, uint64_t seed, uint64_t step,
                        int coll, int slot, int32_t *out) {
  keyidx *t = (keyidx *)malloc(sizeof(keyidx) * (size_t)(n > 0 ? n : 1));
  if (!t) return ORC_ERR_OOM;
  for (int32_t i = 0; i < n; ++i) {
    uint32_t r[4];
    draw4(seed, (uint32_t)(i >> 2), cell, step, coll, PURPOSE_SHUFFLE0 + slot, r);
    t[i].key = r[i & 3];
    t[i].idx = i;
  }
  qsort(t, (size_t)n, sizeof(keyidx), cmp_keyidx);
  for (int32_t i = 0; i < n; ++i) out[i] = t[i].idx;
  free(t);
  return ORC_OK;
}

void oracle_shuffle(int32_t n, uint32_t cell, uint64_t seed, uint64_t step,
                    int32_t coll, int32_t slot, int32_t *out) {
  shuffle_list(n, cell, seed, step, coll, slot, out);
}

/* ------------------------------------------------------------------------ */
/* N97 angle (Sec. 3.2, last paragraphs: TA77 and N97 differ only in the map */
/* from s to the angle).  Nanbu's cumulative-angle method: cos chi has       */
/* density proportional to exp(A cos chi) on [-1,1] with                      */
/*   <cos chi> = coth A - 1/A = exp(-s).                                      */
/* We solve  M(A) := 1 - (coth A - 1/A) = 1 - exp(-s) =: t  for A >= 0.       */
/* ------------------------------------------------------------------------ */

/* coth A - 1/A via Lambert's continued fraction
 *   coth x = 1/x + x/(3 + x^2/(5 + x^2/(7 + ...)))   (used for small A). */
static double langevin_small(double A) {
  double x2 = A * A, d = 43.0; /* depth 20: 2*21+1 */
  for (int k = 20; k >= 1; --k) d = (2.0 * k + 1.0) + x2 / d;
  return A / d;
}

double oracle_n97_M(double A) { /* 1 - (coth A - 1/A), decreasing from 1 to 0 */
  if (A < 0.5) return 1.0 - langevin_small(A);
  return 1.0 / A - 2.0 / expm1(2.0 * A);
}

/* d/dA (coth A - 1/A) = 1/A^2 - 1/sinh^2 A (only steers Newton below) */
static double langevin_deriv(double A) {
  if (A < 0.5) {
    double x2 = A * A;
    return 1.0 / 3.0 - x2 / 15.0 + 2.0 * x2 * x2 / 189.0 -
           x2 * x2 * x2 / 675.0;
  }
  double sh = sinh(A);
  return 1.0 / (A * A) - 1.0 / (sh * sh);
}

/* coth A - 1/A for any A >= 0 */
double oracle_n97_L(double A) {
  if (A < 0.5) return langevin_small(A);
  return 1.0 + 2.0 / expm1(2.0 * A) - 1.0 / A;
}

/* Root A of coth A - 1/A = exp(-s), by bracketed Newton.  For s <= ln 2 the
 * equation is solved as M(A) = 1 - exp(-s) = -expm1(-s) (A >= ~1.3, where
 * 1 - L carries the information); otherwise as L(A) = exp(-s) (A small).
 * s = 0 gives A = infinity (no scattering); exp(-s) = 0 gives A = 0
 * (isotropic). */
double oracle_n97_A(double s) {
  if (!(s > 0.0)) return INFINITY;
  /* For s > 50, A = 3 e^{-s} (1 + O(A^2)) < 6e-22 and the inverse CDF below
   * equals its isotropic limit 1 - cos chi = 2 u to far below an ulp, while
   * evaluating it would run through subnormal A (e^{-s} < 2.2e-308 for
   * s > 708) and lose all precision: take the limit. */
  if (s > 50.0) return 0.0;
  const double eps = 2.220446049250313e-16;
  const int use_M = (s <= 0.6931471805599453);
  double target, lo = 0.0, hi, A;
  if (use_M) {
    target = -expm1(-s);          /* in (0, 1/2] */
    hi = 1.0 / target;            /* M(1/t) < t because M(A) < 1/A */
    A = hi;
  } else {
    target = exp(-s);             /* in [0, 1/2) */
    if (target == 0.0) return 0.0;
    hi = 1.0 / (1.0 - target);    /* L(A) > 1 - 1/A, so L(hi) > target */
    A = 3.0 * target;             /* small-A start: L ~ A/3 */
    if (A >= hi) A = 0.5 * hi;
  }
  for (int it = 0; it < 400; ++it) {
    /* g(A) increasing in A: g = target - M(A)  or  g = L(A) - target */
    double gval = use_M ? (target - oracle_n97_M(A)) : (oracle_n97_L(A) - target);
    if (gval == 0.0) return A;
    if (gval < 0.0)
      lo = A;
    else
      hi = A;
    if (hi - lo <= 4.0 * eps * hi) break;
    double d = langevin_deriv(A); /* dg/dA in both forms */
    double An = A - gval / d;
    if (!(An > lo && An < hi)) An = 0.5 * (lo + hi);
    if (fabs(An - A) <= 0.5 * eps * A) {
      A = An;
      break;
    }
    A = An;
  }
  return A;
}

/* Sampled angle: returns oc = 1 - cos(Theta) in [0,2] and sin(Theta).
 * TA77: delta = tan(Theta/2) ~ N(0, s/2) by Box-Muller (u0, u1), so that
 *       <Theta^2> = 2 s as in Eq. (6) with s = <Theta^2>/2 of Eq. (9);
 *       sin Theta = 2 delta/(1+delta^2), 1-cos Theta = 2 delta^2/(1+delta^2).
 * N97:  1 - cos chi = -log1p(u0 * expm1(-2A)) / A  (inverse CDF of the
 *       exp(A cos chi) density); A = 0 is isotropic: 1 - cos chi = 2 u0. */
double oracle_sample_angle(int method, double s, double u0, double u1,
                           double *sin_theta) {
  double oc, st;
  if (method == ORC_TA77) {
    double z = sqrt(-2.0 * log(u0)) * cos(2.0 * PI * u1);
    double delta = sqrt(0.5 * s) * z;
    double d2 = delta * delta;
    if (isinf(d2)) {
      oc = 2.0;
      st = 0.0;
    } else {
      double q = 1.0 / (1.0 + d2);
      st = 2.0 * delta * q;
      oc = 2.0 * d2 * q;
    }
  } else {
    double A = oracle_n97_A(s);
    if (isinf(A)) {
      oc = 0.0;
    } else if (A == 0.0) {
      oc = 2.0 * u0;
    } else {
      oc = -log1p(u0 * expm1(-2.0 * A)) / A;
    }
    if (oc < 0.0) oc = 0.0;
    if (oc > 2.0) oc = 2.0;
    st = sqrt(oc * (2.0 - oc));
  }
  *sin_theta = st;
  return oc;
}

/* Rotation of a relative velocity u by polar angle Theta (given as sin Theta
 * and 1 - cos Theta) and azimuth phi about u (TA77's formula); returns the
 * change du so that |u + du| = |u| and (u + du).u = |u|^2 cos Theta. */
void oracle_rotate(const double u[3], double st, double oc, double phi,
                   double du[3]) {
  double up = sqrt(u[0] * u[0] + u[1] * u[1]);
  double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double cp = cos(phi), sp = sin(phi);
  if (up > 0.0) {
    du[0] = (u[0] / up) * u[2] * st * cp - (u[1] / up) * um * st * sp - u[0] * oc;
    du[1] = (u[1] / up) * u[2] * st * cp + (u[0] / up) * um * st * sp - u[1] * oc;
    du[2] = -up * st * cp - u[2] * oc;
  } else {
    du[0] = um * st * cp;
    du[1] = um * st * sp;
    du[2] = -u[2] * oc;
  }
}

/* ------------------------------------------------------------------------ */
/* Step configuration                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_species;
  const double *mass, *charge;
  int32_t n_coll;
  const int32_t *coll_a, *coll_b;
  double dt, lnL, eps0, c;
  uint64_t seed, step;
  int32_t method, rel, corr, sortw, max_passes, keep_on_fail;
  double fE;
  int32_t pairing; /* ORC_ORDER_N, ORC_NXN or ORC_DUPLICITY */
  const double *sigma; /* [n_coll] cross-sections (ORC_HARD_SPHERE only) */
  int32_t unif23;      /* 1: 23-bit uniforms for the angle and azimuth */
} cfg_t;

typedef struct {
  int64_t pairs;      /* binary scatter pairs formed */
  int64_t corr_pairs; /* energy-correction pairs with U != 0 */
  int64_t failed;     /* (cell, collision) energy-correction failures */
  int64_t collisions; /* (cell, collision) applications with pairs */
  double max_rel_dP, max_rel_dE;
} stats_t;

/* Test hook: when set, collide_one records intermediate states of every
 * collision it processes (absolute particle indices).  Single-threaded. */
typedef struct {
  double *vps;  /* [3*n] post-scatter velocities (x block, y block, z block) */
  double *vpm;  /* [3*n] post-momentum-restore velocities */
  double *dE;   /* [n_cells*n_coll] energy violation of Eq. (18) */
  double *dEs;  /* [2*n_cells*n_coll] partition of Eq. (24) */
  int64_t n;
  int32_t n_coll;
} trace_t;
static trace_t *g_trace = NULL;

/* Accept flags for a pair (Sec. 3.1 rejection, Alg. 1 update steps): the
 * lighter-weight particle always moves; the heavier one iff
 * u3 <= w_min/w_max; equal weights move both. */
static void acceptance(double wi, double wj, double u3, int *ai, int *aj) {
  if (wi == wj) {
    *ai = 1;
    *aj = 1;
  } else if (wi < wj) {
    *ai = 1;
    *aj = (u3 <= wi / wj);
  } else {
    *aj = 1;
    *ai = (u3 <= wj / wi);
  }
}

/* Non-relativistic weighted pair scatter, Eq. (12) and Sec. 3.2.
 * f = 1/2 for the three pairs of an odd intra-species triple. */
static void scatter_pair_nr(const cfg_t *g, uint32_t cell, int coll,
                            uint32_t pair_k, double f, double nmin, double dV,
                            double mi, double qi, double mj, double qj,
                            double wi, double wj, double *vi, double *vj) {
  double u[3] = {vi[0] - vj[0], vi[1] - vj[1], vi[2] - vj[2]};
  double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  if (um == 0.0) return;
  double wmax = wi > wj ? wi : wj;
  uint32_t r[4];
  double st, oc;
  if (g->method == ORC_HARD_SPHERE) {
    /* s = f sigma n_eff |u| dt: the expected number of collisions of the
     * pair in the step; at least one happens with probability 1 - e^-s */
    double s = f * g->sigma[coll] * (wmax * nmin / dV) * um * g->dt;
    if (!(s > 0.0)) return;
    draw4(g->seed, pair_k, cell, g->step, coll, PURPOSE_PAIR, r);
    if (!(unif(r[0]) < -expm1(-s))) return;
    oc = 2.0 * unif(r[1]); /* cos chi uniform on (-1, 1) */
    st = sqrt(oc * (2.0 - oc));
  } else {
    double mu = mi * mj / (mi + mj);
    double s = f * (qi * qi * qj * qj * g->lnL) * (wmax * nmin / dV) * g->dt /
               (4.0 * PI * g->eps0 * g->eps0 * mu * mu * um * um * um);
    if (!(s > 0.0)) return;
    draw4(g->seed, pair_k, cell, g->step, coll, PURPOSE_PAIR, r);
    if (g->unif23)
      oc = oracle_sample_angle(g->method, s, unif23(r[0]), unif23(r[1]), &st);
    else
      oc = oracle_sample_angle(g->method, s, unif(r[0]), unif(r[1]), &st);
  }
  double phi = 2.0 * PI * (g->unif23 && g->method != ORC_HARD_SPHERE ? unif23(r[2]) : unif(r[2]));
  double du[3];
  oracle_rotate(u, st, oc, phi, du);
  int ai, aj;
  acceptance(wi, wj, unif(r[3]), &ai, &aj);
  double fi = mj / (mi + mj), fj = mi / (mi + mj);
  if (ai)
    for (int d = 0; d < 3; ++d) vi[d] += fi * du[d];
  if (aj)
    for (int d = 0; d < 3; ++d) vj[d] -= fj * du[d];
}

/* Relativistic pair scatter (the paper gives none; this is the reading used
 * throughout this repository).  Species (unweighted) masses m_i, m_j;
 * proper velocities u = gamma v.  The pair's centre-of-momentum (CM) frame
 * moves with v_CM of Eq. (A.1).  The CM momentum p* is rotated by the sampled
 * angles, and boosted back; the change of p_i is the boost of the CM change.
 * s uses the invariant collision rate n v_Moller and the CM deflection
 * Theta ~ dp_perp / |p*|, dp_perp = 2 q_i q_j / (4 pi eps0 b v_rel):
 *   s = q_i^2 q_j^2 lnL (w_max N_min / dV) dt v_M / (4 pi eps0^2 |p*|^2 v_rel^2)
 * which equals Eq. (12) as c -> infinity. */
static void scatter_pair_rel(const cfg_t *g, uint32_t cell, int coll,
                             uint32_t pair_k, double f, double nmin, double dV,
                             double mi, double qi, double mj, double qj,
                             double wi, double wj, double *ui, double *uj) {
  const double c = g->c, c2 = c * c;
  double du[3] = {ui[0] - uj[0], ui[1] - uj[1], ui[2] - uj[2]};
  double du2 = du[0] * du[0] + du[1] * du[1] + du[2] * du[2];
  if (du2 == 0.0) return;
  double gi = sqrt(1.0 + (ui[0] * ui[0] + ui[1] * ui[1] + ui[2] * ui[2]) / c2);
  double gj = sqrt(1.0 + (uj[0] * uj[0] + uj[1] * uj[1] + uj[2] * uj[2]) / c2);
  double sum[3] = {ui[0] + uj[0], ui[1] + uj[1], ui[2] + uj[2]};
  double dus = du[0] * sum[0] + du[1] * sum[1] + du[2] * sum[2];
  double dgam = dus / (c2 * (gi + gj)); /* gamma_i - gamma_j */
  /* gamma_rel - 1 = (|du|^2/c^2 - (gamma_i - gamma_j)^2) / 2 */
  double gr1 = 0.5 * (du2 / c2 - dgam * dgam);
  if (!(gr1 > 0.0)) return;
  double grel2m1 = gr1 * (gr1 + 2.0); /* gamma_rel^2 - 1 */
  double M = mi + mj;
  double ecm = sqrt(M * M + 2.0 * mi * mj * gr1); /* E_cm / c^2 */
  double etot = mi * gi + mj * gj;                /* E_tot / c^2 */
  double sq = sqrt(grel2m1);
  double pstar = mi * mj * c * sq / ecm;
  double vM = c * sq / (gi * gj);
  double vrel = c * sq / (1.0 + gr1);
  double wmax = wi > wj ? wi : wj;
  double s = f * (qi * qi * qj * qj * g->lnL) * (wmax * nmin / dV) * g->dt * vM /
             (4.0 * PI * g->eps0 * g->eps0 * pstar * pstar * vrel * vrel);
  if (!(s > 0.0)) return;
  /* p_i* = (E_j p_i - E_i p_j)/E_cm + c^2 p_tot x (p_j x p_i)/(E_cm (E_tot+E_cm)) */
  double Q[3], ujxdu[3], ptot[3], ps[3], cr[3];
  for (int d = 0; d < 3; ++d) {
    Q[d] = mi * mj * (gj * du[d] - dgam * uj[d]);
    ptot[d] = mi * ui[d] + mj * uj[d];
  }
  ujxdu[0] = uj[1] * du[2] - uj[2] * du[1];
  ujxdu[1] = uj[2] * du[0] - uj[0] * du[2];
  ujxdu[2] = uj[0] * du[1] - uj[1] * du[0];
  for (int d = 0; d < 3; ++d) ujxdu[d] *= mi * mj; /* p_j x p_i */
  cr[0] = ptot[1] * ujxdu[2] - ptot[2] * ujxdu[1];
  cr[1] = ptot[2] * ujxdu[0] - ptot[0] * ujxdu[2];
  cr[2] = ptot[0] * ujxdu[1] - ptot[1] * ujxdu[0];
  for (int d = 0; d < 3; ++d)
    ps[d] = Q[d] / ecm + cr[d] / (c2 * ecm * (etot + ecm));
  uint32_t r[4];
  draw4(g->seed, pair_k, cell, g->step, coll, PURPOSE_PAIR, r);
  double st;
  double oc = oracle_sample_angle(g->method, s, unif(r[0]), unif(r[1]), &st);
  double phi = 2.0 * PI * unif(r[2]);
  double D[3];
  oracle_rotate(ps, st, oc, phi, D);
  double Dp = D[0] * ptot[0] + D[1] * ptot[1] + D[2] * ptot[2];
  double kb = Dp / (c2 * ecm * (etot + ecm));
  double dp[3];
  for (int d = 0; d < 3; ++d) dp[d] = D[d] + kb * ptot[d];
  int ai, aj;
  acceptance(wi, wj, unif(r[3]), &ai, &aj);
  if (ai)
    for (int d = 0; d < 3; ++d) ui[d] += dp[d] / mi;
  if (aj)
    for (int d = 0; d < 3; ++d) uj[d] -= dp[d] / mj;
}

/* ------------------------------------------------------------------------ */
/* Compensated (Neumaier) summation for the per-cell moment sums.            */
/* ------------------------------------------------------------------------ */
typedef struct {
  double s, c;
} nsum_t;
static void nadd(nsum_t *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static double nval(const nsum_t *a) { return a->s + a->c; }

/* Non-relativistic zero-angle inelastic pair correction, Eqs. (19)-(23):
 * weighted masses m1, m2; the pair's relative kinetic energy K changes by -U
 * with v'_R = v_R sqrt(1 - U/K); (sqrt(1-x) - 1) = -x/(1+sqrt(1-x)). */
void oracle_energy_pair_nr(double m1, double m2, double U, double *v1,
                           double *v2) {
  double mu = m1 * m2 / (m1 + m2);
  double vr[3] = {v1[0] - v2[0], v1[1] - v2[1], v1[2] - v2[2]};
  double K = 0.5 * mu * (vr[0] * vr[0] + vr[1] * vr[1] + vr[2] * vr[2]);
  if (K == 0.0) return;
  double x = U / K;
  double gm = -x / (1.0 + sqrt(1.0 - x));
  for (int d = 0; d < 3; ++d) {
    v1[d] += (mu / m1) * gm * vr[d];
    v2[d] -= (mu / m2) * gm * vr[d];
  }
}

/* Kinetic energy of the pair in its CM frame, relativistic (Appendix A):
 * KE_cm = E_cm - (m1+m2) c^2 with E_cm^2 = (m1+m2)^2 c^4 + 2 m1 m2 c^4
 * (gamma_rel - 1), written without cancellation. */
static double rel_kecm(double m1, double m2, const double *u1, const double *u2,
                       double c) {
  double c2 = c * c;
  double du[3] = {u1[0] - u2[0], u1[1] - u2[1], u1[2] - u2[2]};
  double du2 = du[0] * du[0] + du[1] * du[1] + du[2] * du[2];
  double g1 = sqrt(1.0 + (u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]) / c2);
  double g2 = sqrt(1.0 + (u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]) / c2);
  double dus = du[0] * (u1[0] + u2[0]) + du[1] * (u1[1] + u2[1]) +
               du[2] * (u1[2] + u2[2]);
  double dg = dus / (c2 * (g1 + g2));
  double gr1 = 0.5 * (du2 / c2 - dg * dg);
  if (gr1 < 0.0) gr1 = 0.0;
  double M = m1 + m2;
  double ecm = sqrt(M * M + 2.0 * m1 * m2 * gr1);
  return 2.0 * m1 * m2 * c2 * gr1 / (ecm + M);
}

/* h(alpha) = E1(alpha) + E2(alpha) - E1 - E2 + U, Eq. (A.5) rearranged
 * without rest-mass cancellation; p1' = p1 + alpha du, p2' = p2 - alpha du. */
static double rel_h(double m1, double m2, const double *p1, const double *p2,
                    const double *du, double E1, double E2, double c2,
                    double U, double alpha, double *dh) {
  double a1[3], a2[3];
  for (int d = 0; d < 3; ++d) {
    a1[d] = p1[d] + alpha * du[d];
    a2[d] = p2[d] - alpha * du[d];
  }
  double E1n = sqrt(m1 * m1 * c2 * c2 + c2 * (a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]));
  double E2n = sqrt(m2 * m2 * c2 * c2 + c2 * (a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]));
  double p1du = p1[0] * du[0] + p1[1] * du[1] + p1[2] * du[2];
  double p2du = p2[0] * du[0] + p2[1] * du[1] + p2[2] * du[2];
  double du2 = du[0] * du[0] + du[1] * du[1] + du[2] * du[2];
  double h = c2 * ((2.0 * alpha * p1du + alpha * alpha * du2) / (E1n + E1) +
                   (-2.0 * alpha * p2du + alpha * alpha * du2) / (E2n + E2)) +
             U;
  double a1du = a1[0] * du[0] + a1[1] * du[1] + a1[2] * du[2];
  double a2du = a2[0] * du[0] + a2[1] * du[1] + a2[2] * du[2];
  *dh = c2 * (a1du / E1n - a2du / E2n);
  return h;
}

/* Relativistic pair energy correction, Appendix A: find alpha with
 * E1' + E2' = E_tot - U (Eq. (A.5)), taking the root continuous with the
 * non-relativistic one (the root on the branch alpha > -mu_R, where h is
 * increasing and convex), then p1 += alpha du, p2 -= alpha du (Eqs. (A.3),
 * (A.4)).  Returns 0 when no such root exists (U above the energy removable
 * at fixed pair momentum), leaving the pair unchanged. */
int oracle_energy_pair_rel(double m1, double m2, double U, double c, double *u1,
                           double *u2) {
  double c2 = c * c;
  double du[3] = {u1[0] - u2[0], u1[1] - u2[1], u1[2] - u2[2]};
  double p1[3], p2[3];
  for (int d = 0; d < 3; ++d) {
    p1[d] = m1 * u1[d];
    p2[d] = m2 * u2[d];
  }
  double g1 = sqrt(1.0 + (u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]) / c2);
  double g2 = sqrt(1.0 + (u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]) / c2);
  double E1 = m1 * c2 * g1, E2 = m2 * c2 * g2;
  double muR = m1 * m2 / (m1 + m2);
  double dh;
  double lo, hi;
  if (U > 0.0) {
    lo = -muR;
    hi = 0.0;
    double hlo = rel_h(m1, m2, p1, p2, du, E1, E2, c2, U, lo, &dh);
    if (hlo > 0.0) return 0; /* minimum of h above zero: no root */
  } else {
    lo = 0.0;
    hi = muR;
    while (rel_h(m1, m2, p1, p2, du, E1, E2, c2, U, hi, &dh) < 0.0) hi *= 2.0;
  }
  /* non-relativistic starting value alpha = mu_R (sqrt(1 - U/K) - 1) */
  double du2 = du[0] * du[0] + du[1] * du[1] + du[2] * du[2];
  double K = 0.5 * muR * du2;
  double x = U / K;
  double a = (x < 1.0) ? muR * (-x / (1.0 + sqrt(1.0 - x))) : 0.5 * (lo + hi);
  if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double h = rel_h(m1, m2, p1, p2, du, E1, E2, c2, U, a, &dh);
    if (h == 0.0) break;
    if (h > 0.0)
      hi = a;
    else
      lo = a;
    if (hi - lo <= 4.0 * 2.220446049250313e-16 * fabs(a)) break;
    double an = a - h / dh;
    if (!(an > lo && an < hi)) an = 0.5 * (lo + hi);
    if (fabs(an - a) <= 0.5 * 2.220446049250313e-16 * fabs(a)) {
      a = an;
      break;
    }
    a = an;
  }
  for (int d = 0; d < 3; ++d) {
    u1[d] += (a / m1) * du[d];
    u2[d] -= (a / m2) * du[d];
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* One collision (species a, species b) in one cell: Algorithm 1.            */
/* base: index of the cell's first particle; oa, ob: species segment offsets */
/* (absolute); na, nb: counts.                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  double w;
  int32_t pos;
  int32_t idx;
} wpos_t;

static int cmp_wpos(const void *pa, const void *pb) {
  const wpos_t *a = (const wpos_t *)pa, *b = (const wpos_t *)pb;
  if (a->w != b->w) return a->w > b->w ? -1 : 1; /* descending weight */
  return a->pos < b->pos ? -1 : (a->pos > b->pos ? 1 : 0);
}

static double kin_nr(double m, const double *v) {
  return 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

static double kin_rel(double m, const double *u, double c) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double g = sqrt(1.0 + uu / (c * c));
  return m * uu / (g + 1.0);
}

static int collide_one(const cfg_t *g, uint32_t cell, int coll, int64_t oa,
                       int32_t na, int64_t ob, int32_t nb, int sa, int sb,
                       double dV, const double *w, double *vx, double *vy,
                       double *vz, stats_t *st, int32_t *cell_corr) {
  const int intra = (sa == sb);
  if (intra) {
    if (na < 2) return ORC_OK;
  } else {
    if (na == 0 || nb == 0) return ORC_OK;
  }
  const int ns = intra ? 1 : 2;
  const int32_t nsp[2] = {na, intra ? 0 : nb};
  const int64_t off[2] = {oa, ob};
  const int sid[2] = {sa, sb};
  const int32_t ntot = na + (intra ? 0 : nb);
  /* participants: slot 0 = species a [0, na), slot 1 = species b [na, na+nb) */
  double *V = (double *)malloc(sizeof(double) * 6 * (size_t)ntot);
  double *Wt = (double *)malloc(sizeof(double) * (size_t)ntot);
  double *Ms = (double *)malloc(sizeof(double) * (size_t)ntot);
  int32_t *L[2] = {NULL, NULL};
  L[0] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(na > 0 ? na : 1));
  L[1] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nb > 0 ? nb : 1));
  if (!V || !Wt || !Ms || !L[0] || !L[1]) {
    free(V); free(Wt); free(Ms); free(L[0]); free(L[1]);
    return ORC_ERR_OOM;
  }
  double *vc = V, *vbs = V + 3 * (size_t)ntot; /* current, before-scatter */
  for (int sl = 0; sl < ns; ++sl) {
    int32_t base = sl == 0 ? 0 : na;
    for (int32_t i = 0; i < nsp[sl]; ++i) {
      int64_t p = off[sl] + i;
      vc[3 * (base + i) + 0] = vx[p];
      vc[3 * (base + i) + 1] = vy[p];
      vc[3 * (base + i) + 2] = vz[p];
      Wt[base + i] = w[p];
      Ms[base + i] = g->mass[sid[sl]];
    }
  }
  memcpy(vbs, vc, sizeof(double) * 3 * (size_t)ntot);
  const double ma = g->mass[sa], qa = g->charge[sa];
  const double mb = g->mass[sb], qb = g->charge[sb];

  /* random binary pairs (Fig. 1) */
  shuffle_list(na, cell, g->seed, g->step, coll, 0, L[0]);
  if (!intra) {
    shuffle_list(nb, cell, g->seed, g->step, coll, 1, L[1]);
    for (int32_t i = 0; i < nb; ++i) L[1][i] += na; /* participant index */
  }

#define SCATTER(pk, f, nmin, I, J)                                             \
  do {                                                                         \
    double *vi_ = vc + 3 * (I), *vj_ = vc + 3 * (J);                           \
    if (g->rel)                                                                \
      scatter_pair_rel(g, cell, coll, (uint32_t)(pk), f, nmin, dV, ma, qa, mb, \
                       qb, Wt[I], Wt[J], vi_, vj_);                            \
    else                                                                       \
      scatter_pair_nr(g, cell, coll, (uint32_t)(pk), f, nmin, dV, ma, qa, mb,  \
                      qb, Wt[I], Wt[J], vi_, vj_);                             \
  } while (0)

  int64_t npairs = 0;
  if (g->pairing == ORC_NXN) {
    /* Sec. 3.1: all pairs, each once, s with w_max / dV (N_min = 1) */
    if (intra) {
      int32_t np = na + (na & 1), R = np - 1, P = np / 2;
      for (int32_t r = 0; r < R; ++r)
        for (int32_t m = 0; m < P; ++m) {
          int32_t x = m == 0 ? r : (r + m) % R;
          int32_t y = m == 0 ? np - 1 : (r - m + R) % R;
          if (x >= na || y >= na) continue; /* the pad of an odd N */
          SCATTER((int64_t)r * P + m, 1.0, 1.0, L[0][x], L[0][y]);
          ++npairs;
        }
    } else {
      int32_t nmax = na >= nb ? na : nb;
      for (int32_t r = 0; r < nmax; ++r)
        for (int32_t i = 0; i < na; ++i) {
          int32_t j = (i + r) % nmax;
          if (j >= nb) continue;
          SCATTER((int64_t)r * na + i, 1.0, 1.0, L[0][i], L[1][j]);
          ++npairs;
        }
    }
  } else if (intra) {
    /* Sec. 3.2 last paragraphs: N_min = N_alpha - 1; odd N: first three
     * particles paired N x N with s/2. */
    double nmin = (double)(na - 1);
    int32_t k = 0, start = 0;
    if (na & 1) {
      SCATTER(0, 0.5, nmin, L[0][0], L[0][1]);
      SCATTER(1, 0.5, nmin, L[0][1], L[0][2]);
      SCATTER(2, 0.5, nmin, L[0][2], L[0][0]);
      k = 3;
      start = 3;
      npairs += 3;
    }
    for (int32_t i = start; i + 1 < na; i += 2, ++k) {
      SCATTER(k, 1.0, nmin, L[0][i], L[0][i + 1]);
      ++npairs;
    }
  } else {
    /* TA77 order-N pairing: N_max pairs, each particle of the larger
     * population once, the smaller one N_max/N_min times on average. */
    int32_t nmax = na >= nb ? na : nb, nmn = na >= nb ? nb : na;
    for (int32_t k = 0; k < nmax; ++k) {
      int32_t I, J;
      if (na >= nb) {
        I = L[0][k];
        J = L[1][k % nmn];
      } else {
        I = L[0][k % nmn];
        J = L[1][k];
      }
      double nfac = (double)nmn;
      if (g->pairing == ORC_DUPLICITY) {
        /* D: the pairs k' < N_max with k' = k (mod N_min) */
        int32_t dup = (nmax - k % nmn + nmn - 1) / nmn;
        nfac = (double)nmax / (double)dup;
      }
      SCATTER(k, 1.0, nfac, I, J);
    }
    npairs += nmax;
  }
#undef SCATTER
  st->pairs += npairs;
  st->collisions += 1;
  if (g_trace) {
    for (int sl = 0; sl < ns; ++sl) {
      int32_t base = sl == 0 ? 0 : na;
      for (int32_t i = 0; i < nsp[sl]; ++i)
        for (int d = 0; d < 3; ++d)
          g_trace->vps[d * g_trace->n + off[sl] + i] = vc[3 * (base + i) + d];
    }
  }

  int failed = 0;
  int32_t corr_used = 0;
  if (g->corr) {
    const double c = g->c;
    /* Eq. (17): B = sum m_p (v_ps - v_bs) / sum m_p w_p, m_p = m_s w_p */
    nsum_t P[3] = {{0, 0}, {0, 0}, {0, 0}}, Dn = {0, 0};
    for (int32_t p = 0; p < ntot; ++p) {
      double mp = Ms[p] * Wt[p];
      for (int d = 0; d < 3; ++d) nadd(&P[d], mp * (vc[3 * p + d] - vbs[3 * p + d]));
      nadd(&Dn, mp * Wt[p]);
    }
    double B[3] = {nval(&P[0]) / nval(&Dn), nval(&P[1]) / nval(&Dn),
                   nval(&P[2]) / nval(&Dn)};
    for (int32_t p = 0; p < ntot; ++p)
      for (int d = 0; d < 3; ++d) vc[3 * p + d] -= B[d] * Wt[p];

    if (g_trace) {
      for (int sl = 0; sl < ns; ++sl) {
        int32_t base = sl == 0 ? 0 : na;
        for (int32_t i = 0; i < nsp[sl]; ++i)
          for (int d = 0; d < 3; ++d)
            g_trace->vpm[d * g_trace->n + off[sl] + i] = vc[3 * (base + i) + d];
      }
    }
    /* Eq. (18) in difference form; Eq. (24) partition */
    nsum_t dE = {0, 0}, Es[2] = {{0, 0}, {0, 0}}, Ws[2] = {{0, 0}, {0, 0}};
    for (int32_t p = 0; p < ntot; ++p) {
      double mp = Ms[p] * Wt[p];
      const double *v = vc + 3 * p, *b = vbs + 3 * p;
      double term;
      if (g->rel) {
        double c2 = c * c;
        double gv = sqrt(1.0 + (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / c2);
        double gb = sqrt(1.0 + (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]) / c2);
        term = mp * ((v[0] - b[0]) * (v[0] + b[0]) + (v[1] - b[1]) * (v[1] + b[1]) +
                     (v[2] - b[2]) * (v[2] + b[2])) /
               (gv + gb);
      } else {
        term = 0.5 * mp * ((v[0] - b[0]) * (v[0] + b[0]) + (v[1] - b[1]) * (v[1] + b[1]) +
                           (v[2] - b[2]) * (v[2] + b[2]));
      }
      nadd(&dE, term);
      int sl = p < na ? 0 : 1;
      nadd(&Es[sl], g->rel ? kin_rel(mp, v, c) : kin_nr(mp, v));
      nadd(&Ws[sl], Wt[p]);
    }
    double dEtot = nval(&dE);
    double dEs[2] = {dEtot, 0.0};
    if (!intra && dEtot != 0.0) {
      double wa = nval(&Ws[0]) / na, wb = nval(&Ws[1]) / nb;
      double ea = wa * nval(&Es[0]), eb = wb * nval(&Es[1]);
      dEs[0] = ea / (ea + eb) * dEtot;
      dEs[1] = eb / (ea + eb) * dEtot;
    }

    if (g_trace) {
      int64_t slot = (int64_t)cell * g_trace->n_coll + coll;
      g_trace->dE[slot] = dEtot;
      g_trace->dEs[2 * slot] = dEs[0];
      g_trace->dEs[2 * slot + 1] = dEs[1];
    }
    /* per species: order, then pair energy correction (Alg. 1 final loop) */
    for (int sl = 0; sl < ns; ++sl) {
      int32_t n = nsp[sl];
      int32_t base = sl == 0 ? 0 : na;
      int32_t *O = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
      wpos_t *wp = (wpos_t *)malloc(sizeof(wpos_t) * (size_t)(n > 0 ? n : 1));
      if (!O || !wp) {
        free(O); free(wp); free(V); free(Wt); free(Ms); free(L[0]); free(L[1]);
        return ORC_ERR_OOM;
      }
      for (int32_t q = 0; q < n; ++q) O[q] = L[sl][q]; /* shuffled order */
      if (g->sortw) {
        for (int32_t q = 0; q < n; ++q) {
          wp[q].w = Wt[O[q]];
          wp[q].pos = q;
          wp[q].idx = O[q];
        }
        qsort(wp, (size_t)n, sizeof(wpos_t), cmp_wpos);
        for (int32_t q = 0; q < n; ++q) O[q] = wp[q].idx;
      }
      double E = dEs[sl];
      const double ms = Ms[base];
      for (int pass = 0; pass < g->max_passes && E != 0.0; ++pass) {
        for (int32_t k = 0; 2 * k + 1 < n; ++k) {
          if (E == 0.0) break;
          int32_t p = O[2 * k], q = O[2 * k + 1];
          double m1 = ms * Wt[p], m2 = ms * Wt[q];
          double *v1 = vc + 3 * p, *v2 = vc + 3 * q;
          double K;
          if (g->rel) {
            K = rel_kecm(m1, m2, v1, v2, c);
          } else {
            double mu = m1 * m2 / (m1 + m2);
            K = 0.5 * mu * ((v1[0] - v2[0]) * (v1[0] - v2[0]) +
                            (v1[1] - v2[1]) * (v1[1] - v2[1]) +
                            (v1[2] - v2[2]) * (v1[2] - v2[2]));
          }
          if (K == 0.0) continue;
          /* Eq. (23) */
          double lim = g->fE * K;
          double U = fabs(E) < lim ? E : copysign(lim, E);
          if (g->rel) {
            if (!oracle_energy_pair_rel(m1, m2, U, c, v1, v2)) continue;
          } else {
            oracle_energy_pair_nr(m1, m2, U, v1, v2);
          }
          E -= U;
          ++corr_used;
        }
      }
      if (E != 0.0) failed = 1;
      free(O);
      free(wp);
    }
    if (failed) {
      st->failed += 1;
      if (!g->keep_on_fail) memcpy(vc, vbs, sizeof(double) * 3 * (size_t)ntot);
    }
    /* diagnostics: residual momentum / energy relative to the cell totals */
    nsum_t rP[3] = {{0, 0}, {0, 0}, {0, 0}}, rE = {0, 0}, aP = {0, 0}, aE = {0, 0};
    for (int32_t p = 0; p < ntot; ++p) {
      double mp = Ms[p] * Wt[p];
      const double *v = vc + 3 * p, *b = vbs + 3 * p;
      for (int d = 0; d < 3; ++d) nadd(&rP[d], mp * (v[d] - b[d]));
      nadd(&aP, mp * sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
      double term;
      if (g->rel) {
        double c2 = c * c;
        double gv = sqrt(1.0 + (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / c2);
        double gb = sqrt(1.0 + (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]) / c2);
        term = mp * ((v[0] - b[0]) * (v[0] + b[0]) + (v[1] - b[1]) * (v[1] + b[1]) +
                     (v[2] - b[2]) * (v[2] + b[2])) / (gv + gb);
        nadd(&aE, kin_rel(mp, b, c));
      } else {
        term = 0.5 * mp * ((v[0] - b[0]) * (v[0] + b[0]) + (v[1] - b[1]) * (v[1] + b[1]) +
                           (v[2] - b[2]) * (v[2] + b[2]));
        nadd(&aE, kin_nr(mp, b));
      }
      nadd(&rE, term);
    }
    double rp = sqrt(nval(&rP[0]) * nval(&rP[0]) + nval(&rP[1]) * nval(&rP[1]) +
                     nval(&rP[2]) * nval(&rP[2]));
    double ap = nval(&aP), ae = nval(&aE);
    double relP = ap > 0.0 ? rp / ap : 0.0;
    double relE = ae > 0.0 ? fabs(nval(&rE)) / ae : 0.0;
    if (relP > st->max_rel_dP) st->max_rel_dP = relP;
    if (relE > st->max_rel_dE) st->max_rel_dE = relE;
  }
  st->corr_pairs += corr_used;
  if (cell_corr) *cell_corr += corr_used;

  /* write back */
  for (int sl = 0; sl < ns; ++sl) {
    int32_t base = sl == 0 ? 0 : na;
    for (int32_t i = 0; i < nsp[sl]; ++i) {
      int64_t p = off[sl] + i;
      vx[p] = vc[3 * (base + i) + 0];
      vy[p] = vc[3 * (base + i) + 1];
      vz[p] = vc[3 * (base + i) + 2];
    }
  }
  free(V);
  free(Wt);
  free(Ms);
  free(L[0]);
  free(L[1]);
  return ORC_OK;
}

static int check_common(int64_t n, int32_t n_cells, int32_t n_species,
                        const double *mass, const double *charge,
                        int32_t n_coll, const int32_t *ca, const int32_t *cb,
                        const double *w, double dt, double lnL, int32_t method,
                        int32_t rel, int32_t max_passes, double fE, double eps0,
                        double c, const double *cell_volume, double dVs) {
  if (n < 0 || n_cells < 0 || n_species < 1 || n_coll < 0 || n_coll > 256)
    return ORC_ERR_INVALID;
  if (!mass || !charge || (n_coll > 0 && (!ca || !cb))) return ORC_ERR_INVALID;
  for (int s = 0; s < n_species; ++s)
    if (!(mass[s] > 0.0) || !isfinite(mass[s]) || !isfinite(charge[s]))
      return ORC_ERR_INVALID;
  for (int k = 0; k < n_coll; ++k)
    if (ca[k] < 0 || ca[k] >= n_species || cb[k] < 0 || cb[k] >= n_species)
      return ORC_ERR_INVALID;
  for (int64_t i = 0; i < n; ++i)
    if (!(w[i] > 0.0) || !isfinite(w[i])) return ORC_ERR_INVALID;
  if (!isfinite(dt) || dt < 0.0 || !isfinite(lnL) || lnL < 0.0) return ORC_ERR_INVALID;
  if (method != ORC_TA77 && method != ORC_N97 && method != ORC_HARD_SPHERE)
    return ORC_ERR_INVALID;
  if (method == ORC_HARD_SPHERE && rel) return ORC_ERR_INVALID;
  if (max_passes < 1) return ORC_ERR_INVALID;
  if (!(fE > 0.0) || !(fE < 1.0)) return ORC_ERR_INVALID;
  if (!(eps0 > 0.0)) return ORC_ERR_INVALID;
  if (rel && !(c > 0.0 && isfinite(c))) return ORC_ERR_INVALID;
  if (!cell_volume && !(dVs > 0.0)) return ORC_ERR_INVALID;
  if (cell_volume)
    for (int32_t i = 0; i < n_cells; ++i)
      if (!(cell_volume[i] > 0.0)) return ORC_ERR_INVALID;
  return ORC_OK;
}

/* Threads of the cell loop (OpenMP, dynamic schedule).  Cells are
 * independent and every random number is keyed by the cell, so the result
 * does not depend on the thread count: every thread runs the same
 * sequential code on its cells. */
static int g_threads = 1;
void oracle_set_threads(int32_t n) { g_threads = n > 0 ? n : 1; }

/*
 * One collision step over particles grouped by (cell, species).
 * offsets[n_cells*n_species + 1]: particles of cell c, species s occupy
 * [offsets[c*S+s], offsets[c*S+s+1]).  cell_list (nullable): process only
 * these cells.  counters[4] (nullable): pairs, correction pairs, failures,
 * collisions.  diag[2] (nullable): max relative residual momentum, energy.
 */
int oracle_collide_sorted(
    int64_t n, int32_t n_cells, int32_t n_species, const int64_t *offsets,
    const double *mass, const double *charge, int32_t n_coll,
    const int32_t *coll_a, const int32_t *coll_b, const double *w, double *vx,
    double *vy, double *vz, const double *cell_volume, double cell_volume_scalar,
    double dt, double coulomb_log, uint64_t seed, uint64_t step, int32_t method,
    int32_t pairing, int32_t relativistic, int32_t moment_correction,
    int32_t sort_by_weight, int32_t max_passes, int32_t keep_on_fail, double f_E,
    double eps0, double c, const int32_t *cell_list, int32_t n_list,
    int64_t *counters, double *diag, int32_t *cell_corr_pairs,
    const double *cross_section, int32_t uniform23) {
  int rc = check_common(n, n_cells, n_species, mass, charge, n_coll, coll_a,
                        coll_b, w, dt, coulomb_log, method, relativistic,
                        max_passes, f_E, eps0, c, cell_volume, cell_volume_scalar);
  if (rc) return rc;
  if (pairing != ORC_ORDER_N && pairing != ORC_NXN && pairing != ORC_DUPLICITY)
    return ORC_ERR_INVALID;
  if (method == ORC_HARD_SPHERE) {
    if (n_coll > 0 && !cross_section) return ORC_ERR_INVALID;
    for (int k = 0; k < n_coll; ++k)
      if (!(cross_section[k] >= 0.0) || !isfinite(cross_section[k])) return ORC_ERR_INVALID;
  }
  const int64_t S = n_species;
  if (offsets[0] != 0 || offsets[(int64_t)n_cells * S] != n) return ORC_ERR_INVALID;
  for (int64_t i = 0; i < (int64_t)n_cells * S; ++i)
    if (offsets[i + 1] < offsets[i]) return ORC_ERR_INVALID;
  cfg_t g = {n_species, mass, charge, n_coll, coll_a, coll_b, dt, coulomb_log,
             eps0, c, seed, step, method, relativistic, moment_correction,
             sort_by_weight, max_passes, keep_on_fail, f_E, pairing,
             cross_section, uniform23 ? 1 : 0};
  stats_t st;
  memset(&st, 0, sizeof(st));
  int32_t nl = cell_list ? n_list : n_cells;
  for (int32_t li = 0; cell_list && li < nl; ++li)
    if (cell_list[li] < 0 || cell_list[li] >= n_cells) return ORC_ERR_INVALID;
  int rc_all = ORC_OK;
  /* the trace hook records into shared arrays: one thread then */
  const int nthr = g_trace ? 1 : g_threads;
#pragma omp parallel num_threads(nthr)
  {
    stats_t lst;
    memset(&lst, 0, sizeof(lst));
#pragma omp for schedule(dynamic, 1)
    for (int32_t li = 0; li < nl; ++li) {
      int32_t cell = cell_list ? cell_list[li] : li;
      double dV = cell_volume ? cell_volume[cell] : cell_volume_scalar;
      int32_t *cc = cell_corr_pairs ? &cell_corr_pairs[cell] : NULL;
      if (cc) *cc = 0;
      for (int k = 0; k < n_coll; ++k) {
        int sa = coll_a[k], sb = coll_b[k];
        int64_t oa = offsets[cell * S + sa], ob = offsets[cell * S + sb];
        int32_t na = (int32_t)(offsets[cell * S + sa + 1] - oa);
        int32_t nb = (int32_t)(offsets[cell * S + sb + 1] - ob);
        int rc1 = collide_one(&g, (uint32_t)cell, k, oa, na, ob, nb, sa, sb, dV, w, vx,
                              vy, vz, &lst, cc);
        if (rc1) {
#pragma omp critical(oracle_rc)
          if (rc_all == ORC_OK) rc_all = rc1;
          break;
        }
      }
    }
#pragma omp critical(oracle_stats)
    {
      st.pairs += lst.pairs;
      st.corr_pairs += lst.corr_pairs;
      st.failed += lst.failed;
      st.collisions += lst.collisions;
      if (lst.max_rel_dP > st.max_rel_dP) st.max_rel_dP = lst.max_rel_dP;
      if (lst.max_rel_dE > st.max_rel_dE) st.max_rel_dE = lst.max_rel_dE;
    }
  }
  if (rc_all) return rc_all;
  if (counters) {
    counters[0] = st.pairs;
    counters[1] = st.corr_pairs;
    counters[2] = st.failed;
    counters[3] = st.collisions;
  }
  if (diag) {
    diag[0] = st.max_rel_dP;
    diag[1] = st.max_rel_dE;
  }
  return ORC_OK;
}

/*
 * Unsorted entry: particles in any order with cells[i], species[i].  The
 * particles are grouped by (cell, species) keeping ascending index order
 * within each group (a stable counting sort), the sorted step is applied,
 * and the velocities are written back to their original positions.
 */
int oracle_collide(int64_t n, const int32_t *cells, const int32_t *species,
                   int32_t n_cells, int32_t n_species, const double *mass,
                   const double *charge, int32_t n_coll, const int32_t *coll_a,
                   const int32_t *coll_b, const double *w, double *vx,
                   double *vy, double *vz, const double *cell_volume,
                   double cell_volume_scalar, double dt, double coulomb_log,
                   uint64_t seed, uint64_t step, int32_t method,
                   int32_t pairing, int32_t relativistic, int32_t moment_correction,
                   int32_t sort_by_weight, int32_t max_passes,
                   int32_t keep_on_fail, double f_E, double eps0, double c,
                   int64_t *counters, double *diag, int32_t *cell_corr_pairs,
                   const double *cross_section, int32_t uniform23) {
  if (n < 0 || n_cells < 0 || n_species < 1) return ORC_ERR_INVALID;
  const int64_t S = n_species, nk = (int64_t)n_cells * S;
  for (int64_t i = 0; i < n; ++i)
    if (cells[i] < 0 || cells[i] >= n_cells || species[i] < 0 || species[i] >= n_species)
      return ORC_ERR_INVALID;
  int64_t *off = (int64_t *)calloc((size_t)nk + 1, sizeof(int64_t));
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nk + 1));
  int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  double *g = (double *)malloc(sizeof(double) * 4 * (size_t)(n > 0 ? n : 1));
  if (!off || !cur || !perm || !g) {
    free(off); free(cur); free(perm); free(g);
    return ORC_ERR_OOM;
  }
  for (int64_t i = 0; i < n; ++i) off[(int64_t)cells[i] * S + species[i] + 1]++;
  for (int64_t k = 0; k < nk; ++k) off[k + 1] += off[k];
  memcpy(cur, off, sizeof(int64_t) * ((size_t)nk + 1));
  for (int64_t i = 0; i < n; ++i) perm[cur[(int64_t)cells[i] * S + species[i]]++] = i;
  double *gw = g, *gx = g + n, *gy = g + 2 * n, *gz = g + 3 * n;
  for (int64_t j = 0; j < n; ++j) {
    gw[j] = w[perm[j]];
    gx[j] = vx[perm[j]];
    gy[j] = vy[perm[j]];
    gz[j] = vz[perm[j]];
  }
  int rc = oracle_collide_sorted(
      n, n_cells, n_species, off, mass, charge, n_coll, coll_a, coll_b, gw, gx,
      gy, gz, cell_volume, cell_volume_scalar, dt, coulomb_log, seed, step,
      method, pairing, relativistic, moment_correction, sort_by_weight,
      max_passes, keep_on_fail, f_E, eps0, c, NULL, 0, counters, diag,
      cell_corr_pairs, cross_section, uniform23);
  if (rc == ORC_OK) {
    for (int64_t j = 0; j < n; ++j) {
      vx[perm[j]] = gx[j];
      vy[perm[j]] = gy[j];
      vz[perm[j]] = gz[j];
    }
  }
  free(off);
  free(cur);
  free(perm);
  free(g);
  return rc;
}

/* Grouping used by the unsorted entry, exposed for tests: offsets and the
 * stable permutation (sorted position -> original index). */
int oracle_bin(int64_t n, const int32_t *cells, const int32_t *species,
               int32_t n_cells, int32_t n_species, int64_t *offsets,
               int64_t *perm) {
  const int64_t S = n_species, nk = (int64_t)n_cells * S;
  for (int64_t i = 0; i < n; ++i)
    if (cells[i] < 0 || cells[i] >= n_cells || species[i] < 0 || species[i] >= n_species)
      return ORC_ERR_INVALID;
  memset(offsets, 0, sizeof(int64_t) * ((size_t)nk + 1));
  for (int64_t i = 0; i < n; ++i) offsets[(int64_t)cells[i] * S + species[i] + 1]++;
  for (int64_t k = 0; k < nk; ++k) offsets[k + 1] += offsets[k];
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nk + 1));
  if (!cur) return ORC_ERR_OOM;
  memcpy(cur, offsets, sizeof(int64_t) * ((size_t)nk + 1));
  for (int64_t i = 0; i < n; ++i) perm[cur[(int64_t)cells[i] * S + species[i]]++] = i;
  free(cur);
  return ORC_OK;
}

/* Single-pair entry points for the tests' closed-form and statistical pins. */
void oracle_scatter_pair(int32_t method, int32_t relativistic, double s_factor,
                         double nmin, double dV, double dt, double lnL,
                         double eps0, double c, uint64_t seed, uint64_t step,
                         uint32_t cell, int32_t coll, uint32_t pair_k, double mi,
                         double qi, double mj, double qj, double wi, double wj,
                         double *vi, double *vj) {
  cfg_t g;
  memset(&g, 0, sizeof(g));
  g.dt = dt;
  g.lnL = lnL;
  g.eps0 = eps0;
  g.c = c;
  g.seed = seed;
  g.step = step;
  g.method = method;
  g.rel = relativistic;
  if (method != ORC_TA77 && method != ORC_N97) return; /* Coulomb methods only */
  if (relativistic)
    scatter_pair_rel(&g, cell, coll, pair_k, s_factor, nmin, dV, mi, qi, mj, qj,
                     wi, wj, vi, vj);
  else
    scatter_pair_nr(&g, cell, coll, pair_k, s_factor, nmin, dV, mi, qi, mj, qj,
                    wi, wj, vi, vj);
}

double oracle_rel_kecm(double m1, double m2, const double *u1, const double *u2,
                       double c) {
  return rel_kecm(m1, m2, u1, u2, c);
}

/* Test hook: oracle_collide_sorted with intermediate states recorded. */
int oracle_collide_sorted_traced(
    int64_t n, int32_t n_cells, int32_t n_species, const int64_t *offsets,
    const double *mass, const double *charge, int32_t n_coll,
    const int32_t *coll_a, const int32_t *coll_b, const double *w, double *vx,
    double *vy, double *vz, double cell_volume_scalar, double dt,
    double coulomb_log, uint64_t seed, uint64_t step, int32_t method,
    int32_t relativistic, int32_t sort_by_weight, double f_E, double c,
    double *vps, double *vpm, double *dE, double *dEs) {
  trace_t t = {vps, vpm, dE, dEs, n, n_coll};
  g_trace = &t;
  int rc = oracle_collide_sorted(
      n, n_cells, n_species, offsets, mass, charge, n_coll, coll_a, coll_b, w,
      vx, vy, vz, NULL, cell_volume_scalar, dt, coulomb_log, seed, step, method,
      ORC_ORDER_N, relativistic, 1, sort_by_weight, 1, 0, f_E, 1.0, c, NULL, 0,
      NULL, NULL, NULL, NULL, 0);
  g_trace = NULL;
  return rc;
}
