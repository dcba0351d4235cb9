// mcc_collide.hpp -- the per-cell collision kernel (Algorithm 1 of the paper),
// one workgroup per cell, cells taken from a size-bucketed work list.
//
// Template parameters:
//   TPC  threads per cell (workgroup size, multiple of 64)
//   CAP  largest cell (all species) this variant holds
//   KR   type of the pair kinematics (double, or float for the FP32 form)
//   REL  relativistic (Appendix A; FP64 only)
//   LAY  where the cell lives: LAYOUT_LDS (everything in LDS), LAYOUT_COMPACT
//        (LDS with aliased scratch and the weights read from the input, for
//        cells up to 4096), LAYOUT_GLOBAL (per-workgroup global scratch for
//        cells up to MCC_MAX_CELL; one, four or eight waves per cell, whose
//        scratch accesses the workgroup barriers order as they do LDS ones,
//        the waves of a workgroup sharing their CU's L1)
//
// Data flow per cell: the cell's velocities and weights are staged in LDS
// (coalesced loads), every collision of the list is applied in order, and
// the velocities are written back once.  Pre-scatter velocities are kept in
// the owner thread's registers (particle e is owned by thread e % TPC).
#pragma once

#include "mcc_device.hpp"
#include "mcc_kernel_args.hpp"
#include "mcc_variants.hpp"

namespace mcc {

// Where the arrays of a cell live (all cross-thread data is in LDS unless the
// layout is GLOBAL, whose workgroup is a single wave).
enum Layout : int { LAYOUT_LDS = 0, LAYOUT_COMPACT = 1, LAYOUT_GLOBAL = 2 };
enum Pairing : int { PAIR_ORDER_N = 0, PAIR_NXN = 1, PAIR_DUPLICITY = 2 };

struct CellMem {
  double *vx, *vy, *vz;
  const double *w;        // LDS copy, or the read-only input (COMPACT)
  uint16_t *list0, *list1, *ord0, *ord1, *mem;
  uint16_t *word;         // descending-weight order per species (not kept in the compact layout)
  uint32_t *key;          // shuffle keys (CAP)
  uint32_t *cnt;          // CAP+1 bucket counters, always LDS (atomics)
  double *kbuf;           // per-pair K / U of the energy loop (+ h(-mu) for REL)
  uint32_t *slotbuf;      // GLOBAL: per-item bucket slots
  double *bx, *by, *bz;   // GLOBAL: pre-scatter snapshot
  // tangent form: tangent of the velocities, its pre-scatter snapshot, and
  // per-pair tangents of K (then of U)
  double *tx, *ty, *tz, *btx, *bty, *btz, *kdot;
};

// ---------------------------------------------------------------------------
// Pair scatter (Sec. 3.1-3.2, Eq. (12)); non-relativistic
// ---------------------------------------------------------------------------
template <typename KR, class Tab>
__device__ __forceinline__ void scatter_pair_nr(double *vx, double *vy, double *vz,
                                                const double *w, int I, int J, uint32_t kp,
                                                double coef_f_nmin_dV, double fa, double fb,
                                                int method, uint32_t cell, uint32_t step_lo,
                                                uint32_t c3, uint32_t k0, uint32_t k1,
                                                const Tab *n97tab) {
  using K = KMath<KR>;
  const double vix = vx[I], viy = vy[I], viz = vz[I];
  const double vjx = vx[J], vjy = vy[J], vjz = vz[J];
  const double wi = w[I], wj = w[J];
  const KR ux = (KR)(vix - vjx), uy = (KR)(viy - vjy), uz = (KR)(viz - vjz);
  const KR um2 = ux * ux + uy * uy + uz * uz;
  if (um2 == KR(0)) return;
  const KR um = K::sqrt_(um2);
  const double wmax = wi > wj ? wi : wj;
  const KR s = K::div((KR)(coef_f_nmin_dV * wmax), um2 * um);
  if (!(s > KR(0))) return;
  const U4 r = philox(kp, cell, step_lo, c3, k0, k1);
  KR oc, st;
  sample_angle<KR>(method, s, r.x, r.y, oc, st, n97tab);
  KR sp, cp;
  K::sincos2pi(K::u(r.z), sp, cp);
  KR dx, dy, dz;
  rotate_delta<KR>(ux, uy, uz, st, oc, sp, cp, dx, dy, dz);
  // acceptance of the heavier particle, decided in FP64 in every mode
  // (w_min / w_max: one division for either branch)
  const double u3 = unif64(r.w);
  const double wratio = (wi < wj ? wi : wj) / wmax;
  bool ai = true, aj = true;
  if (wi < wj)
    aj = u3 <= wratio;
  else if (wj < wi)
    ai = u3 <= wratio;
  if (ai) {
    vx[I] = vix + fa * (double)dx;
    vy[I] = viy + fa * (double)dy;
    vz[I] = viz + fa * (double)dz;
  }
  if (aj) {
    vx[J] = vjx - fb * (double)dx;
    vy[J] = vjy - fb * (double)dy;
    vz[J] = vjz - fb * (double)dz;
  }
}

// Hard-sphere pair (the non-Coulomb process of the collision integral of
// Sec. 2 with the weighting of Sec. 3): s = sigma n_eff |u| dt is the
// expected number of collisions in the step; the pair collides with
// probability 1 - exp(-s) and then scatters isotropically (1 - cos chi
// uniform on (0, 2)).  Words: x the collision, y the angle, z the azimuth,
// w the heavier particle's acceptance.  FP64.
__device__ __forceinline__ void scatter_pair_hs(double *vx, double *vy, double *vz,
                                                const double *w, int I, int J, uint32_t kp,
                                                double sigma_dt_f_nmin_dV, double fa, double fb,
                                                uint32_t cell, uint32_t step_lo, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
  const double vix = vx[I], viy = vy[I], viz = vz[I];
  const double vjx = vx[J], vjy = vy[J], vjz = vz[J];
  const double wi = w[I], wj = w[J];
  const double ux = vix - vjx, uy = viy - vjy, uz = viz - vjz;
  const double um2 = ux * ux + uy * uy + uz * uz;
  if (um2 == 0.0) return;
  const double wmax = wi > wj ? wi : wj;
  const double s = sigma_dt_f_nmin_dV * wmax * sqrt(um2);
  if (!(s > 0.0)) return;
  const U4 r = philox(kp, cell, step_lo, c3, k0, k1);
  if (!(unif64(r.x) < -expm1(-s))) return;
  const double oc = 2.0 * unif64(r.y);
  const double st = sqrt(oc * (2.0 - oc));
  double sp, cp;
  KMath<double>::sincos2pi(unif64(r.z), sp, cp);
  double dx, dy, dz;
  rotate_delta<double>(ux, uy, uz, st, oc, sp, cp, dx, dy, dz);
  const double u3 = unif64(r.w);
  const double wratio = (wi < wj ? wi : wj) / wmax;
  bool ai = true, aj = true;
  if (wi < wj)
    aj = u3 <= wratio;
  else if (wj < wi)
    ai = u3 <= wratio;
  if (ai) {
    vx[I] = vix + fa * dx;
    vy[I] = viy + fa * dy;
    vz[I] = viz + fa * dz;
  }
  if (aj) {
    vx[J] = vjx - fb * dx;
    vy[J] = vjy - fb * dy;
    vz[J] = vjz - fb * dz;
  }
}

// The FP64 pair kinematics as a call rather than inline: its transcendental
// code then does not share a register allocation with the rest of the cell
// kernel, which roughly halves the kernel's registers (measured: the FP64
// step runs in 0.63x the time); the FP32 form is cheaper inline.
__device__ __attribute__((noinline)) void scatter_pair_nr_f64(
    double *vx, double *vy, double *vz, const double *w, int I, int J, uint32_t kp,
    double coef_f_nmin_dV, double fa, double fb, int method, uint32_t cell, uint32_t step_lo,
    uint32_t c3, uint32_t k0, uint32_t k1, const double2 *n97tab) {
  if (method == MCC_HARD_SPHERE)
    scatter_pair_hs(vx, vy, vz, w, I, J, kp, coef_f_nmin_dV, fa, fb, cell, step_lo, c3, k0, k1);
  else
    scatter_pair_nr<double>(vx, vy, vz, w, I, J, kp, coef_f_nmin_dV, fa, fb, method, cell,
                            step_lo, c3, k0, k1, n97tab);
}

// ---------------------------------------------------------------------------
// Tangent (forward-mode) pair scatter, FP64: the primal update exactly as
// scatter_pair_nr<double>, and the derivative of the pair's new velocities
// along the tangent (t of the velocities, dlnl = d lnL / lnL) with the
// random numbers and the acceptance fixed.  A(s) is differentiated as the
// root of Nanbu's equation: dA/ds = -exp(-s) / L'(A).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double langevin_prime(double A) {
  if (A < 0.5) {
    double L, dL;
    langevin_series(A, L, dL);
    return dL;
  }
  // 1/sinh^2 A = 4 e^{-2A} / (1 - e^{-2A})^2, finite for every A
  const double em = expm1(-2.0 * A), ra = 1.0 / A;
  return ra * ra - 4.0 * (em + 1.0) / (em * em);
}

// Tangent of a pair's velocity change du (the rotation of u = v_I - v_J by
// the sampled angle, TA77 form) along (tu, ts): tu the tangent of u and ts
// that of s, with the random numbers fixed; u0 the angle's uniform and A
// Nanbu's parameter of s (N97).  oc = 1 - cos(theta), st = sin(theta), and
// (sp, cp) the azimuth's sine and cosine, as the primal sampled them.
__device__ __forceinline__ void rot_tangent(int method, double ux, double uy, double uz, double um,
                                            double s, double oc, double st, double sp,
                                            double cp, double u0, double A, double tux,
                                            double tuy, double tuz, double ts, double &tdx,
                                            double &tdy, double &tdz) {
  using K = KMath<double>;
  const double tum = (ux * tux + uy * tuy + uz * tuz) / um;
  // tangent of 1 - cos(theta) and sin(theta)
  double toc = 0.0;
  if (method == 0) {  // TA77: delta = sqrt(s/2) z scales as sqrt(s)
    if (oc < 2.0) {
      const double d2 = oc / (2.0 - oc);  // delta^2, from oc = 2 d2 / (1 + d2)
      // d oc / d(delta^2) = 2 / (1 + d2)^2 and d(delta^2) = delta^2 ds / s
      toc = 2.0 / ((1.0 + d2) * (1.0 + d2)) * d2 * ts / s;
    }
  } else {
    if (A > 0.0 && !__builtin_isinf(A) && oc > 0.0 && oc < 2.0) {
      const double e = expm1(-2.0 * A);
      const double den = 1.0 + u0 * e;
      const double dl_dA = -2.0 * u0 * (e + 1.0) / den;  // d log1p(u0 e) / dA
      const double doc_dA = -dl_dA / A - oc / A;
      const double dA_ds = -exp(-s) / langevin_prime(A);
      toc = doc_dA * dA_ds * ts;
    }
  }
  // st^2 = oc (2 - oc) for either sign of st
  const double tst = st != 0.0 ? (1.0 - oc) * toc / st : 0.0;
  // tangent of the rotation
  const double up2 = ux * ux + uy * uy;
  const double up = K::sqrt_(up2);
  if (up > 0.0) {
    const double tup = (ux * tux + uy * tuy) / up;
    const double ax = ux / up, ay = uy / up;
    const double tax = (tux - ax * tup) / up, tay = (tuy - ay * tup) / up;
    tdx = tax * uz * st * cp + ax * (tuz * st + uz * tst) * cp - tay * um * st * sp -
          ay * (tum * st + um * tst) * sp - tux * oc - ux * toc;
    tdy = tay * uz * st * cp + ay * (tuz * st + uz * tst) * cp + tax * um * st * sp +
          ax * (tum * st + um * tst) * sp - tuy * oc - uy * toc;
    tdz = -(tup * st + up * tst) * cp - tuz * oc - uz * toc;
  } else {
    tdx = (tum * st + um * tst) * cp;
    tdy = (tum * st + um * tst) * sp;
    tdz = -tuz * oc - uz * toc;
  }
}

__device__ __attribute__((noinline)) void scatter_pair_nr_tan(
    double *vx, double *vy, double *vz, double *tx, double *ty, double *tz, const double *w,
    int I, int J, uint32_t kp, double coef_f_nmin_dV, double fa, double fb, int method,
    uint32_t cell, uint32_t step_lo, uint32_t c3, uint32_t k0, uint32_t k1,
    const double2 *n97tab, double dlnl) {
  using K = KMath<double>;
  const double vix = vx[I], viy = vy[I], viz = vz[I];
  const double vjx = vx[J], vjy = vy[J], vjz = vz[J];
  const double wi = w[I], wj = w[J];
  const double ux = vix - vjx, uy = viy - vjy, uz = viz - vjz;
  const double um2 = ux * ux + uy * uy + uz * uz;
  if (um2 == 0.0) return;
  const double um = K::sqrt_(um2);
  const double wmax = wi > wj ? wi : wj;
  const double s = (coef_f_nmin_dV * wmax) / (um2 * um);
  if (!(s > 0.0)) return;
  const U4 r = philox(kp, cell, step_lo, c3, k0, k1);
  double oc, st;
  sample_angle<double>(method, s, r.x, r.y, oc, st, n97tab);
  double sp, cp;
  K::sincos2pi(K::u(r.z), sp, cp);
  double dx, dy, dz;
  rotate_delta<double>(ux, uy, uz, st, oc, sp, cp, dx, dy, dz);
  const double u3 = unif64(r.w);
  bool ai = true, aj = true;
  if (wi < wj)
    aj = u3 <= wi / wj;
  else if (wj < wi)
    ai = u3 <= wj / wi;

  // tangent of u, |u| and s (s ~ lnL / |u|^3)
  const double tux = tx[I] - tx[J], tuy = ty[I] - ty[J], tuz = tz[I] - tz[J];
  const double tum = (ux * tux + uy * tuy + uz * tuz) / um;
  const double ts = s * (dlnl - 3.0 * tum / um);
  const double A = method == 0 ? 0.0 : n97_A_fast<double>(s, n97tab);
  double tdx, tdy, tdz;
  rot_tangent(method, ux, uy, uz, um, s, oc, st, sp, cp, K::u(r.x), A, tux, tuy, tuz, ts, tdx,
              tdy, tdz);
  if (ai) {
    vx[I] = vix + fa * dx;
    vy[I] = viy + fa * dy;
    vz[I] = viz + fa * dz;
    tx[I] += fa * tdx;
    ty[I] += fa * tdy;
    tz[I] += fa * tdz;
  }
  if (aj) {
    vx[J] = vjx - fb * dx;
    vy[J] = vjy - fb * dy;
    vz[J] = vjz - fb * dz;
    tx[J] -= fb * tdx;
    ty[J] -= fb * tdy;
    tz[J] -= fb * tdz;
  }
}

// ---------------------------------------------------------------------------
// Relativistic pair scatter (the paper gives none; see the design notes):
// rotation of the pair's centre-of-momentum momentum p* by the sampled angle,
// boosted back; s from the invariant rate with the CM deflection.
// Species (unweighted) masses ma, mb; u = gamma v.  All FP64.
// ---------------------------------------------------------------------------
__device__ __attribute__((noinline)) void scatter_pair_rel(
    double *vx, double *vy, double *vz, const double *w, int I, int J, uint32_t kp,
    double coef_f_nmin_dV, double ma, double mb, double c, int method, uint32_t cell,
    uint32_t step_lo, uint32_t c3, uint32_t k0, uint32_t k1, const double2 *n97tab) {
  const double c2 = c * c;
  const double uix = vx[I], uiy = vy[I], uiz = vz[I];
  const double ujx = vx[J], ujy = vy[J], ujz = vz[J];
  const double wi = w[I], wj = w[J];
  const double dx = uix - ujx, dy = uiy - ujy, dz = uiz - ujz;
  const double du2 = dx * dx + dy * dy + dz * dz;
  if (du2 == 0.0) return;
  const double gi = sqrt(1.0 + (uix * uix + uiy * uiy + uiz * uiz) / c2);
  const double gj = sqrt(1.0 + (ujx * ujx + ujy * ujy + ujz * ujz) / c2);
  const double dus = dx * (uix + ujx) + dy * (uiy + ujy) + dz * (uiz + ujz);
  const double dg = dus / (c2 * (gi + gj));  // gamma_i - gamma_j
  const double gr1 = 0.5 * (du2 / c2 - dg * dg);  // gamma_rel - 1
  if (!(gr1 > 0.0)) return;
  const double sq = sqrt(gr1 * (gr1 + 2.0));
  const double Mt = ma + mb;
  const double ecm = sqrt(Mt * Mt + 2.0 * ma * mb * gr1);  // E_cm / c^2
  const double etot = ma * gi + mb * gj;                   // E_tot / c^2
  const double pstar = ma * mb * c * sq / ecm;
  const double vM = c * sq / (gi * gj);
  const double vrel = c * sq / (1.0 + gr1);
  const double wmax = wi > wj ? wi : wj;
  const double s = coef_f_nmin_dV * wmax * vM / (pstar * pstar * vrel * vrel);
  if (!(s > 0.0)) return;
  // p_i* = (E_j p_i - E_i p_j)/E_cm + p_tot x (p_j x p_i) / (c^2 E_cm (E_tot + E_cm))
  const double mm = ma * mb;
  const double Qx = mm * (gj * dx - dg * ujx), Qy = mm * (gj * dy - dg * ujy),
               Qz = mm * (gj * dz - dg * ujz);
  const double ptx = ma * uix + mb * ujx, pty = ma * uiy + mb * ujy, ptz = ma * uiz + mb * ujz;
  const double jx = mm * (ujy * dz - ujz * dy), jy = mm * (ujz * dx - ujx * dz),
               jz = mm * (ujx * dy - ujy * dx);  // p_j x p_i
  const double crx = pty * jz - ptz * jy, cry = ptz * jx - ptx * jz, crz = ptx * jy - pty * jx;
  const double kb = 1.0 / (c2 * ecm * (etot + ecm));
  const double psx = Qx / ecm + crx * kb, psy = Qy / ecm + cry * kb, psz = Qz / ecm + crz * kb;
  const U4 r = philox(kp, cell, step_lo, c3, k0, k1);
  double oc, st;
  sample_angle<double>(method, s, r.x, r.y, oc, st, n97tab);
  double sp, cp;
  KMath<double>::sincos2pi(unif64(r.z), sp, cp);
  double Dx, Dy, Dz;
  rotate_delta<double>(psx, psy, psz, st, oc, sp, cp, Dx, Dy, Dz);
  const double Dp = (Dx * ptx + Dy * pty + Dz * ptz) * kb;
  const double px = Dx + Dp * ptx, py = Dy + Dp * pty, pz = Dz + Dp * ptz;
  const double u3 = unif64(r.w);
  bool ai = true, aj = true;
  if (wi < wj)
    aj = u3 <= wi / wj;
  else if (wj < wi)
    ai = u3 <= wj / wi;
  if (ai) {
    vx[I] = uix + px / ma;
    vy[I] = uiy + py / ma;
    vz[I] = uiz + pz / ma;
  }
  if (aj) {
    vx[J] = ujx - px / mb;
    vy[J] = ujy - py / mb;
    vz[J] = ujz - pz / mb;
  }
}

// ---------------------------------------------------------------------------
// Pair energy correction helpers (Eqs. (19)-(23); Appendix A)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pair_K_nr(double m1, double m2, double ax, double ay, double az,
                                            double bx, double by, double bz) {
  const double mu = m1 * m2 / (m1 + m2);
  const double rx = ax - bx, ry = ay - by, rz = az - bz;
  return 0.5 * mu * (rx * rx + ry * ry + rz * rz);
}

// relativistic CM kinetic energy of the weighted pair
__device__ __forceinline__ double pair_K_rel(double m1, double m2, double ax, double ay, double az,
                                             double bx, double by, double bz, double c) {
  const double c2 = c * c;
  const double dx = ax - bx, dy = ay - by, dz = az - bz;
  const double du2 = dx * dx + dy * dy + dz * dz;
  const double g1 = sqrt(1.0 + (ax * ax + ay * ay + az * az) / c2);
  const double g2 = sqrt(1.0 + (bx * bx + by * by + bz * bz) / c2);
  const double dus = dx * (ax + bx) + dy * (ay + by) + dz * (az + bz);
  const double dg = dus / (c2 * (g1 + g2));
  double gr1 = 0.5 * (du2 / c2 - dg * dg);
  if (gr1 < 0.0) gr1 = 0.0;
  const double Mt = m1 + m2;
  const double ecm = sqrt(Mt * Mt + 2.0 * m1 * m2 * gr1);
  return 2.0 * m1 * m2 * c2 * gr1 / (ecm + Mt);
}

struct RelPair {
  double p1x, p1y, p1z, p2x, p2y, p2z, dx, dy, dz, E1, E2, m1, m2, c2;
  __device__ __forceinline__ void init(double m1_, double m2_, double ax, double ay, double az,
                                       double bx, double by, double bz, double c) {
    m1 = m1_;
    m2 = m2_;
    c2 = c * c;
    dx = ax - bx;
    dy = ay - by;
    dz = az - bz;
    p1x = m1 * ax;
    p1y = m1 * ay;
    p1z = m1 * az;
    p2x = m2 * bx;
    p2y = m2 * by;
    p2z = m2 * bz;
    E1 = m1 * c2 * sqrt(1.0 + (ax * ax + ay * ay + az * az) / c2);
    E2 = m2 * c2 * sqrt(1.0 + (bx * bx + by * by + bz * bz) / c2);
  }
  // E1(alpha) + E2(alpha) - E1 - E2 (without U) and its derivative
  __device__ __forceinline__ double h0(double al, double &dh) const {
    const double a1x = p1x + al * dx, a1y = p1y + al * dy, a1z = p1z + al * dz;
    const double a2x = p2x - al * dx, a2y = p2y - al * dy, a2z = p2z - al * dz;
    const double E1n = sqrt(m1 * m1 * c2 * c2 + c2 * (a1x * a1x + a1y * a1y + a1z * a1z));
    const double E2n = sqrt(m2 * m2 * c2 * c2 + c2 * (a2x * a2x + a2y * a2y + a2z * a2z));
    const double p1d = p1x * dx + p1y * dy + p1z * dz;
    const double p2d = p2x * dx + p2y * dy + p2z * dz;
    const double d2 = dx * dx + dy * dy + dz * dz;
    dh = c2 * ((a1x * dx + a1y * dy + a1z * dz) / E1n - (a2x * dx + a2y * dy + a2z * dz) / E2n);
    return c2 * ((2.0 * al * p1d + al * al * d2) / (E1n + E1) +
                 (-2.0 * al * p2d + al * al * d2) / (E2n + E2));
  }
  __device__ __forceinline__ double mu() const { return m1 * m2 / (m1 + m2); }
};

// alpha with E1' + E2' = E_tot - U on the branch alpha > -mu_R (Eq. (A.5));
// the caller has checked that a root exists (h(-mu_R) <= 0 when U > 0).
__device__ double rel_alpha(const RelPair &R, double U) {
  const double muR = R.mu();
  double dh, lo, hi;
  if (U > 0.0) {
    lo = -muR;
    hi = 0.0;
  } else {
    lo = 0.0;
    hi = muR;
    for (int it = 0; it < 200 && R.h0(hi, dh) + U < 0.0; ++it) hi *= 2.0;
  }
  const double d2 = R.dx * R.dx + R.dy * R.dy + R.dz * R.dz;
  const double x = U / (0.5 * muR * d2);
  double a = (x < 1.0) ? muR * (-x / (1.0 + sqrt(1.0 - x))) : 0.5 * (lo + hi);
  if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
  const double eps = 2.220446049250313e-16;
  for (int it = 0; it < 200; ++it) {
    const double h = R.h0(a, dh) + U;
    if (h == 0.0) break;
    if (h > 0.0)
      hi = a;
    else
      lo = a;
    if (hi - lo <= 4.0 * eps * fabs(a)) break;
    double an = a - h / dh;
    if (!(an > lo && an < hi)) an = 0.5 * (lo + hi);
    if (fabs(an - a) <= 0.5 * eps * fabs(a)) {
      a = an;
      break;
    }
    a = an;
  }
  return a;
}

// ---------------------------------------------------------------------------
// Random permutation of one species list: ordered by (Philox word, index).
// out[q] = cell-local particle index (off + item).
// ---------------------------------------------------------------------------
template <int TPC, int PPT, bool G>
__device__ __forceinline__ void shuffle_species(const CellMem &M, int ns, int off, uint32_t cell,
                                                uint32_t step_lo, uint32_t c3, uint32_t k0,
                                                uint32_t k1, uint16_t *out, uint32_t *wsum,
                                                uint32_t *maxocc) {
  uint32_t *key = M.key;
  uint32_t *cnt = M.cnt;
  const int t = threadIdx.x;
  for (int q = t; 4 * q < ns; q += TPC) {
    const U4 r = philox((uint32_t)q, cell, step_lo, c3, k0, k1);
    const int i = 4 * q;
    key[i] = r.x;
    if (i + 1 < ns) key[i + 1] = r.y;
    if (i + 2 < ns) key[i + 2] = r.z;
    if (i + 3 < ns) key[i + 3] = r.w;
  }
  // the sort's bucket counters are cleared under the same barrier
  for (int i = t; i < ns; i += TPC) cnt[i] = 0u;
  if (t == 0) *maxocc = 0u;
  __syncthreads();
  const uint64_t nsu = (uint64_t)ns;
  if constexpr (!G) {
    key_rank_sort<TPC, PPT>(
        ns, key, cnt, M.mem, out, wsum,
        [&](int, uint32_t k) -> uint32_t { return (uint32_t)(((uint64_t)k * nsu) >> 32); },
        [&](int i) -> int { return i + off; });
  } else {
    bucket_rank_sort<TPC, PPT, G, true>(
        ns, cnt, M.mem, out, wsum, maxocc,
        [&](int i) -> uint32_t { return (uint32_t)(((uint64_t)key[i] * nsu) >> 32); },
        [&](int o, int i) -> bool {
          const uint32_t ko = key[o], ki = key[i];
          return ko < ki || (ko == ki && o < i);
        },
        M.slotbuf, [&](int i) -> int { return i + off; });
  }
}

// The random permutations of both species of an inter-species collision in
// one LDS sort: species a's items take buckets [0, na) and species b's
// [na, na + nb), so items of different species are never compared and each
// species comes out sorted by (Philox word, index) exactly as alone.
// out[0..na) = species a, out[na..na+nb) = species b (cell-local indices).
template <int TPC, int PPT, bool G>
__device__ __forceinline__ void shuffle_two(const CellMem &M, int na, int oa, int nb, int ob,
                                            uint32_t cell, uint32_t step_lo, uint32_t c3a,
                                            uint32_t c3b, uint32_t k0, uint32_t k1,
                                            uint16_t *out, uint32_t *wsum, uint32_t *maxocc) {
  uint32_t *key = M.key;
  const int t = threadIdx.x;
  const int n = na + nb;
  const int qa = (na + 3) >> 2;
  for (int q = t; q < qa + ((nb + 3) >> 2); q += TPC) {
    const bool sa = q < qa;
    const int qq = sa ? q : q - qa;
    const U4 r = philox((uint32_t)qq, cell, step_lo, sa ? c3a : c3b, k0, k1);
    const int ns = sa ? na : nb;
    const int i = 4 * qq;
    uint32_t *kk = key + (sa ? 0 : na);
    kk[i] = r.x;
    if (i + 1 < ns) kk[i + 1] = r.y;
    if (i + 2 < ns) kk[i + 2] = r.z;
    if (i + 3 < ns) kk[i + 3] = r.w;
  }
  // the sort's bucket counters are cleared under the same barrier
  for (int i = t; i < n; i += TPC) M.cnt[i] = 0u;
  if (t == 0) *maxocc = 0u;
  __syncthreads();
  const uint64_t nau = (uint64_t)na, nbu = (uint64_t)nb;
  if constexpr (!G) {
    key_rank_sort<TPC, PPT>(
        n, key, M.cnt, M.mem, out, wsum,
        [&](int i, uint32_t k) -> uint32_t {
          return i < na ? (uint32_t)(((uint64_t)k * nau) >> 32)
                        : (uint32_t)na + (uint32_t)(((uint64_t)k * nbu) >> 32);
        },
        [&](int i) -> int { return i < na ? oa + i : ob + (i - na); });
  } else {
    bucket_rank_sort<TPC, PPT, G, true>(
        n, M.cnt, M.mem, out, wsum, maxocc,
        [&](int i) -> uint32_t {
          return i < na ? (uint32_t)(((uint64_t)key[i] * nau) >> 32)
                        : (uint32_t)na + (uint32_t)(((uint64_t)key[i] * nbu) >> 32);
        },
        [&](int o, int i) -> bool {
          const uint32_t ko = key[o], ki = key[i];
          return ko < ki || (ko == ki && o < i);
        },
        M.slotbuf, [&](int i) -> int { return i < na ? oa + i : ob + (i - na); });
  }
}

// Descending-weight order of ns particles, stable in list position (Alg. 1,
// optional step): the particles are L[0..ns) (cell-local indices), or, with
// L == nullptr, off, off+1, ..., off+ns-1.  O receives cell-local indices.
// lo < hi are the bit patterns of the smallest and largest weight.
// weight order: a bucket above this occupancy switches to the per-value pass
// (at most MAX_WEIGHT_VALUES distinct values among the crowded ties)
constexpr uint32_t OCC_LIMIT = 48;
constexpr int MAX_WEIGHT_VALUES = 32;

template <int TPC, int PPT, bool G>
__device__ __forceinline__ void weight_sort(const CellMem &M, int ns, const uint16_t *L, int off,
                                            uint16_t *O, uint64_t lo, uint64_t hi,
                                            uint32_t *wsum, uint32_t *maxocc) {
  const int t = threadIdx.x;
  const double scale = (double)ns / ((double)(hi - lo) + 1.0);
  const double *w = M.w;
  auto item = [&](int q) -> int { return L ? (int)L[q] : off + q; };
  auto before = [&](int o, int q) -> bool {
    const double wo = w[item(o)], wq = w[item(q)];
    return wo > wq || (wo == wq && o < q);
  };
  const uint32_t occ = bucket_rank_sort<TPC, PPT, G>(
      ns, M.cnt, M.mem, O, wsum, maxocc,
      [&](int q) -> uint32_t {
        const uint64_t b = (uint64_t)__double_as_longlong(w[item(q)]);
        const uint32_t k = (uint32_t)((double)(hi - b) * scale);
        return k < (uint32_t)ns ? k : (uint32_t)(ns - 1);
      },
      before, M.slotbuf, IdentityMap(), OCC_LIMIT);
  if (occ > OCC_LIMIT) {
    // Crowded buckets come from ties, usually among few distinct weights:
    // ranking inside a bucket would cost its occupancy squared.  Instead,
    // one pass per distinct weight value, largest first, appends the items
    // of that weight in list order (each thread scans a contiguous chunk of
    // the list, so thread order is list order).
    auto wbits = [&](int q) -> uint64_t {
      return (uint64_t)__double_as_longlong(w[item(q)]);  // (w > 0: bit order = value order)
    };
    const int C = (ns + TPC - 1) / TPC;
    const int q0 = t * C, q1 = q0 + C < ns ? q0 + C : ns;
    uint64_t *redu = reinterpret_cast<uint64_t *>(M.cnt);  // (free: the sort stopped early)
    uint64_t cur = hi;
    int placed = 0;
    for (int round = 0; round < MAX_WEIGHT_VALUES && placed < ns; ++round) {
      uint32_t c = 0;
      for (int q = q0; q < q1; ++q) c += wbits(q) == cur ? 1u : 0u;
      uint32_t tot;
      uint32_t pos = (uint32_t)placed + block_excl_scan1<TPC, G>(c, wsum, tot);
      uint64_t lo1[1] = {~0ull}, nxt[1] = {0ull};
      for (int q = q0; q < q1; ++q) {
        const uint64_t b = wbits(q);
        if (b == cur)
          O[pos++] = (uint16_t)q;
        else if (b < cur && b > nxt[0])
          nxt[0] = b;
      }
      block_minmax_u64<TPC, 1, G>(lo1, nxt, redu);
      placed += (int)tot;
      cur = nxt[0];
    }
    if (placed < ns) {
      // many distinct values among the ties: a bitonic network
      int P = 1;
      while (P < ns) P <<= 1;
      for (int i = t; i < P; i += TPC) M.mem[i] = i < ns ? (uint16_t)i : (uint16_t)0xFFFF;
      __syncthreads();
      bitonic_sort_ids<TPC>(M.mem, P, before);
      for (int q = t; q < ns; q += TPC) O[q] = M.mem[q];
    }
    __syncthreads();
  }
  for (int q = t; q < ns; q += TPC) O[q] = (uint16_t)item(O[q]);
  __syncthreads();
}

// weight classes of a species, decided once per cell
enum : int { WORDER_EQUAL = 0, WORDER_DISTINCT = 1, WORDER_TIES = 2 };

// Owner loop: particle e = threadIdx.x + j*TPC, j < PPT, unrolled when the
// per-thread count is small.
template <int TPC, int PPT, bool UNROLL, class F>
__device__ __forceinline__ void for_owned(int n, F &&f) {
  if constexpr (UNROLL) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int e = threadIdx.x + j * TPC;
      if (e < n) f(j, e);
    }
  } else {
    for (int j = 0; j < PPT; ++j) {
      const int e = threadIdx.x + j * TPC;
      if (e >= n) break;
      f(j, e);
    }
  }
}

// ---------------------------------------------------------------------------
// The kernel
// ---------------------------------------------------------------------------
// PAIRING: PAIR_ORDER_N, PAIR_NXN (every pair once, Sec. 3.1) or
// PAIR_DUPLICITY (the order-N pairs with Higginson et al.'s duplicity s);
// the other pairings have their own instantiations, so the order-N kernels
// carry none of their registers
template <int TPC, int CAP, typename KR, bool REL, int LAY, bool TAN = false, bool DIAG = false,
          int PAIRING = PAIR_ORDER_N>
__global__ void __launch_bounds__(TPC, min_waves(TPC, CAP, LAY, sizeof(KR) == 8, TAN))
    collide_kernel(CollideArgs A) {
  constexpr int PPT = CAP / TPC;
  constexpr int NW = TPC / WAVE;
  constexpr bool GL = LAY == LAYOUT_GLOBAL;
  constexpr bool BIG = GL;  // snapshot in memory, runtime owner loops
  static_assert(CAP % TPC == 0 && TPC % WAVE == 0, "bad variant");
  static_assert(!(REL && LAY == LAYOUT_COMPACT), "REL needs the full pair buffer");
  // the descending-weight order has an LDS home up to 1024 particles in the
  // compact layout (above, its room would cost a second resident cell per
  // CU); there a plan's order is read from HBM
  constexpr bool HAS_WORD = LAY != LAYOUT_COMPACT || CAP <= 1024;
  // weights: in LDS except in the compact layout above 1024 particles, where
  // their room would cost a resident cell per CU (read from HBM there)
  constexpr bool W_LDS = LAY != LAYOUT_COMPACT || CAP <= 1024;
  // pairs of intra-species collisions run as one pass (not in the tangent,
  // relativistic, diagnostic and N x N forms)
  constexpr bool NXN = PAIRING == PAIR_NXN;
  constexpr bool DUP = PAIRING == PAIR_DUPLICITY;
  constexpr bool DUAL = !TAN && !REL && !DIAG && PAIRING == PAIR_ORDER_N;
  static_assert(PAIRING == PAIR_ORDER_N || !(TAN || DIAG),
                "the N x N and duplicity pairings have no tangent or diagnostic form");
  static_assert(!GL || TPC <= 512, "the global layout runs at most 8 waves per cell");
  static_assert(!TAN || (!REL && sizeof(KR) == 8 && LAY != LAYOUT_COMPACT && !DIAG),
                "the tangent form is FP64 non-relativistic, without diagnostics");
  // FP32 kinematics in the compact layout from 1024 particles up: the N97
  // table in LDS as the FP32 values its uses take (room the smaller
  // variants would pay for in resident cells)
  constexpr bool TAB_LDS = sizeof(KR) == 4 && !REL && LAY == LAYOUT_COMPACT && CAP >= 1024;
  __shared__ float2 s_tab[TAB_LDS ? N97_TN : 1];
  if constexpr (TAB_LDS) {
    for (int i = threadIdx.x; i < N97_TN; i += TPC)
      s_tab[i] = make_float2((float)A.n97[i].x, (float)A.n97[i].y);
  }
  __shared__ double red[2 * 6 * NW];
  uint64_t *redu = reinterpret_cast<uint64_t *>(red);
  __shared__ uint32_t wsum[NW];
  __shared__ uint32_t maxocc;
  __shared__ int s_so[MCC_MAX_SPECIES + 1];
  __shared__ int s_bad;
  __shared__ long long s_cb;  // first particle of the cell
  __shared__ uint32_t s_next[2];  // the next work-list entry (double-buffered)
  // per species: sum w, sum w^2, the weight range (bit patterns) and class
  __shared__ unsigned long long s_wlo[MCC_MAX_SPECIES], s_whi[MCC_MAX_SPECIES];
  __shared__ double s_sw[MCC_MAX_SPECIES], s_sw2[MCC_MAX_SPECIES];
  __shared__ int s_wflag[MCC_MAX_SPECIES];
  __shared__ unsigned long long s_st[4];  // pairs, correction pairs, failures, collisions
  // the workgroup's totals of s_st and s_sd over its cells (thread 0), added
  // to the caller's statistics once at the end: one atomic per cell and
  // counter would serialize the whole grid on four addresses
  __shared__ unsigned long long s_acc[4];
  __shared__ double s_accd[2];
  __shared__ double s_sd[2];              // diagnostics maxima
  __shared__ int s_ncut[2];
  __shared__ double s_res[2];
  __shared__ double s_tres[2];  // tangent form: tangent of the residuals
  __shared__ int s_used[2];
  __shared__ CollConst s_cc[2];  // the collision(s) of the current pass
  // bucket counters stay in LDS in every layout: global atomics complete in
  // L2, and later plain loads could hit stale L1 lines
  __shared__ __attribute__((aligned(16))) uint32_t lcnt[CAP + 2];
#ifdef MCC_PHASE_TIMING
  // profiling build: thread 0 charges the clock ticks between phase marks
  __shared__ unsigned long long s_ph[16];
  uint64_t ph_last = 0;
  int ph_cur = 15;
  if (threadIdx.x < 16) s_ph[threadIdx.x] = 0;
#define MCC_PHASE(i)                                     \
  do {                                                   \
    if (threadIdx.x == 0) {                              \
      const uint64_t now_ = clock64();                   \
      if (ph_last) s_ph[ph_cur] += now_ - ph_last;       \
      ph_last = now_;                                    \
      ph_cur = (i);                                      \
    }                                                    \
  } while (0)
#else
#define MCC_PHASE(i) ((void)0)
#endif

  CellMem M;
  double *wdst = nullptr;  // where the load phase copies the weights (LDS layout)
  M.cnt = lcnt;
  M.slotbuf = nullptr;
  M.bx = M.by = M.bz = nullptr;
  if constexpr (LAY == LAYOUT_LDS) {
    __shared__ double lv[4 * CAP];
    __shared__ uint64_t lscr[CAP + 1];
    __shared__ __attribute__((aligned(16))) uint16_t lidx[6 * CAP + 4];
    M.vx = lv;
    M.vy = lv + CAP;
    M.vz = lv + 2 * CAP;
    wdst = lv + 3 * CAP;
    M.w = wdst;
    M.key = reinterpret_cast<uint32_t *>(lscr);
    M.kbuf = reinterpret_cast<double *>(lscr);
    M.list0 = lidx;
    M.list1 = lidx + CAP;
    M.ord0 = lidx + 2 * CAP;
    M.ord1 = lidx + 3 * CAP;
    M.mem = lidx + 4 * CAP;
    M.word = lidx + 5 * CAP;
    if constexpr (TAN) {
      __shared__ double lt[7 * CAP];
      M.tx = lt;
      M.ty = lt + CAP;
      M.tz = lt + 2 * CAP;
      M.btx = lt + 3 * CAP;
      M.bty = lt + 4 * CAP;
      M.btz = lt + 5 * CAP;
      M.kdot = lt + 6 * CAP;
    }
  } else if constexpr (LAY == LAYOUT_COMPACT) {
    __shared__ double lv[(W_LDS ? 4 : 3) * CAP];
    __shared__ __attribute__((aligned(16))) uint16_t lidx[(HAS_WORD ? 6 : 5) * CAP + 4];
    M.vx = lv;
    M.vy = lv + CAP;
    M.vz = lv + 2 * CAP;
    if constexpr (W_LDS) {
      wdst = lv + 3 * CAP;
      M.w = wdst;
    }
    M.list0 = lidx;
    M.list1 = lidx + CAP;
    M.ord0 = lidx + 2 * CAP;
    M.ord1 = lidx + 3 * CAP;
    M.mem = lidx + 4 * CAP;
    // shuffle keys live in ord0/ord1 (dead until the weight order); the pair
    // energies live in the bucket counters (dead after the weight order)
    M.key = reinterpret_cast<uint32_t *>(lidx + 2 * CAP);
    M.kbuf = reinterpret_cast<double *>(lcnt);
    M.word = HAS_WORD ? lidx + 5 * CAP : M.list0;  // (list0: scratch of the plan's weight pass)
  } else {
    char *base = A.big_scratch + (uint64_t)blockIdx.x * A.big_stride;
    double *dv = reinterpret_cast<double *>(base);
    M.vx = dv;
    M.vy = dv + CAP;
    M.vz = dv + 2 * CAP;
    wdst = dv + 3 * CAP;
    M.w = wdst;
    M.bx = dv + 4 * CAP;
    M.by = dv + 5 * CAP;
    M.bz = dv + 6 * CAP;
    M.kbuf = dv + 7 * CAP;                                       // CAP doubles
    M.key = reinterpret_cast<uint32_t *>(dv + 8 * CAP);          // CAP u32
    M.slotbuf = M.key + CAP;                                     // CAP u32
    uint16_t *ix = reinterpret_cast<uint16_t *>(M.slotbuf + CAP);
    M.list0 = ix;
    M.list1 = ix + CAP;
    M.ord0 = ix + 2 * CAP;
    M.ord1 = ix + 3 * CAP;
    M.mem = ix + 4 * CAP;
    M.word = ix + 5 * CAP;
    if constexpr (TAN) {
      double *lt = reinterpret_cast<double *>(base + big_stride_bytes(CAP, false));
      M.tx = lt;
      M.ty = lt + CAP;
      M.tz = lt + 2 * CAP;
      M.btx = lt + 3 * CAP;
      M.bty = lt + 4 * CAP;
      M.btz = lt + 5 * CAP;
      M.kdot = lt + 6 * CAP;
    }
  }

  uint16_t *const wbase = M.word;  // LDS home of the descending-weight order
  const int t = threadIdx.x;
  const int S = A.S;
  const uint64_t step = A.step_dev ? *A.step_dev : A.step;
  const uint32_t step_lo = (uint32_t)step;
  const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
  const uint32_t count = *A.cell_count;
  // Cells are handed out at run time, so no workgroup idles while another
  // still holds several.  The work list is split into NQ interleaved queues
  // (queue q: entries q, q + NQ, q + 2 NQ, ...) whose counters sit in
  // separate 256-byte lines, so claims on different queues do not serialize;
  // the first entries of a queue go to its workgroups in order, the rest are
  // claimed one at a time (qctr[0]).  qctr[1] counts the workgroups of the
  // queue that ran out; the last one resets both for the next launch.
  const uint32_t NQ = gridDim.x < WORK_QUEUES ? gridDim.x : WORK_QUEUES;
  const uint32_t q = blockIdx.x % NQ;
  const uint32_t nq = (gridDim.x - q + NQ - 1) / NQ;  // workgroups on queue q
  uint32_t *const qctr = A.work + q * WORK_STRIDE;
  int par = 0;
  // per-species and per-collision constants in LDS (indexed at run time)

  if (t == 0) {
    for (int i = 0; i < 4; ++i) s_acc[i] = 0ull;
    s_accd[0] = s_accd[1] = 0.0;
  }

  for (uint32_t li = q + NQ * (blockIdx.x / NQ); li < count;) {
    MCC_PHASE(0);  // header and staging
    // Wave priority: the phases that end in workgroup barriers (staging,
    // shuffles, reductions, cut-off, corrections) run at priority 1, the pair
    // scatter, long runs of arithmetic between two barriers, at 0.  A SIMD then
    // issues first for the waves that hold a barrier of their cell, and fills
    // the gaps with other cells' scatter.
    __builtin_amdgcn_s_setprio(1);
    const int cell = A.cell_list[li];
    // the next entry, claimed now and needed only when this cell is done
    uint32_t claim = 0;
    if (t == 0) claim = atomicAdd(qctr, 1u);
    // cell header: the S + 1 segment offsets, one per lane of wave 0 (one
    // load latency), validated once
    if (t < WAVE) {
      const int64_t o = t <= S ? A.offsets[(int64_t)cell * S + t] : 0;
      const int64_t cb = __shfl(o, 0), ce = __shfl(o, S);
      const int64_t o1 = __shfl_down(o, 1);
      int bad = (t == 0 && !(cb >= 0 && ce >= cb && ce <= A.n)) ||
                (t < S && (o < cb || o1 < o || o1 > ce));
      bad = __ballot(bad) ? 1 : 0;
      if (!bad && ce - cb > CAP) bad = 2;
      if (t <= S) s_so[t] = (int)(o - cb);
      if (t == 0) {
        if (bad) atomicCAS(A.err, 0, bad);
        s_bad = bad;
        s_cb = cb;
        for (int q = 0; q < 4; ++q) s_st[q] = 0ull;
        s_sd[0] = s_sd[1] = 0.0;
      }
    }
    __syncthreads();
    if (s_bad) {
      if (t == 0) s_next[par] = q + NQ * (nq + claim);
      __syncthreads();
      li = uni((int)s_next[par]);  // (the next write goes to the other slot)
      par ^= 1;
      continue;  // uniform over the workgroup
    }
    const int64_t cb = uni(s_cb);
    const int n = uni(s_so[S]);
    const double dV = A.cell_volume ? A.cell_volume[cell] : A.dV;
    if constexpr (!W_LDS) M.w = A.w + cb;
    const bool prep_read = A.corr && A.prep_mode == PREP_READ;

    if constexpr (!GL) {
      // straight from HBM into LDS (no registers), every copy of the cell in
      // flight at once: the cell costs one HBM latency
      lds_copy<TPC>(A.vx + cb, M.vx, 2 * n);
      lds_copy<TPC>(A.vy + cb, M.vy, 2 * n);
      lds_copy<TPC>(A.vz + cb, M.vz, 2 * n);
      if constexpr (W_LDS) lds_copy<TPC>(A.w + cb, wdst, 2 * n);
      if constexpr (TAN) {
        lds_copy<TPC>(A.tx + cb, M.tx, 2 * n);
        lds_copy<TPC>(A.ty + cb, M.ty, 2 * n);
        lds_copy<TPC>(A.tz + cb, M.tz, 2 * n);
      }
      SpeciesPrep P{};
      if (prep_read && t < S) P = A.prep[(int64_t)cell * S + t];
      if (prep_read) {
        // the plan's weight data of this cell; its u16 word order is copied
        // in whole dwords from the even entry at or below cb, so the cell's
        // first entry lands at (cb & 1)
        if constexpr (HAS_WORD) {
          const int odd0 = (int)(cb & 1);
          lds_copy<TPC>(A.prep_word + (cb - odd0), wbase, (n + odd0 + 1) >> 1);
          M.word = wbase + odd0;
        }
      } else if constexpr (HAS_WORD) {
        M.word = wbase;
      }
      lds_copy_wait();
      if (prep_read && t < S) {
        s_sw[t] = P.sw;
        s_sw2[t] = P.sw2;
        s_wlo[t] = P.lo;
        s_whi[t] = P.hi;
        s_wflag[t] = P.flag;
      }
      __syncthreads();
    } else {
      for (int e = t; e < n; e += TPC) {
        M.vx[e] = A.vx[cb + e];
        M.vy[e] = A.vy[cb + e];
        M.vz[e] = A.vz[cb + e];
        if constexpr (W_LDS) wdst[e] = A.w[cb + e];
        if constexpr (TAN) {
          M.tx[e] = A.tx[cb + e];
          M.ty[e] = A.ty[cb + e];
          M.tz[e] = A.tz[cb + e];
        }
      }
      __syncthreads();
      if (prep_read) {
        // the plan's weight data of this cell
        if (t < S) {
          const SpeciesPrep P = A.prep[(int64_t)cell * S + t];
          s_sw[t] = P.sw;
          s_sw2[t] = P.sw2;
          s_wlo[t] = P.lo;
          s_whi[t] = P.hi;
          s_wflag[t] = P.flag;
        }
        if constexpr (HAS_WORD) {
          for (int e = t; e < n; e += TPC) M.word[e] = A.prep_word[cb + e];
        }
        __syncthreads();
      }
    }
    if (!prep_read && A.corr) {
      // per species, once per cell: sum w and sum w^2 (the denominator of
      // Eq. (17) and the mean weights of Eq. (24)), the weight range, and
      // for unequal weights the descending-weight order, which is the
      // correction order of every collision when no two weights are equal
      for (int sp = 0; sp < S; ++sp) {
        const int o = s_so[sp], ns = s_so[sp + 1] - o;
        CSum<2> acc;  // compensated, as every per-cell moment sum
        acc.zero();
        uint64_t lo[1] = {~0ull}, hi[1] = {0ull};
        for (int e = o + t; e < o + ns; e += TPC) {
          const double we = M.w[e];
          acc.add(0, we);
          acc.add(1, we * we);
          const uint64_t bits = (uint64_t)__double_as_longlong(we);
          lo[0] = bits < lo[0] ? bits : lo[0];
          hi[0] = bits > hi[0] ? bits : hi[0];
        }
        double tot[2];
        block_csum<TPC, 2>(acc, red, tot);
        block_minmax_u64<TPC, 1>(lo, hi, redu);
        int flag = WORDER_EQUAL;
        if (A.sortw && ns >= 2 && lo[0] != hi[0]) {
          flag = WORDER_TIES;
          // without an LDS home the order is kept only by a plan's weight
          // pass (M.word is list0 then, free before any collision)
          if (HAS_WORD || A.prep_mode == PREP_WRITE) {
            weight_sort<TPC, PPT, GL>(M, ns, nullptr, o, M.word + o, lo[0], hi[0], wsum,
                                      &maxocc);
            int tie = 0;
            for (int q = t; q + 1 < ns; q += TPC)
              if (M.w[M.word[o + q]] == M.w[M.word[o + q + 1]]) tie = 1;
            flag = __syncthreads_or(tie) ? WORDER_TIES : WORDER_DISTINCT;
          }
        }
        if (t == 0) {
          s_sw[sp] = tot[0];
          s_sw2[sp] = tot[1];
          s_wlo[sp] = lo[0];
          s_whi[sp] = hi[0];
          s_wflag[sp] = flag;
          if (A.prep_mode == PREP_WRITE)
            A.prep[(int64_t)cell * S + sp] = SpeciesPrep{tot[0], tot[1], lo[0], hi[0], flag, 0};
        }
      }
      __syncthreads();
      if (A.prep_mode == PREP_WRITE) {
        for (int e = t; e < n; e += TPC) A.prep_word[cb + e] = M.word[e];
      }
    }

    for (int k = 0, kn = 0; k < A.n_coll; k = kn) {
      kn = k + 1;
      const int a = uni(A.coll[k].a);
      const bool intra = a == uni(A.coll[k].b);
      const int oa = uni(s_so[a]), na = uni(s_so[a + 1]) - oa;
      if (intra && na < 2) continue;
      // Two consecutive intra-species collisions of different species touch
      // disjoint particles, so they commute and run as one pass ("dual"):
      // each keeps its own random numbers, momentum restore, energy
      // correction and failure decision; species b is then the second one's.
      bool dual = false;
      int b = uni(A.coll[k].b);
      if constexpr (DUAL) {
        if (intra && k + 1 < A.n_coll) {
          const int a2 = uni(A.coll[k + 1].a);
          if (a2 == uni(A.coll[k + 1].b) && a2 != a && uni(s_so[a2 + 1]) - uni(s_so[a2]) >= 2) {
            dual = true;
            b = a2;
            kn = k + 2;
          }
        }
      }
      const int ob = uni(s_so[b]), nb = uni(s_so[b + 1]) - ob;
      if (!intra && (na == 0 || nb == 0)) continue;
      const bool two = !intra || dual;  // a second species takes part
      const double ma = A.mass[a], mb = A.mass[b];
      // the constants the scatter reads (written before the shuffles' barriers;
      // the previous pass read them before its scatter barrier)
      if (t == 0) {
        s_cc[0] = A.coll[k];
        if (dual) s_cc[1] = A.coll[k + 1];
      }
      const CollConst &C = s_cc[0];

      MCC_PHASE(1);  // snapshot and shuffles
      // pre-scatter snapshot (Alg. 1, first step)
      double bx[GL ? 1 : PPT], by[GL ? 1 : PPT], bz[GL ? 1 : PPT];
      if constexpr (!GL && !TAN) {
        // every owned slot (those past n hold LDS contents nobody uses)
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
          const int e = t + j * TPC;
          bx[j] = M.vx[e];
          by[j] = M.vy[e];
          bz[j] = M.vz[e];
        }
      } else
      for_owned<TPC, PPT, !GL>(n, [&](int j, int e) {
        if (e < n) {
          if constexpr (BIG) {
            M.bx[e] = M.vx[e];
            M.by[e] = M.vy[e];
            M.bz[e] = M.vz[e];
          } else {
            bx[j] = M.vx[e];
            by[j] = M.vy[e];
            bz[j] = M.vz[e];
          }
          if constexpr (TAN) {
            M.btx[e] = M.tx[e];
            M.bty[e] = M.ty[e];
            M.btz[e] = M.tz[e];
          }
        }
      });
#define SNAPX(j, e) (BIG ? M.bx[e] : bx[BIG ? 0 : (j)])
#define SNAPY(j, e) (BIG ? M.by[e] : by[BIG ? 0 : (j)])
#define SNAPZ(j, e) (BIG ? M.bz[e] : bz[BIG ? 0 : (j)])

      // random binary pairs (Fig. 1)
      // L0, L1: the shuffled lists of species a and b
      const uint16_t *L0 = M.list0, *L1 = M.list0 + na;
      if (!two)
        shuffle_species<TPC, PPT, GL>(M, na, oa, (uint32_t)cell, step_lo,
                                      ctr3(step, k, PURPOSE_SHUFFLE0 + 0), k0, k1, M.list0,
                                      wsum, &maxocc);
      else
        shuffle_two<TPC, PPT, GL>(M, na, oa, nb, ob, (uint32_t)cell, step_lo,
                                  ctr3(step, k, PURPOSE_SHUFFLE0 + 0),
                                  dual ? ctr3(step, k + 1, PURPOSE_SHUFFLE0 + 0)
                                       : ctr3(step, k, PURPOSE_SHUFFLE0 + 1),
                                  k0, k1, M.list0, wsum, &maxocc);

      // scatter (Sec. 3.2 pairing) in rounds of disjoint pairs:
      //  intra, even N: one round (L0,L1),(L2,L3),...
      //  intra, odd N : the triple (L0,L1),(L1,L2),(L2,L0) at s/2 in three
      //                 rounds; the regular pairs (L3,L4),... in round 0
      //  inter        : pair k = (big[k], small[k mod N_min]) in rounds of N_min
      MCC_PHASE(2);  // scatter
      __builtin_amdgcn_s_setprio(0);
      const uint32_t c3p = ctr3(step, k, PURPOSE_PAIR);
      const bool abig = na >= nb;
      const int Nmax = abig ? na : nb, Nmin = abig ? nb : na;
      const double nmin = intra ? (double)(na - 1) : (double)Nmin;
      // N_min / dV of each collision of the pass (once per pass, not per chain)
      // (scalar: a per-lane select would pull the division into the chain loop)
      const double nmin_dv = uni(nmin / dV), nmin_dv_b = uni((double)(nb - 1) / dV);
      const bool odd = intra && (na & 1);
      if constexpr (NXN) {
        // N x N (Sec. 3.1): every pair once with s of Eq. (10)
        // (w_max / dV), in rounds of disjoint pairs, one barrier per round.
        //  intra: the circle schedule on np = N rounded up to even; round r
        //         pairs (r, np-1) and ((r+m) mod R, (r-m) mod R), 0 < m <
        //         np/2, R = np - 1 rounds; pairs that touch the pad are skipped
        //  inter: round r pairs list-a entry i with list-b entry
        //         (i + r) mod N_max; N_max rounds of min(N_a, N_b) pairs,
        //         visited from the shorter list
        // kp = r * P + slot, P = np / 2 (intra) or N_a (inter).
        const double cf = C.coef / dV;
        const int np = na + (na & 1), R = intra ? np - 1 : Nmax;
        const int P = intra ? np / 2 : na;
        const int per = intra ? np / 2 : Nmin;  // slots visited per round
        for (int r = 0; r < R; ++r) {
          for (int sl = t; sl < per; sl += TPC) {
            int I = -1, J = -1, i = sl;
            if (intra) {
              const int x = sl == 0 ? r : (r + sl) % R;
              const int y = sl == 0 ? np - 1 : (r - sl + R) % R;
              if (x < na && y < na) {
                I = L0[x];
                J = L0[y];
              }
            } else {
              // a slot of the shorter list; i indexes list a, j list b
              i = abig ? (sl - r + Nmax) % Nmax : sl;
              const int j = abig ? sl : (sl + r) % Nmax;
              I = L0[i];
              J = L1[j];
            }
            if (I < 0) continue;
            const uint32_t kp = (uint32_t)(r * P + i);
            if constexpr (REL)
              scatter_pair_rel(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, ma, mb, A.c, A.method,
                               (uint32_t)cell, step_lo, c3p, k0, k1, A.n97);
            else if constexpr (sizeof(KR) == 8)
              scatter_pair_nr_f64(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, C.fa, C.fb, A.method,
                                  (uint32_t)cell, step_lo, c3p, k0, k1, A.n97);
            else if constexpr (TAB_LDS)
              scatter_pair_nr<KR>(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, C.fa, C.fb, A.method,
                                  (uint32_t)cell, step_lo, c3p, k0, k1, s_tab);
            else
              scatter_pair_nr<KR>(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, C.fa, C.fb, A.method,
                                  (uint32_t)cell, step_lo, c3p, k0, k1, A.n97);
          }
          if (r + 1 < R) __syncthreads();
        }
        __syncthreads();
        if (t == 0) {
          s_st[0] += intra ? (unsigned long long)na * (na - 1) / 2 : (unsigned long long)na * nb;
          s_st[3] += 1;
        }
      } else {
        // Pairs that share a particle form a chain, run in order by one lane:
        // the odd triple (L0,L1),(L1,L2),(L2,L0); in an inter-species collision
        // the pairs k, k + N_min, k + 2 N_min, ... (they share small[k]).
        // Different chains touch disjoint particles, so one barrier ends the
        // scatter and every particle sees its pairs in ascending k.  A dual
        // pass runs the chains of species b after those of species a.
        const int ncha = intra ? (odd ? 1 + (na - 3) / 2 : na / 2) : Nmin;
        const bool oddb = dual && (nb & 1);
        const int nchb = dual ? (oddb ? 1 + (nb - 3) / 2 : nb / 2) : 0;
        const uint32_t c3pb = ctr3(step, k + 1, PURPOSE_PAIR);
        // inter: N_max = q N_min + rem, so chain ch holds q + (ch < rem) pairs
        const int q_int = (!intra && Nmin > 0) ? uni(Nmax / Nmin) : 0;
        const int rem_int = Nmax - q_int * Nmin;
        for (int ch0 = t; ch0 < ncha + nchb; ch0 += TPC) {
          const bool sb = ch0 >= ncha;  // (dual pass) a chain of species b
          const int ch = sb ? ch0 - ncha : ch0;
          const bool odds = sb ? oddb : odd;
          const int len = intra ? ((odds && ch == 0) ? 3 : 1) : q_int + (ch < rem_int ? 1 : 0);
          // the constants of the collision this chain belongs to
          const CollConst &Cs = s_cc[sb ? 1 : 0];
          const double nmins_dv = sb ? nmin_dv_b : nmin_dv;
          const uint32_t c3s = sb ? c3pb : c3p;
          for (int r = 0; r < len; ++r) {
            int I, J;
            uint32_t kp;
            double f = 1.0;
            if (intra) {
              const uint16_t *L = sb ? L1 : L0;
              if (odds) {
                if (ch == 0) {
                  I = L[r];
                  J = L[r == 2 ? 0 : r + 1];
                  kp = (uint32_t)r;
                  f = 0.5;
                } else {
                  const int m = ch - 1;
                  I = L[3 + 2 * m];
                  J = L[4 + 2 * m];
                  kp = (uint32_t)(3 + m);
                }
              } else {
                I = L[2 * ch];
                J = L[2 * ch + 1];
                kp = (uint32_t)ch;
              }
            } else {
              const int kk = r * Nmin + ch;
              I = abig ? L0[kk] : L0[ch];
              J = abig ? L1[ch] : L1[kk];
              kp = (uint32_t)kk;
            }
            double cf = Cs.coef * f * nmins_dv;
            if constexpr (DUP) {
              // duplicity s: N_max / D for N_min, D = this chain's length
              // (the pairs of its fewer-population particle)
              if (!intra) cf = Cs.coef * ((double)Nmax / dV) / (double)len;
            }
            if constexpr (REL)
              scatter_pair_rel(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, ma, mb, A.c, A.method,
                               (uint32_t)cell, step_lo, c3p, k0, k1, A.n97);
            else if constexpr (TAN)
              scatter_pair_nr_tan(M.vx, M.vy, M.vz, M.tx, M.ty, M.tz, M.w, I, J, kp, cf, C.fa, C.fb,
                                  A.method, (uint32_t)cell, step_lo, c3p, k0, k1, A.n97, A.dlnl);
            else if constexpr (sizeof(KR) == 8)
              scatter_pair_nr_f64(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, Cs.fa, Cs.fb, A.method,
                                  (uint32_t)cell, step_lo, c3s, k0, k1, A.n97);
            else if constexpr (TAB_LDS)
              scatter_pair_nr<KR>(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, Cs.fa, Cs.fb, A.method,
                                  (uint32_t)cell, step_lo, c3s, k0, k1, s_tab);
            else
              scatter_pair_nr<KR>(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, Cs.fa, Cs.fb, A.method,
                                  (uint32_t)cell, step_lo, c3s, k0, k1, A.n97);
          }
        }
        __syncthreads();
        if (t == 0) {
          s_st[0] += intra ? (odd ? 3 + (na - 3) / 2 : na / 2) : Nmax;
          if (dual) s_st[0] += oddb ? 3 + (nb - 3) / 2 : nb / 2;
          s_st[3] += dual ? 2 : 1;
        }
      }

      MCC_PHASE(3);  // momentum restore and energy sums
      __builtin_amdgcn_s_setprio(1);
      if (!A.corr) continue;

      auto in_a = [&](int e) { return (unsigned)(e - oa) < (unsigned)na; };
      auto in_b = [&](int e) { return two && (unsigned)(e - ob) < (unsigned)nb; };
      auto part = [&](int e) { return in_a(e) || in_b(e); };
      auto mass_of = [&](int e) { return in_a(e) ? ma : mb; };

      // momentum restore, Eq. (17): B = sum m_p (v_ps - v_bs) / sum m_p w_p;
      // v -= B w is applied in the energy pass below
      double Bx, By, Bz;
      double Bbx = 0.0, Bby = 0.0, Bbz = 0.0;  // species b of a dual pass
      {
        constexpr int NP = TAN ? 6 : 3;  // the tangent of the sums rides along
        // P[3..5]: the tangent sums, or species b's sums of a dual pass
        double P[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) P[i] = 0.0;
        // branch-free where everything is in LDS: every owned slot is
        // visited and non-members add nothing (slots past n lie in the LDS
        // arrays, and what they hold is selected away)
        auto mom = [&](int j, int e) {
          const bool ia = in_a(e), ib = in_b(e);
          const double mp = (ia ? ma : mb) * M.w[e];
          const double dx = mp * (M.vx[e] - SNAPX(j, e));
          const double dy = mp * (M.vy[e] - SNAPY(j, e));
          const double dz = mp * (M.vz[e] - SNAPZ(j, e));
          const bool to_a = ia || (ib && !dual), to_b = ib && dual;
          P[0] += to_a ? dx : 0.0;
          P[1] += to_a ? dy : 0.0;
          P[2] += to_a ? dz : 0.0;
          if constexpr (!TAN) {
            P[3] += to_b ? dx : 0.0;
            P[4] += to_b ? dy : 0.0;
            P[5] += to_b ? dz : 0.0;
          } else if (ia || ib) {
            P[3] += mp * (M.tx[e] - M.btx[e]);
            P[4] += mp * (M.ty[e] - M.bty[e]);
            P[5] += mp * (M.tz[e] - M.btz[e]);
          }
        };
        if constexpr (!GL && W_LDS) {
#pragma unroll
          for (int j = 0; j < PPT; ++j) mom(j, t + j * TPC);
        } else {
          for_owned<TPC, PPT, !GL>(n, mom);
        }
        MCC_PHASE(10);  // momentum reduction
        // (no closing barrier: the energy reduction below writes the other
        // part of `red`, and its own barrier orders these reads before any
        // later write; the tangent form's energy sums need all of `red`)
        double tot[6];
        if (dual)
          block_sum<TPC, 6, TAN>(P, red, tot);
        else
          block_sum<TPC, NP, TAN>(P, red, tot);
        const double D = ma * s_sw2[a] + (intra ? 0.0 : mb * s_sw2[b]);
        Bx = tot[0] / D;
        By = tot[1] / D;
        Bz = tot[2] / D;
        if (dual) {
          const double Db = mb * s_sw2[b];
          Bbx = tot[3] / Db;
          Bby = tot[4] / Db;
          Bbz = tot[5] / Db;
        }
        if constexpr (TAN) {
          const double tBx = tot[3] / D, tBy = tot[4] / D, tBz = tot[5] / D;
          for_owned<TPC, PPT, !GL>(n, [&](int j, int e) {
            if (e < n && part(e)) {
              const double we = M.w[e];
              M.tx[e] -= tBx * we;
              M.ty[e] -= tBy * we;
              M.tz[e] -= tBz * we;
            }
          });
        }
      }
      MCC_PHASE(11);  // energy pass
      // energy violation, Eq. (18) (difference form), and the sums of Eq. (24)
      double dEs0, dEs1;
      double tdEs0 = 0.0, tdEs1 = 0.0;  // tangent form
      {
        // per particle: the energy change (difference form, summed with
        // compensation: its total is a small difference of large terms and
        // decides how many pairs the correction uses) and, for an
        // inter-species collision, the kinetic energy of each species
        double es = 0.0, ec = 0.0;
        double es1 = 0.0, ec1 = 0.0;  // species b of a dual pass
        // KE_a, KE_b (inter-species only: sums of positive terms, plain);
        // tangent form: then the tangents of dE, KE_a, KE_b
        constexpr int NE = TAN ? 5 : 2;
        double Ev[NE];
#pragma unroll
        for (int i = 0; i < NE; ++i) Ev[i] = 0.0;
        const double c2 = A.c * A.c;
        // mem: the particle takes part (with every slot visited, the sums
        // select non-members away and only the stores are predicated)
        auto energy = [&](int j, int e, bool mem) {
          {
            const bool isa = in_a(e);
            const bool sb = dual && !isa;
            const double we = M.w[e];
            const double mp = (isa ? ma : mb) * we;
            const double rbx = sb ? Bbx : Bx, rby = sb ? Bby : By, rbz = sb ? Bbz : Bz;
            const double vx = M.vx[e] - rbx * we, vy = M.vy[e] - rby * we,
                         vz = M.vz[e] - rbz * we;
            if (mem) {
              M.vx[e] = vx;
              M.vy[e] = vy;
              M.vz[e] = vz;
            }
            const double ox = SNAPX(j, e), oy = SNAPY(j, e), oz = SNAPZ(j, e);
            const double dd = (vx - ox) * (vx + ox) + (vy - oy) * (vy + oy) + (vz - oz) * (vz + oz);
            double term, ke;
            if constexpr (REL) {
              const double vv = vx * vx + vy * vy + vz * vz;
              const double gv = sqrt(1.0 + vv / c2);
              const double gb = sqrt(1.0 + (ox * ox + oy * oy + oz * oz) / c2);
              term = mp * dd / (gv + gb);
              ke = mp * vv / (gv + 1.0);
            } else {
              term = 0.5 * mp * dd;
              ke = 0.5 * mp * (vx * vx + vy * vy + vz * vz);
            }
            csum_add(es, ec, (mem && !sb) ? term : 0.0);
            if constexpr (DUAL) csum_add(es1, ec1, (mem && sb) ? term : 0.0);
            if (TAN || !intra) {
              Ev[0] += (mem && isa) ? ke : 0.0;
              Ev[1] += (mem && !isa) ? ke : 0.0;
            }
            if constexpr (TAN) {
              const double tvx = M.tx[e], tvy = M.ty[e], tvz = M.tz[e];
              const double dke = mp * (vx * tvx + vy * tvy + vz * tvz);
              Ev[2 % NE] += dke - mp * (ox * M.btx[e] + oy * M.bty[e] + oz * M.btz[e]);
              if (isa)
                Ev[3 % NE] += dke;
              else
                Ev[4 % NE] += dke;
            }
          }
        };
        if constexpr (!GL && W_LDS && !TAN) {
#pragma unroll
          for (int j = 0; j < PPT; ++j) {
            const int e = t + j * TPC;
            energy(j, e, part(e));
          }
        } else {
          for_owned<TPC, PPT, !GL>(n, [&](int j, int e) {
            if (part(e)) energy(j, e, true);
          });
        }
        MCC_PHASE(12);  // energy reduction
        // the part of `red` the momentum reduction left alone; no closing
        // barrier unless the diagnostics reuse all of `red` next
        double *ered = red + 6 * NW;
        dEs1 = 0.0;
        if constexpr (TAN) {
          double tot[NE];
          block_sum_c1<TPC, NE>(es, ec, Ev, red, dEs0, tot);
          tdEs0 = tot[2 % NE];
          tdEs1 = 0.0;
          if (!intra && dEs0 != 0.0) {
            const double dE = dEs0, tdE = tot[2 % NE];
            const double ea = s_sw[a] / na * tot[0], eb = s_sw[b] / nb * tot[1];
            const double tea = s_sw[a] / na * tot[3 % NE], teb = s_sw[b] / nb * tot[4 % NE];
            const double ra = ea / (ea + eb), rb = eb / (ea + eb);
            const double tr = (tea * eb - ea * teb) / ((ea + eb) * (ea + eb));
            dEs0 = ra * dE;
            dEs1 = rb * dE;
            tdEs0 = tr * dE + ra * tdE;
            tdEs1 = -tr * dE + rb * tdE;
          }
        } else if (dual) {
          // two intra-species violations, each corrected on its own species
          block_sum_c2<TPC, DIAG>(es, ec, es1, ec1, ered, dEs0, dEs1);
        } else if (intra) {
          CSum<1> Cv;
          Cv.s[0] = es;
          Cv.c[0] = ec;
          double out[1];
          block_csum<TPC, 1, false, DIAG>(Cv, ered, out);
          dEs0 = out[0];
        } else {
          double tot[2];
          block_sum_c1<TPC, 2, DIAG>(es, ec, Ev, ered, dEs0, tot);
          if (dEs0 != 0.0) {
            const double dE = dEs0;
            const double ea = s_sw[a] / na * tot[0], eb = s_sw[b] / nb * tot[1];
            dEs0 = ea / (ea + eb) * dE;
            dEs1 = eb / (ea + eb) * dE;
          }
        }
      }

      MCC_PHASE(4);  // correction order
      // correction order per species (Alg. 1, optional sort), then the pair loop
      const int nsl = two ? 2 : 1;
      const uint16_t *O0 = L0, *O1 = L1;
      if (A.sortw) {
        auto order = [&](int sp, int o, int ns, const uint16_t *L, uint16_t *ord) {
          const int f = s_wflag[sp];
          if (f == WORDER_EQUAL) return L;  // all weights equal: the shuffled order
          if (f == WORDER_DISTINCT) {
            // (without an LDS home: only a plan marks a species distinct, and
            // its order is read from HBM)
            if constexpr (HAS_WORD)
              return (const uint16_t *)(M.word + o);
            else
              return (const uint16_t *)(A.prep_word + cb + o);
          }
          weight_sort<TPC, PPT, GL>(M, ns, L, 0, ord, s_wlo[sp], s_whi[sp], wsum, &maxocc);
          return (const uint16_t *)ord;
        };
        O0 = order(a, oa, na, L0, M.ord0);
        if (two) O1 = order(b, ob, nb, L1, M.ord1);
      }
      double *Kb = M.kbuf;
      const int base1 = na / 2;           // pair slots of the second species
      double *Xb = Kb + CAP / 2;          // REL: h(-mu_R) per pair
      double resid0 = dEs0, resid1 = dEs1;
      double tresid0 = tdEs0, tresid1 = tdEs1;  // tangent form
      int used_total = 0;
      for (int pass = 0; pass < A.max_passes; ++pass) {
        if (resid0 == 0.0 && resid1 == 0.0) break;
        MCC_PHASE(5);  // pair energies
        // K of every pair; pairs are disjoint, so each K is the value the
        // sequential loop of Alg. 1 sees.  In the plain non-relativistic
        // form the cut-off computes K itself, 64 pairs at a time and only up
        // to the cut pair (usually within the first 64).
        constexpr bool KCUT = !REL && !TAN;
        const int np0 = (!KCUT && resid0 != 0.0) ? na / 2 : 0;
        const int np1 = (!KCUT && nsl == 2 && resid1 != 0.0) ? nb / 2 : 0;
        for (int m = t; m < np0 + np1; m += TPC) {
          const bool s1 = m >= np0;
          const int mm = s1 ? m - np0 : m;
          const uint16_t *O = s1 ? O1 : O0;
          const double ms = s1 ? mb : ma;
          const int slot = (s1 ? base1 : 0) + mm;
          const int p = O[2 * mm], q = O[2 * mm + 1];
          const double m1 = ms * M.w[p], m2 = ms * M.w[q];
          if constexpr (REL) {
            Kb[slot] = pair_K_rel(m1, m2, M.vx[p], M.vy[p], M.vz[p], M.vx[q], M.vy[q], M.vz[q],
                                  A.c);
            RelPair R;
            R.init(m1, m2, M.vx[p], M.vy[p], M.vz[p], M.vx[q], M.vy[q], M.vz[q], A.c);
            double dh;
            Xb[slot] = R.h0(-R.mu(), dh);
          } else {
            Kb[slot] = pair_K_nr(m1, m2, M.vx[p], M.vy[p], M.vz[p], M.vx[q], M.vy[q], M.vz[q]);
            if constexpr (TAN) {
              const double mu = m1 * m2 / (m1 + m2);
              M.kdot[slot] = mu * ((M.vx[p] - M.vx[q]) * (M.tx[p] - M.tx[q]) +
                                   (M.vy[p] - M.vy[q]) * (M.ty[p] - M.ty[q]) +
                                   (M.vz[p] - M.vz[q]) * (M.tz[p] - M.tz[q]));
            }
          }
        }
        if constexpr (!KCUT) __syncthreads();
        MCC_PHASE(6);  // sequential cut-off loop
        if constexpr (REL) {
          // the running violation, in the paper's order (one lane per species):
          // whether a pair can take U depends on the running value itself
          const int sl = (t == 0) ? 0 : ((NW > 1 && t == WAVE) ? 1 : -1);
          for (int s2 = (NW > 1 ? sl : 0); s2 >= 0 && s2 < nsl; s2 += (NW > 1 ? nsl : 1)) {
            if (NW == 1 && t != 0) break;
            double E = s2 == 0 ? resid0 : resid1;
            const int np = (s2 == 0 ? na : nb) / 2, kb = s2 == 0 ? 0 : base1;
            int m = 0, used = 0;
            for (; m < np; ++m) {
              if (E == 0.0) break;
              const double K = Kb[kb + m];
              double U = 0.0;
              if (K != 0.0) {
                const double lim = A.fE * K;
                U = fabs(E) < lim ? E : copysign(lim, E);
                if (U > 0.0 && Xb[kb + m] + U > 0.0) U = 0.0;  // no root: skip the pair
              }
              Kb[kb + m] = U;
              if (U != 0.0) {
                E -= U;
                ++used;
              }
            }
            s_ncut[s2] = m;
            s_res[s2] = E;
            s_used[s2] = used;
          }
        } else {
          // The running violation E of one species, one wave per species.
          // Pairs take U = sign(E) f_E K in order until the remainder is
          // smaller than f_E K of the next pair, which takes the remainder
          // (Eq. (23)); that pair is the first whose inclusive prefix sum of
          // f_E K reaches |E|.  The prefix sums run over 64 pairs at a time.
          const int lane = t & (WAVE - 1);
          auto cutoff = [&](int s2) {
            const double E0 = s2 == 0 ? resid0 : resid1;
            const double sgn = E0 < 0.0 ? -1.0 : 1.0;
            const int np = (s2 == 0 ? na : nb) / 2, kb = s2 == 0 ? 0 : base1;
            double absE = fabs(E0);
            // tangent form: tangent of |E| (the cut pair's U is |E| minus the
            // prefix before it; the others take f_E K)
            double tabsE = TAN ? sgn * (s2 == 0 ? tresid0 : tresid1) : 0.0;
            int ncut = 0, used = 0;
            for (int m0 = 0; m0 < np && absE != 0.0; m0 += WAVE) {
              const int m = m0 + lane;
              double lim = 0.0;
              if (m < np) {
                if constexpr (KCUT) {
                  const uint16_t *O = s2 ? O1 : O0;
                  const double ms = s2 ? mb : ma;
                  const int p = O[2 * m], q = O[2 * m + 1];
                  lim = A.fE * pair_K_nr(ms * M.w[p], ms * M.w[q], M.vx[p], M.vy[p], M.vz[p],
                                         M.vx[q], M.vy[q], M.vz[q]);
                } else {
                  lim = A.fE * Kb[kb + m];
                }
              }
              const double P = wave_incl_scan(lim);
              const double Pprev = wave_shr1(P);  // (0 in lane 0)
              double tlim = 0.0, tP = 0.0, tPprev = 0.0;
              if constexpr (TAN) {
                tlim = m < np ? A.fE * M.kdot[kb + m] : 0.0;
                tP = wave_incl_scan(tlim);
                tPprev = wave_shr1(tP);
              }
              const unsigned long long hit = __ballot(m < np && P >= absE);
              if (hit) {
                const int kc = __builtin_ctzll(hit);
                const double U = lane < kc ? lim : absE - Pprev;
                if (lane <= kc) Kb[kb + m] = sgn * U;
                if constexpr (TAN) {
                  if (lane <= kc) M.kdot[kb + m] = sgn * (lane < kc ? tlim : tabsE - tPprev);
                }
                used += __popcll(__ballot(lane <= kc && U != 0.0));
                ncut = m0 + kc + 1;
                absE = 0.0;
                tabsE = 0.0;
              } else {
                if (m < np) Kb[kb + m] = sgn * lim;
                if constexpr (TAN) {
                  if (m < np) M.kdot[kb + m] = sgn * tlim;
                }
                used += __popcll(__ballot(m < np && lim != 0.0));
                const int last = (np - m0 < WAVE ? np - m0 : WAVE) - 1;
                absE -= wave_bcast(P, last);
                if constexpr (TAN) tabsE -= wave_bcast(tP, last);
                ncut = m0 + last + 1;
              }
            }
            if (lane == 0) {
              s_ncut[s2] = ncut;
              s_res[s2] = sgn * absE;
              s_used[s2] = used;
              if constexpr (TAN) s_tres[s2] = sgn * tabsE;
            }
          };
          if constexpr (NW > 1) {
            if (t / WAVE < nsl) cutoff(t / WAVE);
          } else {
            cutoff(0);
            if (nsl == 2) cutoff(1);
          }
        }
        if (nsl == 1 && t == 0) {
          s_ncut[1] = 0;
          s_res[1] = 0.0;
          s_tres[1] = 0.0;
          s_used[1] = 0;
        }
        __syncthreads();
        MCC_PHASE(7);  // apply pair corrections
        // apply the pair corrections, Eqs. (19)-(22) / (A.3)-(A.5)
        const int nc0 = s_ncut[0], nc1 = s_ncut[1];
        for (int m = t; m < nc0 + nc1; m += TPC) {
          const bool s1 = m >= nc0;
          const int mm = s1 ? m - nc0 : m;
          const int slot = (s1 ? base1 : 0) + mm;
          const double U = Kb[slot];
          if (U == 0.0) continue;
          const uint16_t *O = s1 ? O1 : O0;
          const double ms = s1 ? mb : ma;
          const int p = O[2 * mm], q = O[2 * mm + 1];
          const double m1 = ms * M.w[p], m2 = ms * M.w[q];
          if constexpr (REL) {
            RelPair R;
            R.init(m1, m2, M.vx[p], M.vy[p], M.vz[p], M.vx[q], M.vy[q], M.vz[q], A.c);
            const double al = rel_alpha(R, U);
            const double f1 = al / m1, f2 = al / m2;
            M.vx[p] += f1 * R.dx;
            M.vy[p] += f1 * R.dy;
            M.vz[p] += f1 * R.dz;
            M.vx[q] -= f2 * R.dx;
            M.vy[q] -= f2 * R.dy;
            M.vz[q] -= f2 * R.dz;
          } else {
            const double mu = m1 * m2 / (m1 + m2);
            const double rx = M.vx[p] - M.vx[q], ry = M.vy[p] - M.vy[q], rz = M.vz[p] - M.vz[q];
            const double K = 0.5 * mu * (rx * rx + ry * ry + rz * rz);
            const double x = U / K;
            const double g = -x / (1.0 + sqrt(1.0 - x));
            const double f1 = mu / m1 * g, f2 = mu / m2 * g;
            if constexpr (TAN) {
              // g = sqrt(1 - x) - 1, x = U / K
              const double trx = M.tx[p] - M.tx[q], try_ = M.ty[p] - M.ty[q],
                           trz = M.tz[p] - M.tz[q];
              const double tK = mu * (rx * trx + ry * try_ + rz * trz);
              const double tx_ = (M.kdot[slot] - x * tK) / K;
              const double tg = -0.5 * tx_ / sqrt(1.0 - x);
              const double c1 = mu / m1, c2 = mu / m2;
              M.tx[p] += c1 * (tg * rx + g * trx);
              M.ty[p] += c1 * (tg * ry + g * try_);
              M.tz[p] += c1 * (tg * rz + g * trz);
              M.tx[q] -= c2 * (tg * rx + g * trx);
              M.ty[q] -= c2 * (tg * ry + g * try_);
              M.tz[q] -= c2 * (tg * rz + g * trz);
            }
            M.vx[p] += f1 * rx;
            M.vy[p] += f1 * ry;
            M.vz[p] += f1 * rz;
            M.vx[q] -= f2 * rx;
            M.vy[q] -= f2 * ry;
            M.vz[q] -= f2 * rz;
          }
        }
        resid0 = s_res[0];
        resid1 = s_res[1];
        if constexpr (TAN) {
          tresid0 = s_tres[0];
          tresid1 = s_tres[1];
        }
        used_total += s_used[0] + s_used[1];
        __syncthreads();
      }
      MCC_PHASE(8);  // failure handling and diagnostics
      // one decision per collision: for both species of an inter-species
      // collision, per species in a dual pass
      const bool failA = dual ? resid0 != 0.0 : (resid0 != 0.0 || resid1 != 0.0);
      const bool failB = dual ? resid1 != 0.0 : failA;
      if (t == 0) {
        s_st[1] += used_total;
        s_st[2] += (failA ? 1 : 0) + (dual && failB ? 1 : 0);
      }
      if ((failA || failB) && !A.keep) {  // Sec. 6.2: reset this collision in this cell
        for_owned<TPC, PPT, !GL>(n, [&](int j, int e) {
          if (e < n && part(e) && ((e >= oa && e < oa + na) ? failA : failB)) {
            M.vx[e] = SNAPX(j, e);
            M.vy[e] = SNAPY(j, e);
            M.vz[e] = SNAPZ(j, e);
            if constexpr (TAN) {
              M.tx[e] = M.btx[e];
              M.ty[e] = M.bty[e];
              M.tz[e] = M.btz[e];
            }
          }
        });
      }
      __syncthreads();
      if constexpr (DIAG) {  // residual momentum and energy of this collision
        CSum<6> D;
        D.zero();
        const double c2 = A.c * A.c;
        for_owned<TPC, PPT, !GL>(n, [&](int j, int e) {
                    if (e < n && part(e)) {
            const double mp = mass_of(e) * M.w[e];
            const double vx = M.vx[e], vy = M.vy[e], vz = M.vz[e];
            const double ox = SNAPX(j, e), oy = SNAPY(j, e), oz = SNAPZ(j, e);
            D.add(0, mp * (vx - ox));
            D.add(1, mp * (vy - oy));
            D.add(2, mp * (vz - oz));
            const double oo = ox * ox + oy * oy + oz * oz;
            D.add(3, mp * sqrt(oo));
            const double dd = (vx - ox) * (vx + ox) + (vy - oy) * (vy + oy) + (vz - oz) * (vz + oz);
            if constexpr (REL) {
              const double gv = sqrt(1.0 + (vx * vx + vy * vy + vz * vz) / c2);
              const double gb = sqrt(1.0 + oo / c2);
              D.add(4, mp * dd / (gv + gb));
              D.add(5, mp * oo / (gb + 1.0));
            } else {
              D.add(4, 0.5 * mp * dd);
              D.add(5, 0.5 * mp * oo);
            }
          }
        });
        double tot[6];
        block_csum<TPC, 6>(D, red, tot);
        if (t == 0) {
          const double rp = sqrt(tot[0] * tot[0] + tot[1] * tot[1] + tot[2] * tot[2]);
          const double relP = tot[3] > 0.0 ? rp / tot[3] : 0.0;
          const double relE = tot[5] > 0.0 ? fabs(tot[4]) / tot[5] : 0.0;
          s_sd[0] = relP > s_sd[0] ? relP : s_sd[0];
          s_sd[1] = relE > s_sd[1] ? relE : s_sd[1];
        }
      }
#undef SNAPX
#undef SNAPY
#undef SNAPZ
    }

    MCC_PHASE(9);  // write-back
    __syncthreads();
    for (int e = t; e < n; e += TPC) {
      if (!TAN || A.write_primal) {
        A.vx[cb + e] = M.vx[e];
        A.vy[cb + e] = M.vy[e];
        A.vz[cb + e] = M.vz[e];
      }
      if constexpr (TAN) {
        A.tx[cb + e] = M.tx[e];
        A.ty[cb + e] = M.ty[e];
        A.tz[cb + e] = M.tz[e];
      }
    }
    if (t == 0) {
      if (A.cell_corr) A.cell_corr[cell] = (int32_t)s_st[1];
      for (int i = 0; i < 4; ++i) s_acc[i] += s_st[i];
      s_accd[0] = s_sd[0] > s_accd[0] ? s_sd[0] : s_accd[0];
      s_accd[1] = s_sd[1] > s_accd[1] ? s_sd[1] : s_accd[1];
    }
    if (t == 0) s_next[par] = q + NQ * (nq + claim);
    __syncthreads();
    li = uni((int)s_next[par]);  // (the next write goes to the other slot)
    par ^= 1;
  }
  if (t == 0) {
    if (A.stats) {
      if (s_acc[0]) atomicAdd(&A.stats->pairs, s_acc[0]);
      if (s_acc[1]) atomicAdd(&A.stats->corr_pairs, s_acc[1]);
      if (s_acc[2]) atomicAdd(&A.stats->failed, s_acc[2]);
      if (s_acc[3]) atomicAdd(&A.stats->collisions, s_acc[3]);
      if (A.diag) {
        atomicMax(reinterpret_cast<unsigned long long *>(&A.stats->max_rel_dP),
                  (unsigned long long)__double_as_longlong(s_accd[0]));
        atomicMax(reinterpret_cast<unsigned long long *>(&A.stats->max_rel_dE),
                  (unsigned long long)__double_as_longlong(s_accd[1]));
      }
    }
    // every claim of this workgroup has returned; the last one of its queue
    // resets the queue's counters (all other claims are complete by then)
    if (atomicAdd(qctr + 1, 1u) == nq - 1) {
      atomicExch(qctr, 0u);
      atomicExch(qctr + 1, 0u);
    }
  }
#ifdef MCC_PHASE_TIMING
  MCC_PHASE(15);
  if (threadIdx.x == 0 && A.phase)
    for (int i = 0; i < 16; ++i) atomicAdd(&A.phase[i], s_ph[i]);
#endif
#undef MCC_PHASE
}

}  // namespace mcc
