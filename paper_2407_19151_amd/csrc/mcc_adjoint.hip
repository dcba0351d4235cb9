// mcc_adjoint.hip -- reverse-mode derivative of one collision step: the
// vector-Jacobian product behind mcc_collide_adjoint.
//
// The step (Algorithm 1: pairing, weighted scatter with the TA77/N97 angle of
// Eq. (12), momentum restore of Eq. (17), energy violation and partition of
// Eqs. (18), (24), zero-angle pair correction of Eqs. (19)-(23), failure
// fallback of Sec. 6.2) is a smooth map of the velocities and of lnL once
// every random number and every discrete choice is fixed: the pairs, the
// acceptances, the correction order, the cut pair and the failure decision.
// For an adjoint g of the step's output, this kernel returns g J (the
// adjoint of the step's input) and g dv'/dlnL, cell by cell:
//
//   for each collision k, last to first:
//     recompute the state at the start of collision k (collisions 0..k-1
//     from the step's input), then collision k itself while recording the
//     state before every scatter pair, the state after the momentum restore,
//     and the correction's pair energies, cut pair and failure decision;
//     sweep back: the pair corrections (disjoint pairs; the cut pair's U
//     depends on Delta E_s and on the K of the pairs before it), the energy
//     partition, the momentum restore, then the scatter chains in reverse.
//
// A pair's Jacobian d(du)/d(u, s) is built from the same tangent arithmetic
// as the forward-mode form (rot_tangent), one column per basis direction.
// The recomputed forward runs in the step's own precision form (FP32
// kinematics or FP64) so that it takes the same discrete choices; the
// Jacobians are evaluated in FP64 with that form's uniforms.  One workgroup
// per cell, with the cell and its records in per-workgroup global scratch;
// threads per cell as in the forward-mode kernels, so the per-cell sums
// round, and the cut pair falls, as there.
#include "mcc_adjoint_args.hpp"
#include "mcc_collide.hpp"

namespace mcc {

// The adjoint of one scatter pair, given the pair's input velocities (pi, pj)
// and the adjoints (gI, gJ) of its output, in place: gI, gJ become the
// adjoints of its input; lbar gains the pair's part of the lnL adjoint.
template <typename KR>
__device__ __attribute__((noinline)) void pair_adjoint(
    double pix, double piy, double piz, double pjx, double pjy, double pjz, double wi, double wj,
    uint32_t kp, double cf, double fa, double fb, int method, uint32_t cell, uint32_t step_lo,
    uint32_t c3, uint32_t k0, uint32_t k1, const double2 *n97tab, double inv_lnl, double *gx,
    double *gy, double *gz, int I, int J, double &lbar) {
  using K = KMath<double>;
  const double ux = pix - pjx, uy = piy - pjy, uz = piz - pjz;
  const double wmax = wi > wj ? wi : wj;
  // the primal's skips, in its own precision
  {
    const KR fx = (KR)ux, fy = (KR)uy, fz = (KR)uz;
    const KR f2 = fx * fx + fy * fy + fz * fz;
    if (f2 == KR(0)) return;
    const KR fs = KMath<KR>::div((KR)(cf * wmax), f2 * KMath<KR>::sqrt_(f2));
    if (!(fs > KR(0))) return;
  }
  const double um2 = ux * ux + uy * uy + uz * uz;
  const double um = K::sqrt_(um2);
  const double s = (cf * wmax) / (um2 * um);
  const U4 r = philox(kp, cell, step_lo, c3, k0, k1);
  // the form's uniforms (the FP32 form draws 23-bit ones)
  const double u0 = (double)KMath<KR>::u(r.x), u1 = (double)KMath<KR>::u(r.y);
  const double u2 = (double)KMath<KR>::u(r.z);
  double oc, st, A = 0.0;
  if (method == 0) {
    const double z = sqrt(-2.0 * log(u0)) * cospi(2.0 * u1);
    const double delta = sqrt(0.5 * s) * z;
    const double d2 = delta * delta;
    if (__builtin_isinf(d2)) {
      oc = 2.0;
      st = 0.0;
    } else {
      const double q = 1.0 / (1.0 + d2);
      st = 2.0 * delta * q;
      oc = 2.0 * d2 * q;
    }
  } else {
    A = n97_A_fast<double>(s, n97tab);
    if (__builtin_isinf(A))
      oc = 0.0;
    else if (A == 0.0)
      oc = 2.0 * u0;
    else
      oc = -log1p(u0 * expm1(-2.0 * A)) / A;
    oc = oc < 0.0 ? 0.0 : (oc > 2.0 ? 2.0 : oc);
    st = sqrt(oc * (2.0 - oc));
  }
  double sp, cp;
  sincospi(2.0 * u2, &sp, &cp);
  const double u3 = unif64(r.w);
  const double wratio = (wi < wj ? wi : wj) / wmax;
  bool ai = true, aj = true;
  if (wi < wj)
    aj = u3 <= wratio;
  else if (wj < wi)
    ai = u3 <= wratio;
  // v_I' = v_I + fa du (if accepted), v_J' = v_J - fb du: adjoint of du
  const double dbx = (ai ? fa * gx[I] : 0.0) - (aj ? fb * gx[J] : 0.0);
  const double dby = (ai ? fa * gy[I] : 0.0) - (aj ? fb * gy[J] : 0.0);
  const double dbz = (ai ? fa * gz[I] : 0.0) - (aj ? fb * gz[J] : 0.0);
  if (dbx == 0.0 && dby == 0.0 && dbz == 0.0) return;
  // columns of d(du)/du (s follows |u|: ds = -3 s (u . du) / |u|^2), then
  // d(du)/dlnL (ds = s / lnL)
  double ub[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double ui = i == 0 ? ux : (i == 1 ? uy : uz);
    double tx, ty, tz;
    rot_tangent(method, ux, uy, uz, um, s, oc, st, sp, cp, u0, A, i == 0 ? 1.0 : 0.0,
                i == 1 ? 1.0 : 0.0, i == 2 ? 1.0 : 0.0, -3.0 * s * ui / um2, tx, ty, tz);
    ub[i] = tx * dbx + ty * dby + tz * dbz;
  }
  if (inv_lnl != 0.0) {
    double tx, ty, tz;
    rot_tangent(method, ux, uy, uz, um, s, oc, st, sp, cp, u0, A, 0.0, 0.0, 0.0, s * inv_lnl, tx,
                ty, tz);
    lbar += tx * dbx + ty * dby + tz * dbz;
  }
  gx[I] += ub[0];
  gy[I] += ub[1];
  gz[I] += ub[2];
  gx[J] -= ub[0];
  gy[J] -= ub[1];
  gz[J] -= ub[2];
}

template <int TPC, int CAP, typename KR>
__global__ void __launch_bounds__(TPC) adjoint_kernel(AdjointArgs A) {
  constexpr int PPT = CAP / TPC;
  constexpr int NW = TPC / WAVE;
  static_assert(CAP % TPC == 0 && TPC % WAVE == 0, "bad variant");
  __shared__ double red[2 * 6 * NW];
  uint64_t *redu = reinterpret_cast<uint64_t *>(red);
  __shared__ uint32_t wsum[NW];
  __shared__ uint32_t maxocc;
  __shared__ int s_so[MCC_MAX_SPECIES + 1];
  __shared__ int s_bad;
  __shared__ long long s_cb;
  __shared__ unsigned long long s_wlo[MCC_MAX_SPECIES], s_whi[MCC_MAX_SPECIES];
  __shared__ double s_sw[MCC_MAX_SPECIES], s_sw2[MCC_MAX_SPECIES];
  __shared__ int s_wflag[MCC_MAX_SPECIES];
  __shared__ int s_ncut[2];
  __shared__ double s_res[2];
  __shared__ double s_ubar[2];
  __shared__ __attribute__((aligned(16))) uint32_t lcnt[CAP + 2];

  char *base = A.scratch + (uint64_t)blockIdx.x * A.stride;
  double *dv = reinterpret_cast<double *>(base);
  CellMem M;
  M.vx = dv;
  M.vy = dv + CAP;
  M.vz = dv + 2 * CAP;
  double *const W = dv + 3 * CAP;
  M.w = W;
  M.bx = dv + 4 * CAP;  // state at the collision's start
  M.by = dv + 5 * CAP;
  M.bz = dv + 6 * CAP;
  double *const GX = dv + 7 * CAP;  // the adjoint being swept back
  double *const GY = dv + 8 * CAP;
  double *const GZ = dv + 9 * CAP;
  double *const QX = dv + 10 * CAP;  // state after the momentum restore
  double *const QY = dv + 11 * CAP;
  double *const QZ = dv + 12 * CAP;
  double *const XX = dv + 13 * CAP;  // the step's input
  double *const XY = dv + 14 * CAP;
  double *const XZ = dv + 15 * CAP;
  double *const PIX = dv + 16 * CAP;  // input state of scatter pair kp
  double *const PIY = dv + 17 * CAP;
  double *const PIZ = dv + 18 * CAP;
  double *const PJX = dv + 19 * CAP;
  double *const PJY = dv + 20 * CAP;
  double *const PJZ = dv + 21 * CAP;
  M.kbuf = dv + 22 * CAP;
  double *const HX = dv + 23 * CAP;  // adjoint of the collision's start state
  double *const HY = dv + 24 * CAP;  // through the energy and momentum sums
  double *const HZ = dv + 25 * CAP;
  M.key = reinterpret_cast<uint32_t *>(dv + 26 * CAP);
  M.slotbuf = M.key + CAP;
  uint16_t *ix = reinterpret_cast<uint16_t *>(M.slotbuf + CAP);
  M.list0 = ix;
  M.list1 = ix + CAP;
  M.ord0 = ix + 2 * CAP;
  M.ord1 = ix + 3 * CAP;
  M.mem = ix + 4 * CAP;
  M.word = ix + 5 * CAP;
  M.cnt = lcnt;
  M.tx = M.ty = M.tz = M.btx = M.bty = M.btz = M.kdot = nullptr;

  const int t = threadIdx.x;
  const int lane = t & (WAVE - 1);
  const int S = A.S;
  const uint32_t step_lo = (uint32_t)A.step;
  const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
  const uint32_t count = *A.cell_count;

  for (uint32_t li = blockIdx.x; li < count; li += gridDim.x) {
    const int cell = A.cell_list[li];
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
      }
    }
    __syncthreads();
    if (s_bad) {  // skipped by the step too: its derivative is the identity
      __syncthreads();
      continue;
    }
    const int64_t cb = uni(s_cb);
    const int n = uni(s_so[S]);
    const double dV = A.cell_volume ? A.cell_volume[cell] : A.dV;
    for (int e = t; e < n; e += TPC) {
      W[e] = A.w[cb + e];
      XX[e] = A.vx[cb + e];
      XY[e] = A.vy[cb + e];
      XZ[e] = A.vz[cb + e];
      GX[e] = A.gx[cb + e];
      GY[e] = A.gy[cb + e];
      GZ[e] = A.gz[cb + e];
    }
    __syncthreads();
    if (A.corr) {
      // per species: sum w, sum w^2, the weight range and class, and the
      // descending-weight order (as the step computes them per cell)
      for (int sp = 0; sp < S; ++sp) {
        const int o = s_so[sp], ns = s_so[sp + 1] - o;
        CSum<2> acc;  // compensated, as the step sums them
        acc.zero();
        uint64_t lo[1] = {~0ull}, hi[1] = {0ull};
        for (int e = o + t; e < o + ns; e += TPC) {
          const double we = W[e];
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
          weight_sort<TPC, PPT, true>(M, ns, nullptr, o, M.word + o, lo[0], hi[0], wsum, &maxocc);
          int tie = 0;
          for (int q = t; q + 1 < ns; q += TPC)
            if (W[M.word[o + q]] == W[M.word[o + q + 1]]) tie = 1;
          flag = __syncthreads_or(tie) ? WORDER_TIES : WORDER_DISTINCT;
        }
        if (t == 0) {
          s_sw[sp] = tot[0];
          s_sw2[sp] = tot[1];
          s_wlo[sp] = lo[0];
          s_whi[sp] = hi[0];
          s_wflag[sp] = flag;
        }
      }
      __syncthreads();
    }

    // what the recorded collision leaves for its reverse sweep
    struct Rec {
      double dE, ea, eb, D;
      int nc0, nc1;
      double res0, res1;
      bool fail;
      const uint16_t *O0, *O1;
    } R{};

    // one collision of the step on M.vx/vy/vz (the step's arithmetic, the
    // choices it takes included); rec: keep what the reverse sweep needs
    auto fwd = [&](int k, bool rec) {
      const int a = A.coll[k].a, b = A.coll[k].b;
      const bool intra = a == b;
      const int oa = uni(s_so[a]), na = uni(s_so[a + 1]) - oa;
      const int ob = uni(s_so[b]), nb = uni(s_so[b + 1]) - ob;
      const CollConst &C = A.coll[k];
      const double ma = A.mass[a], mb = A.mass[b];
      auto in_a = [&](int e) { return (unsigned)(e - oa) < (unsigned)na; };
      auto part = [&](int e) { return in_a(e) || (!intra && (unsigned)(e - ob) < (unsigned)nb); };
      for (int e = t; e < n; e += TPC)
        if (part(e)) {
          M.bx[e] = M.vx[e];
          M.by[e] = M.vy[e];
          M.bz[e] = M.vz[e];
        }
      if (intra)
        shuffle_species<TPC, PPT, true>(M, na, oa, (uint32_t)cell, step_lo,
                                        ctr3(A.step, k, PURPOSE_SHUFFLE0 + 0), k0, k1, M.list0,
                                        wsum, &maxocc);
      else
        shuffle_two<TPC, PPT, true>(M, na, oa, nb, ob, (uint32_t)cell, step_lo,
                                    ctr3(A.step, k, PURPOSE_SHUFFLE0 + 0),
                                    ctr3(A.step, k, PURPOSE_SHUFFLE0 + 1), k0, k1, M.list0,
                                    wsum, &maxocc);
      const uint16_t *L0 = M.list0, *L1 = M.list0 + na;
      const uint32_t c3p = ctr3(A.step, k, PURPOSE_PAIR);
      const bool abig = na >= nb;
      const int Nmax = abig ? na : nb, Nmin = abig ? nb : na;
      const double nmin_dv = (intra ? (double)(na - 1) : (double)Nmin) / dV;
      const bool odd = intra && (na & 1);
      const int nch = intra ? (odd ? 1 + (na - 3) / 2 : na / 2) : Nmin;
      for (int ch = t; ch < nch; ch += TPC) {
        const int len = intra ? ((odd && ch == 0) ? 3 : 1) : (Nmax - ch + Nmin - 1) / Nmin;
        for (int r = 0; r < len; ++r) {
          int I, J;
          uint32_t kp;
          double f = 1.0;
          if (intra) {
            if (odd && ch == 0) {
              I = L0[r];
              J = L0[r == 2 ? 0 : r + 1];
              kp = (uint32_t)r;
              f = 0.5;
            } else if (odd) {
              I = L0[3 + 2 * (ch - 1)];
              J = L0[4 + 2 * (ch - 1)];
              kp = (uint32_t)(3 + ch - 1);
            } else {
              I = L0[2 * ch];
              J = L0[2 * ch + 1];
              kp = (uint32_t)ch;
            }
          } else {
            const int kk = r * Nmin + ch;
            I = abig ? L0[kk] : L0[ch];
            J = abig ? L1[ch] : L1[kk];
            kp = (uint32_t)kk;
          }
          if (rec) {
            PIX[kp] = M.vx[I];
            PIY[kp] = M.vy[I];
            PIZ[kp] = M.vz[I];
            PJX[kp] = M.vx[J];
            PJY[kp] = M.vy[J];
            PJZ[kp] = M.vz[J];
          }
          const double cf = C.coef * f * nmin_dv;
          if constexpr (sizeof(KR) == 8)
            scatter_pair_nr_f64(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, C.fa, C.fb, A.method,
                                (uint32_t)cell, step_lo, c3p, k0, k1, A.n97);
          else
            scatter_pair_nr<KR>(M.vx, M.vy, M.vz, M.w, I, J, kp, cf, C.fa, C.fb, A.method,
                                (uint32_t)cell, step_lo, c3p, k0, k1, A.n97);
        }
      }
      __syncthreads();
      if (!A.corr) return;
      // momentum restore, Eq. (17)
      double P[3] = {0.0, 0.0, 0.0};
      for (int e = t; e < n; e += TPC)
        if (part(e)) {
          const double mp = (in_a(e) ? ma : mb) * W[e];
          P[0] += mp * (M.vx[e] - M.bx[e]);
          P[1] += mp * (M.vy[e] - M.by[e]);
          P[2] += mp * (M.vz[e] - M.bz[e]);
        }
      double tot[3];
      block_sum<TPC, 3>(P, red, tot);
      const double D = ma * s_sw2[a] + (intra ? 0.0 : mb * s_sw2[b]);
      const double Bx = tot[0] / D, By = tot[1] / D, Bz = tot[2] / D;
      // energy violation, Eq. (18), and the species energies of Eq. (24)
      double es = 0.0, ec = 0.0;
      double Ev[2] = {0.0, 0.0};
      for (int e = t; e < n; e += TPC)
        if (part(e)) {
          const bool isa = in_a(e);
          const double we = W[e];
          const double mp = (isa ? ma : mb) * we;
          const double vx = M.vx[e] - Bx * we, vy = M.vy[e] - By * we, vz = M.vz[e] - Bz * we;
          M.vx[e] = vx;
          M.vy[e] = vy;
          M.vz[e] = vz;
          if (rec) {
            QX[e] = vx;
            QY[e] = vy;
            QZ[e] = vz;
          }
          const double ox = M.bx[e], oy = M.by[e], oz = M.bz[e];
          const double dd = (vx - ox) * (vx + ox) + (vy - oy) * (vy + oy) + (vz - oz) * (vz + oz);
          csum_add(es, ec, 0.5 * mp * dd);
          const double ke = 0.5 * mp * (vx * vx + vy * vy + vz * vz);
          Ev[0] += isa ? ke : 0.0;
          Ev[1] += isa ? 0.0 : ke;
        }
      double dE, et[2];
      block_sum_c1<TPC, 2>(es, ec, Ev, red, dE, et);
      double dEs0 = dE, dEs1 = 0.0, ea = 0.0, eb = 0.0;
      if (!intra && dE != 0.0) {
        ea = s_sw[a] / na * et[0];
        eb = s_sw[b] / nb * et[1];
        dEs0 = ea / (ea + eb) * dE;
        dEs1 = eb / (ea + eb) * dE;
      }
      // correction order (Alg. 1, optional sort)
      const int nsl = intra ? 1 : 2;
      const uint16_t *O0 = L0, *O1 = L1;
      if (A.sortw) {
        auto order = [&](int sp, int o, int ns, const uint16_t *L, uint16_t *ord) {
          const int f = s_wflag[sp];
          if (f == WORDER_EQUAL) return L;
          if (f == WORDER_DISTINCT) return (const uint16_t *)(M.word + o);
          weight_sort<TPC, PPT, true>(M, ns, L, 0, ord, s_wlo[sp], s_whi[sp], wsum, &maxocc);
          return (const uint16_t *)ord;
        };
        O0 = order(a, oa, na, L0, M.ord0);
        if (!intra) O1 = order(b, ob, nb, L1, M.ord1);
      }
      // cut-off, Eq. (23): the first pair whose prefix sum of f_E K reaches
      // |Delta E_s| takes the remainder (one wave per species, 64 pairs at
      // a time, as the step)
      double *Kb = M.kbuf;
      const int base1 = na / 2;
      auto cutoff = [&](int s2) {
        const double E0 = s2 == 0 ? dEs0 : dEs1;
        const double sgn = E0 < 0.0 ? -1.0 : 1.0;
        const int np = (s2 == 0 ? na : nb) / 2, kb = s2 == 0 ? 0 : base1;
        double absE = fabs(E0);
        int ncut = 0;
        for (int m0 = 0; m0 < np && absE != 0.0; m0 += WAVE) {
          const int m = m0 + lane;
          double lim = 0.0;
          if (m < np) {
            const uint16_t *O = s2 ? O1 : O0;
            const double ms = s2 ? mb : ma;
            const int p = O[2 * m], q = O[2 * m + 1];
            lim = A.fE * pair_K_nr(ms * W[p], ms * W[q], M.vx[p], M.vy[p], M.vz[p], M.vx[q],
                                   M.vy[q], M.vz[q]);
          }
          const double Pi = wave_incl_scan(lim);
          const double Pprev = wave_shr1(Pi);
          const unsigned long long hit = __ballot(m < np && Pi >= absE);
          if (hit) {
            const int kc = __builtin_ctzll(hit);
            const double U = lane < kc ? lim : absE - Pprev;
            if (lane <= kc) Kb[kb + m] = sgn * U;
            ncut = m0 + kc + 1;
            absE = 0.0;
          } else {
            if (m < np) Kb[kb + m] = sgn * lim;
            const int last = (np - m0 < WAVE ? np - m0 : WAVE) - 1;
            absE -= wave_bcast(Pi, last);
            ncut = m0 + last + 1;
          }
        }
        if (lane == 0) {
          s_ncut[s2] = ncut;
          s_res[s2] = sgn * absE;
        }
      };
      if constexpr (NW > 1) {
        if (t / WAVE < nsl) cutoff(t / WAVE);
      } else {
        cutoff(0);
        if (nsl == 2) cutoff(1);
      }
      if (nsl == 1 && t == 0) {
        s_ncut[1] = 0;
        s_res[1] = 0.0;
      }
      __syncthreads();
      const int nc0 = s_ncut[0], nc1 = s_ncut[1];
      for (int m = t; m < nc0 + nc1; m += TPC) {
        const bool s1 = m >= nc0;
        const int mm = s1 ? m - nc0 : m;
        const double U = Kb[(s1 ? base1 : 0) + mm];
        if (U == 0.0) continue;
        const uint16_t *O = s1 ? O1 : O0;
        const double ms = s1 ? mb : ma;
        const int p = O[2 * mm], q = O[2 * mm + 1];
        const double m1 = ms * W[p], m2 = ms * W[q];
        const double mu = m1 * m2 / (m1 + m2);
        const double rx = M.vx[p] - M.vx[q], ry = M.vy[p] - M.vy[q], rz = M.vz[p] - M.vz[q];
        const double K = 0.5 * mu * (rx * rx + ry * ry + rz * rz);
        const double x = U / K;
        const double g = -x / (1.0 + sqrt(1.0 - x));
        const double f1 = mu / m1 * g, f2 = mu / m2 * g;
        M.vx[p] += f1 * rx;
        M.vy[p] += f1 * ry;
        M.vz[p] += f1 * rz;
        M.vx[q] -= f2 * rx;
        M.vy[q] -= f2 * ry;
        M.vz[q] -= f2 * rz;
      }
      const double res0 = s_res[0], res1 = s_res[1];
      __syncthreads();
      const bool fail = res0 != 0.0 || res1 != 0.0;
      if (fail && !A.keep)
        for (int e = t; e < n; e += TPC)
          if (part(e)) {
            M.vx[e] = M.bx[e];
            M.vy[e] = M.by[e];
            M.vz[e] = M.bz[e];
          }
      if (rec) {
        R.dE = dE;
        R.ea = ea;
        R.eb = eb;
        R.D = D;
        R.nc0 = nc0;
        R.nc1 = nc1;
        R.res0 = res0;
        R.res1 = res1;
        R.fail = fail;
        R.O0 = O0;
        R.O1 = O1;
      }
      __syncthreads();
    };

    // the reverse sweep of collision k (recorded by fwd(k, true)): GX/GY/GZ,
    // the adjoint of the collision's output, becomes that of its input
    auto rev = [&](int k, double &lbar) {
      const int a = A.coll[k].a, b = A.coll[k].b;
      const bool intra = a == b;
      const int oa = uni(s_so[a]), na = uni(s_so[a + 1]) - oa;
      const int ob = uni(s_so[b]), nb = uni(s_so[b + 1]) - ob;
      const CollConst &C = A.coll[k];
      const double ma = A.mass[a], mb = A.mass[b];
      auto in_a = [&](int e) { return (unsigned)(e - oa) < (unsigned)na; };
      auto part = [&](int e) { return in_a(e) || (!intra && (unsigned)(e - ob) < (unsigned)nb); };
      if (R.fail && !A.keep) return;  // Sec. 6.2 reset: the output is the input
      if (A.corr) {
        const int nsl = intra ? 1 : 2;
        const int base1 = na / 2;
        const double *Kb = M.kbuf;
        // the cut pair of each species: adjoint of its U (before any pair's
        // adjoint changes GX/GY/GZ)
        if (t < 2) {
          double ub = 0.0;
          const double res = t == 0 ? R.res0 : R.res1;
          const int nc = t == 0 ? R.nc0 : R.nc1;
          if (t < nsl && res == 0.0 && nc > 0) {
            const int c = nc - 1;
            const double U = Kb[(t ? base1 : 0) + c];
            if (U != 0.0) {
              const uint16_t *O = t ? R.O1 : R.O0;
              const double ms = t ? mb : ma;
              const int p = O[2 * c], q = O[2 * c + 1];
              const double m1 = ms * W[p], m2 = ms * W[q];
              const double mu = m1 * m2 / (m1 + m2);
              const double rx = QX[p] - QX[q], ry = QY[p] - QY[q], rz = QZ[p] - QZ[q];
              const double K = 0.5 * mu * (rx * rx + ry * ry + rz * rz);
              const double sq = sqrt(1.0 - U / K);
              const double a1 = mu / m1, a2 = mu / m2;
              const double gb = (a1 * GX[p] - a2 * GX[q]) * rx + (a1 * GY[p] - a2 * GY[q]) * ry +
                                (a1 * GZ[p] - a2 * GZ[q]) * rz;
              ub = -gb / (2.0 * K * sq);  // dg/dU = -1 / (2 K sqrt(1 - U/K))
            }
          }
          s_ubar[t] = ub;
        }
        __syncthreads();
        // every correction pair (disjoint): v1' = v1 + (mu/m1) g r,
        // v2' = v2 - (mu/m2) g r, r = v1 - v2, g = sqrt(1 - U/K) - 1.  A pair
        // before the cut has U/K = +-f_E (g fixed); the cut pair's g moves
        // with its K and with U = Delta E_s - sum over earlier pairs of
        // +-f_E K, whose K then carry -+f_E times the adjoint of U.
        const int nc0 = R.nc0, nc1 = R.nc1;
        for (int m = t; m < nc0 + nc1; m += TPC) {
          const bool s1 = m >= nc0;
          const int mm = s1 ? m - nc0 : m;
          const double U = Kb[(s1 ? base1 : 0) + mm];
          if (U == 0.0) continue;
          const uint16_t *O = s1 ? R.O1 : R.O0;
          const double ms = s1 ? mb : ma;
          const int p = O[2 * mm], q = O[2 * mm + 1];
          const double m1 = ms * W[p], m2 = ms * W[q];
          const double mu = m1 * m2 / (m1 + m2);
          const double rx = QX[p] - QX[q], ry = QY[p] - QY[q], rz = QZ[p] - QZ[q];
          const double K = 0.5 * mu * (rx * rx + ry * ry + rz * rz);
          const double x = U / K;
          const double sq = sqrt(1.0 - x);
          const double g = -x / (1.0 + sq);
          const double a1 = mu / m1, a2 = mu / m2;
          const double dx = a1 * GX[p] - a2 * GX[q], dy = a1 * GY[p] - a2 * GY[q],
                       dz = a1 * GZ[p] - a2 * GZ[q];
          const double res = s1 ? R.res1 : R.res0;
          const int nc = s1 ? nc1 : nc0;
          double Kbar = 0.0;
          if (res == 0.0) {
            if (mm == nc - 1) {
              const double gb = dx * rx + dy * ry + dz * rz;
              Kbar = gb * x / (2.0 * K * sq);  // dg/dK = x / (2 K sqrt(1 - x))
            } else {
              Kbar = -(U < 0.0 ? -1.0 : 1.0) * A.fE * s_ubar[s1 ? 1 : 0];
            }
          }
          // r's adjoint: g (d) + Kbar dK/dr, dK/dr = mu r
          const double rbx = g * dx + Kbar * mu * rx, rby = g * dy + Kbar * mu * ry,
                       rbz = g * dz + Kbar * mu * rz;
          GX[p] += rbx;
          GY[p] += rby;
          GZ[p] += rbz;
          GX[q] -= rbx;
          GY[q] -= rby;
          GZ[q] -= rbz;
        }
        __syncthreads();
        // energy violation (difference form of Eq. (18)) and partition
        // (Eq. (24)): the cut pairs' U adjoints are those of Delta E_s
        const double ua = s_ubar[0], ubb = nsl == 2 ? s_ubar[1] : 0.0;
        double dEbar = 0.0, kina = 0.0, kinb = 0.0;
        if (intra) {
          dEbar = ua;
        } else if (R.dE != 0.0) {
          const double Ssum = R.ea + R.eb;
          dEbar = ua * (R.ea / Ssum) + ubb * (R.eb / Ssum);
          const double eabar = R.dE * (ua - ubb) * R.eb / (Ssum * Ssum);
          const double ebbar = -R.dE * (ua - ubb) * R.ea / (Ssum * Ssum);
          kina = eabar * (s_sw[a] / na);
          kinb = ebbar * (s_sw[b] / nb);
        }
        // Delta E = sum 1/2 m (|q|^2 - |b|^2), E_s = sum over s of 1/2 m |q|^2:
        // q (after the restore) takes (dEbar + kin_s) m q, b takes -dEbar m b
        double P[3] = {0.0, 0.0, 0.0};
        for (int e = t; e < n; e += TPC)
          if (part(e)) {
            const bool isa = in_a(e);
            const double mp = (isa ? ma : mb) * W[e];
            const double cq = (dEbar + (isa ? kina : kinb)) * mp;
            GX[e] += cq * QX[e];
            GY[e] += cq * QY[e];
            GZ[e] += cq * QZ[e];
            HX[e] = -dEbar * mp * M.bx[e];
            HY[e] = -dEbar * mp * M.by[e];
            HZ[e] = -dEbar * mp * M.bz[e];
            // momentum restore, q = v_ps - B w: adjoint of B is -sum w g_q
            P[0] -= W[e] * GX[e];
            P[1] -= W[e] * GY[e];
            P[2] -= W[e] * GZ[e];
          }
        double Bb[3];
        block_sum<TPC, 3>(P, red, Bb);
        // B = sum m (v_ps - b) / D: v_ps takes Bbar m / D, b takes -Bbar m / D
        for (int e = t; e < n; e += TPC)
          if (part(e)) {
            const double c = (in_a(e) ? ma : mb) * W[e] / R.D;
            GX[e] += Bb[0] * c;
            GY[e] += Bb[1] * c;
            GZ[e] += Bb[2] * c;
            HX[e] -= Bb[0] * c;
            HY[e] -= Bb[1] * c;
            HZ[e] -= Bb[2] * c;
          }
        __syncthreads();
      }
      // the scatter: chains of pairs (one lane each), last pair first
      const uint16_t *L0 = M.list0, *L1 = M.list0 + na;
      const uint32_t c3p = ctr3(A.step, k, PURPOSE_PAIR);
      const bool abig = na >= nb;
      const int Nmax = abig ? na : nb, Nmin = abig ? nb : na;
      const double nmin_dv = (intra ? (double)(na - 1) : (double)Nmin) / dV;
      const bool odd = intra && (na & 1);
      const int nch = intra ? (odd ? 1 + (na - 3) / 2 : na / 2) : Nmin;
      for (int ch = t; ch < nch; ch += TPC) {
        const int len = intra ? ((odd && ch == 0) ? 3 : 1) : (Nmax - ch + Nmin - 1) / Nmin;
        for (int r = len - 1; r >= 0; --r) {
          int I, J;
          uint32_t kp;
          double f = 1.0;
          if (intra) {
            if (odd && ch == 0) {
              I = L0[r];
              J = L0[r == 2 ? 0 : r + 1];
              kp = (uint32_t)r;
              f = 0.5;
            } else if (odd) {
              I = L0[3 + 2 * (ch - 1)];
              J = L0[4 + 2 * (ch - 1)];
              kp = (uint32_t)(3 + ch - 1);
            } else {
              I = L0[2 * ch];
              J = L0[2 * ch + 1];
              kp = (uint32_t)ch;
            }
          } else {
            const int kk = r * Nmin + ch;
            I = abig ? L0[kk] : L0[ch];
            J = abig ? L1[ch] : L1[kk];
            kp = (uint32_t)kk;
          }
          pair_adjoint<KR>(PIX[kp], PIY[kp], PIZ[kp], PJX[kp], PJY[kp], PJZ[kp], W[I], W[J], kp,
                           C.coef * f * nmin_dv, C.fa, C.fb, A.method, (uint32_t)cell, step_lo,
                           c3p, k0, k1, A.n97, A.inv_lnl, GX, GY, GZ, I, J, lbar);
        }
      }
      __syncthreads();
      if (A.corr)
        for (int e = t; e < n; e += TPC)
          if (part(e)) {
            GX[e] += HX[e];
            GY[e] += HY[e];
            GZ[e] += HZ[e];
          }
      __syncthreads();
    };

    double lbar = 0.0;
    for (int k = A.n_coll - 1; k >= 0; --k) {
      const int a = A.coll[k].a, b = A.coll[k].b;
      const int na = uni(s_so[a + 1]) - uni(s_so[a]), nb = uni(s_so[b + 1]) - uni(s_so[b]);
      if (a == b ? na < 2 : (na == 0 || nb == 0)) continue;  // no pairs: the identity
      for (int e = t; e < n; e += TPC) {
        M.vx[e] = XX[e];
        M.vy[e] = XY[e];
        M.vz[e] = XZ[e];
      }
      __syncthreads();
      for (int j = 0; j < k; ++j) {
        const int aj = A.coll[j].a, bj = A.coll[j].b;
        const int nja = uni(s_so[aj + 1]) - uni(s_so[aj]);
        const int njb = uni(s_so[bj + 1]) - uni(s_so[bj]);
        if (aj == bj ? nja < 2 : (nja == 0 || njb == 0)) continue;
        fwd(j, false);
      }
      fwd(k, true);
      rev(k, lbar);
    }
    double acc[1] = {lbar}, tot[1];
    block_sum<TPC, 1>(acc, red, tot);
    if (t == 0) A.lnl_part[cell] = tot[0];
    for (int e = t; e < n; e += TPC) {
      A.gx[cb + e] = GX[e];
      A.gy[cb + e] = GY[e];
      A.gz[cb + e] = GZ[e];
    }
    __syncthreads();
  }
}

// deterministic sum of x[0..n) into out[0] (one workgroup, fixed order)
__global__ void __launch_bounds__(1024) k_sum_f64(const double *x, int64_t n, double *out) {
  __shared__ double red[2 * 6 * 16];
  double acc[1] = {0.0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) acc[0] += x[i];
  double tot[1];
  block_sum<1024, 1>(acc, red, tot);
  if (threadIdx.x == 0) out[0] = tot[0];
}

// kernels per (threads per cell, capacity) of the forward-mode variants
template <typename KR>
const void *adjoint_kernel_of(int tpc, int cap) {
  if (cap > 4096) return reinterpret_cast<const void *>(&adjoint_kernel<64, 32768, KR>);
  if (tpc >= 256) return reinterpret_cast<const void *>(&adjoint_kernel<256, 4096, KR>);
  if (tpc >= 128) return reinterpret_cast<const void *>(&adjoint_kernel<128, 4096, KR>);
  return reinterpret_cast<const void *>(&adjoint_kernel<64, 4096, KR>);
}

hipError_t launch_adjoint(const AdjointArgs &base, bool fp32, const int32_t *lists,
                          const uint32_t *counts, int32_t n_cells, int b, int tpc, int cap,
                          int grid, hipStream_t s) {
  AdjointArgs A = base;
  A.cell_list = lists + (int64_t)b * (n_cells > 0 ? n_cells : 1);
  A.cell_count = counts + b;
  void *kargs[] = {&A};
  const void *k = fp32 ? adjoint_kernel_of<float>(tpc, cap) : adjoint_kernel_of<double>(tpc, cap);
  return hipLaunchKernel(k, dim3(grid), dim3(tpc), kargs, 0, s);
}

hipError_t launch_sum_f64(const double *x, int64_t n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(1024), 0, s, x, n, out);
  return hipGetLastError();
}

}  // namespace mcc
