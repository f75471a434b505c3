// chunk.hpp -- the per-bin forward/reverse sweep over a chunk of K
// consecutive bins held by one thread.
//
// Gaussians on a uniform grid.  With z_k = z_0 + k dz (dz = h/s) the factor
// e_k = exp(-z_k^2/2) obeys e_{k+1} = e_k r_k and r_{k+1} = r_k D, with
// r_0 = exp(-dz z_0 - dz^2/2) and D = exp(-dz^2): two exps per Gaussian per
// chunk instead of one per bin.  An exponential background exp(b0 + b1 t) is
// a geometric sequence on the grid, E_{k+1} = E_k exp(b1 dt): one exp per
// chunk.  After k steps the relative error is about k^2/2 ulp.  The
// recurrence is used only when K |dz| <= 1: then an e_0 that underflows
// (|z_0| > 38.6) implies every e_k in the chunk is below 1e-300, so nothing
// that matters is lost; r_0's exponent is clamped (+-700 in FP64, +-80 where
// the FP32 exp takes it) so that 0 * r_0 stays 0.  Otherwise each bin takes
// its own exp.
//
// A polynomial background is advanced by forward differences on a
// recurrence chunk (degree additions per bin instead of forming t and
// evaluating the polynomial); its rounding error grows by about one ulp of
// the largest difference per bin, far below the objective's tolerance.
//
// Objective terms are branch-free (domain cases are only flagged), so the
// compiler can interleave the K bins.
#pragma once

#include "device.hpp"
#include "fastmath.hpp"

namespace hf {

// l(n, mu) and ubar = dl/dmu; returns true for a domain error.  Domain bins
// are only flagged: the kernel then reports L = +inf and a NaN gradient, so
// the common path carries no selects.  mu is clamped to a tiny positive
// value before the division; the empty bin (n = 0) then comes out exactly as
// l = mu, ubar = 1 (including mu = 0), the log of r = 0 being finite.
template <int OBJ, bool F32BIN>
__device__ __forceinline__ bool objective_t(double n, double mu, const double2* __restrict__ lut,
                                            double& l, double& ub) {
  constexpr double kTiny = 1e-300;
  if constexpr (OBJ == OBJ_NEYMAN) {
    const bool pos = n > 0.0;
    const double inv = rcp_fast(fmax(n, kTiny));
    const double d = mu - n;
    const double di = pos ? d * inv : 0.0;
    l = d * di;
    ub = 2.0 * di;
    return false;
  } else if constexpr (OBJ == OBJ_PEARSON) {
    const double inv = rcp_fast(fmax(mu, kTiny));
    const double d = n - mu;
    const double r = n * inv;
    l = d * d * inv;
    ub = fma(-r, r, 1.0);
    return !(mu > 0.0);
  } else {
    // Poisson, saturated: l = mu - n + n ln(n/mu) (n > 0), l = mu (n = 0)
    const double r = div_fast<F32BIN>(n, fmax(mu, kTiny));
    const double lg = log_lut<F32BIN>(r, lut);
    l = fma(n, lg, mu - n);
    ub = 1.0 - r;
    // domain: mu < 0, or mu = 0 with n > 0, i.e. mu below 0 (n = 0) or below
    // the smallest positive double (n > 0) -- one min and one compare
    constexpr double kDenormMin = 4.9406564584124654e-324;
    return mu < fmin(n, kDenormMin);
  }
}

template <int NG, int BKG, int OBJ, bool GRAD, bool F32BIN, bool RECUR, int K, int NV>
__device__ __forceinline__ void chunk_1d(const Model1D<NG, BKG>& M, const double2* __restrict__ lut,
                                         double xs, const double (&n)[K], const double (&w)[K],
                                         double (&acc)[NV], int& flags, double (&lk)[K]) {
  using S = Shape1D<NG, BKG>;
  constexpr int G1 = NG > 0 ? NG : 1;
  double z0[G1], e[G1], r[G1];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    z0[g] = (xs - M.m[g]) * M.is[g];
    if constexpr (RECUR) {
      const double q0 = -0.5 * z0[g] * z0[g];
      const double a0 = clamp_ratio_exponent<F32BIN>(fma(-M.dz[g], z0[g], -0.5 * M.dz[g] * M.dz[g]));
      e[g] = F32BIN ? exp_hw32(q0) : exp_fast(q0);
      r[g] = F32BIN ? exp_hw32(a0) : exp_fast(a0);
    }
  }
  const double t0 = (xs - M.tshift) * M.ta;
  // Reverse sweep of a recurrence chunk by moments.  With z_k = z0 + k dz and
  // t_k = t0 + k dt (k = 0..K-1 known constants), the adjoint sums need only
  //   U_l = sum_k mb_k e_k k^l (l = 0..2) per Gaussian:
  //     sum mb G z   = A (z0 U_0 + dz U_1)
  //     sum mb G z^2 = A (z0^2 U_0 + 2 z0 dz U_1 + dz^2 U_2)
  //   T_l = sum_k mb_k k^l for the polynomial (sum mb t^j by the binomial
  //   expansion of (t0 + k dt)^j), or sum_k mb_k E_k k^l (l < 2) for the
  //   exponential (sum mb E t = t0 T_0 + dt T_1),
  // expanded once at the end of the chunk: a multiply-add per moment per bin
  // instead of forming z and t powers per bin.
  constexpr bool MOM = RECUR && GRAD;
  constexpr int NT = (BKG == BKG_EXP) ? 2 : (S::NB > 0 ? S::NB : 1);
  double U[G1][3], T[NT];
  if constexpr (MOM) {
#pragma unroll
    for (int g = 0; g < NG; ++g) U[g][0] = U[g][1] = U[g][2] = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) T[j] = 0.0;
  }
  double Eb = 0.0;  // exponential background at the current bin (recurrence)
  if constexpr (RECUR && BKG == BKG_EXP) {
    const double a0 = fma(M.c[1], t0, M.c[0]);
    Eb = F32BIN ? exp_hw32(a0) : exp_fast(a0);
  }
  // Polynomial background on a recurrence chunk by forward differences:
  // b(t0 + k dt) = sum_j q_j k^j with q_j = dt^j sum_{i>=j} C(i,j) c_i t0^(i-j),
  // and its differences at k = 0 advance by NB - 1 additions per bin.
  constexpr int NBP = (BKG == BKG_EXP || S::NB <= 0) ? 1 : S::NB;
  double fd[NBP];
  if constexpr (RECUR && BKG != BKG_EXP && S::NB > 0) {
    constexpr double C[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
    double q[NBP];
    double dtp = 1.0;
#pragma unroll
    for (int j = 0; j < NBP; ++j) {
      double sj = 0.0;
#pragma unroll
      for (int i = NBP - 1; i >= j; --i) sj = fma(sj, t0, C[i][j] * M.c[i]);
      q[j] = sj * dtp;
      dtp *= M.dt;
    }
    // differences of sum q_j k^j at k = 0 (degree <= 3)
    fd[0] = q[0];
    if constexpr (NBP > 1) fd[1] = q[1] + (NBP > 2 ? q[2] : 0.0) + (NBP > 3 ? q[3] : 0.0);
    if constexpr (NBP > 2) fd[2] = 2.0 * q[2] + (NBP > 3 ? 6.0 * q[3] : 0.0);
    if constexpr (NBP > 3) fd[3] = 6.0 * q[3];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    // ---- forward sweep ----
    double z[G1], ek[G1], G[G1];
    double mu = 0.0;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      z[g] = fma(static_cast<double>(k), M.dz[g], z0[g]);
      if constexpr (RECUR) {
        ek[g] = e[g];
      } else {
        const double q = -0.5 * z[g] * z[g];
        ek[g] = F32BIN ? exp_hw32(q) : exp_fast(q);
      }
      G[g] = M.A[g] * ek[g];
      mu += G[g];
    }
    const double t = fma(static_cast<double>(k), M.dt, t0);
    double E = 0.0;
    if constexpr (BKG == BKG_EXP) {
      if constexpr (RECUR) {
        E = Eb;
        Eb *= M.qE;
      } else {
        const double a = fma(M.c[1], t, M.c[0]);
        E = F32BIN ? exp_hw32(a) : exp_fast(a);
      }
      mu += E;
    } else if constexpr (S::NB > 0) {
      if constexpr (RECUR) {
        mu += fd[0];
#pragma unroll
        for (int j = 0; j + 1 < NBP; ++j) fd[j] += fd[j + 1];
      } else {
        double b = M.c[S::NB - 1];
#pragma unroll
        for (int j = S::NB - 2; j >= 0; --j) b = fma(b, t, M.c[j]);
        mu += b;
      }
    }
    double l, ub;
    const bool dom = objective_t<OBJ, F32BIN>(n[k], mu, lut, l, ub);
    flags |= dom ? ST_DOMAIN : 0;
    lk[k] = l;
    acc[0] = fma(w[k], l, acc[0]);
    if constexpr (MOM) {
      // ---- reverse sweep, moment form (expanded after the loop) ----
      const double mb = w[k] * ub;
      const double kd = static_cast<double>(k), k2 = kd * kd;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const double u = mb * ek[g];
        U[g][0] += u;
        U[g][1] = fma(u, kd, U[g][1]);
        U[g][2] = fma(u, k2, U[g][2]);
      }
      if constexpr (BKG == BKG_EXP) {
        const double eb = mb * E;
        T[0] += eb;
        T[1] = fma(eb, kd, T[1]);
      } else if constexpr (S::NB > 0) {
        T[0] += mb;
        double kp = kd;
#pragma unroll
        for (int j = 1; j < S::NB; ++j) {
          T[j] = fma(mb, kp, T[j]);
          kp *= kd;
        }
      }
    } else if constexpr (GRAD) {
      // ---- reverse sweep: mu_bar = w ubar ----
      const double mb = w[k] * ub;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        // G = A e:  A_bar += mb e ;  e_bar = mb A
        // e = exp(q): q_bar = e_bar e = mb G ; q = -z^2/2: z_bar = -q_bar z
        // z = (x - m)/s: m_bar = -z_bar/s ; s_bar = -z_bar z / s  (1/s applied
        // once to the totals, see Model1D::final_factor)
        acc[1 + 3 * g] = fma(mb, ek[g], acc[1 + 3 * g]);
        const double zb = mb * G[g] * z[g];
        acc[2 + 3 * g] += zb;
        acc[3 + 3 * g] = fma(zb, z[g], acc[3 + 3 * g]);
      }
      constexpr int k0 = 1 + 3 * NG;
      if constexpr (BKG == BKG_EXP) {
        // E = exp(b0 + b1 t): b0_bar += mb E ; b1_bar += mb E t
        const double eb = mb * E;
        acc[k0] += eb;
        acc[k0 + 1] = fma(eb, t, acc[k0 + 1]);
      } else if constexpr (S::NB > 0) {
        double tj = mb;
#pragma unroll
        for (int j = 0; j < S::NB; ++j) {
          acc[k0 + j] += tj;
          tj *= t;
        }
      }
    }
    if constexpr (RECUR) {
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        e[g] *= r[g];
        r[g] *= M.D[g];
      }
    }
  }
  if constexpr (MOM) {
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const double dz = M.dz[g];
      acc[1 + 3 * g] += U[g][0];
      const double s1 = fma(dz, U[g][1], z0[g] * U[g][0]);  // sum mb e z
      const double s2 = fma(z0[g], fma(2.0 * dz, U[g][1], z0[g] * U[g][0]), dz * dz * U[g][2]);
      acc[2 + 3 * g] = fma(M.A[g], s1, acc[2 + 3 * g]);
      acc[3 + 3 * g] = fma(M.A[g], s2, acc[3 + 3 * g]);
    }
    constexpr int k0 = 1 + 3 * NG;
    if constexpr (BKG == BKG_EXP) {
      acc[k0] += T[0];
      acc[k0 + 1] += fma(M.dt, T[1], t0 * T[0]);
    } else if constexpr (S::NB > 0) {
      // sum_k mb (t0 + k dt)^j = sum_l C(j, l) t0^(j-l) dt^l T_l
      constexpr double C[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
      double D[S::NB];
      double dtp = 1.0;
#pragma unroll
      for (int l = 0; l < S::NB; ++l) {
        D[l] = dtp * T[l];
        dtp *= M.dt;
      }
#pragma unroll
      for (int j = 0; j < S::NB; ++j) {
        double sj = 0.0, t0p = 1.0;
#pragma unroll
        for (int l = j; l >= 0; --l) {
          sj = fma(C[j][l] * t0p, D[l], sj);
          t0p *= t0;
        }
        acc[k0 + j] += sj;
      }
    }
  }
}

}  // namespace hf
