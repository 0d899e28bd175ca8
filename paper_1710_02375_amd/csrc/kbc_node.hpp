// Per-node arithmetic of the KBC step in deviation form.
//
// The state of a node is the deviation d_i = f_i - W_i.  The arithmetic keeps
// every quantity as a deviation from the rest state so that FP32 does not lose
// the O(u) information against the O(1) weights:
//   rho~ = sum d_i, j = sum c_i d_i, rho = 1 + rho~, u = j / rho;
//   f^eq_i - W_i = W_i (rho~ + rho E_i), E_i = prod_a (1 + e_a(c_ia)) - 1,
// where e_a(c) are the per-axis deviations of the entropic equilibrium
// f^eq_i = rho W_i prod_a (2 - s_a) x_a^{c_ia}, s_a = sqrt(1 + 3 u_a^2),
// x_a = (2 u_a + s_a)/(1 - u_a)  (minimiser of H under mass and momentum,
// Sec. II.A Eqs. 4-5):
//   sigma = 3u^2/(1+s) (= s - 1),  e(0) = -sigma,
//   X = (3u + sigma)/(1 - u) (= x - 1),  e(+1) = X - sigma - sigma X,
//   Y = -(3u + sigma)/(2u + s) (= 1/x - 1),  e(-1) = Y - sigma - sigma Y.
#pragma once

#include "lbm_device.hpp"

namespace kbc {

template <typename R>
struct AxisEq {
  R e0, ep, em;   // equilibrium factor deviations for c = 0, +1, -1
  R g0, gp, gm;   // 1 / (w(c) (1 + e(c)))
};

template <typename R>
__device__ __forceinline__ AxisEq<R> axis_eq(R u) {
  AxisEq<R> A;
  const R uu = u * u;
  const R s = fsqrt(R(1) + R(3) * uu);
  const R sig = R(3) * uu * frcp(R(1) + s);
  const R t = R(3) * u + sig;
  const R X = t * frcp(R(1) - u);
  const R Y = -t * frcp(R(2) * u + s);
  A.e0 = -sig;
  A.ep = X - sig - sig * X;
  A.em = Y - sig - sig * Y;
  const R iz = frcp(R(1) - sig);   // 1 / (2 - s)
  A.g0 = R(1.5) * iz;
  A.gp = R(6) * iz * (R(1) + Y);
  A.gm = R(6) * iz * (R(1) + X);
  return A;
}

template <typename R>
__device__ __forceinline__ R sel_e(const AxisEq<R>& A, int c) {
  return c == 0 ? A.e0 : (c > 0 ? A.ep : A.em);
}
template <typename R>
__device__ __forceinline__ R sel_g(const AxisEq<R>& A, int c) {
  return c == 0 ? A.g0 : (c > 0 ? A.gp : A.gm);
}

// E_i for population i from the per-axis deviations (accumulated as
// E <- E + e + E e, exact in exact arithmetic).
template <int Q, typename R>
__device__ __forceinline__ R eq_E(const AxisEq<R> (&A)[3], int i) {
  R E = sel_e(A[0], cx(i));
  {
    const R e = sel_e(A[1], cy(i));
    E = E + e + E * e;
  }
  if (Q == 27) {
    const R e = sel_e(A[2], cz<Q>(i));
    E = E + e + E * e;
  }
  return E;
}

// Equilibrium deviations f^eq_i - W_i for given rho~ = rho - 1 and u.
template <int Q, typename R>
__device__ __forceinline__ void feq_dev(R rt, const R (&u)[3], R (&out)[Q]) {
  AxisEq<R> A[3];
#pragma unroll
  for (int a = 0; a < dims<Q>(); ++a) A[a] = axis_eq(u[a]);
  if (dims<Q>() == 2) A[2] = A[1];   // unused in 2D
  const R rho = R(1) + rt;
#pragma unroll
  for (int i = 0; i < Q; ++i) out[i] = R(weight<Q>(i)) * (rt + rho * eq_E<Q>(A, i));
}

// Moments of a deviation state.
template <int Q, typename R>
__device__ __forceinline__ void moments_dev(const R (&d)[Q], R& rt, R (&j)[3]) {
  rt = R(0);
  j[0] = j[1] = j[2] = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    rt += d[i];
    if (cx(i) > 0) j[0] += d[i];
    if (cx(i) < 0) j[0] -= d[i];
    if (cy(i) > 0) j[1] += d[i];
    if (cy(i) < 0) j[1] -= d[i];
    if (cz<Q>(i) > 0) j[2] += d[i];
    if (cz<Q>(i) < 0) j[2] -= d[i];
  }
}

// ---------------------------------------------------------------------------
// Shear part of Delta = f - f^eq (Sec. II.A, Eqs. 2-3) in the natural moment
// basis: the deviatoric second-order moments.  With P = sum Delta c c,
// T = tr P and Dev = P - T/D I:
//   Delta s_i = Dev_aa / 2            if c_i = +-e_a,
//   Delta s_i = c_ia c_ib P_ab / 4    if c_i has exactly two non-zero a != b,
//   Delta s_i = 0                     otherwise;
// with the trace moved into s: rest -T, faces +T/(2D).
// ---------------------------------------------------------------------------
template <int Q, typename R>
struct Shear {
  R Dxx, Dyy, Dzz, Pxy, Pxz, Pyz, T;
};

template <int Q, typename R>
__device__ __forceinline__ Shear<Q, R> shear_moments(const R (&delta)[Q]) {
  R Pxx = R(0), Pyy = R(0), Pzz = R(0), Pxy = R(0), Pxz = R(0), Pyz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R v = delta[i];
    if (cx(i) != 0) Pxx += v;
    if (cy(i) != 0) Pyy += v;
    if (cz<Q>(i) != 0) Pzz += v;
    if (cx(i) * cy(i) > 0) Pxy += v;
    if (cx(i) * cy(i) < 0) Pxy -= v;
    if (cx(i) * cz<Q>(i) > 0) Pxz += v;
    if (cx(i) * cz<Q>(i) < 0) Pxz -= v;
    if (cy(i) * cz<Q>(i) > 0) Pyz += v;
    if (cy(i) * cz<Q>(i) < 0) Pyz -= v;
  }
  Shear<Q, R> S;
  S.Pxy = Pxy;
  S.Pxz = Pxz;
  S.Pyz = Pyz;
  if (Q == 27) {
    S.T = Pxx + Pyy + Pzz;
    const R t3 = S.T * R(1.0 / 3.0);
    S.Dxx = Pxx - t3;
    S.Dyy = Pyy - t3;
    S.Dzz = -(S.Dxx + S.Dyy);   // trace exactly zero
  } else {
    S.T = Pxx + Pyy;
    S.Dxx = R(0.5) * (Pxx - Pyy);
    S.Dyy = -S.Dxx;
    S.Dzz = R(0);
  }
  return S;
}

template <int Q, typename R>
__device__ __forceinline__ R shear_pop(const Shear<Q, R>& S, int i, R ts) {
  const int n = nnz<Q>(i);
  if (n == 1) {
    const R dev = cx(i) != 0 ? S.Dxx : (cy(i) != 0 ? S.Dyy : S.Dzz);
    return R(0.5) * dev + ts * R(0.5 / dims<Q>());
  }
  if (n == 2) {
    const R p = (cx(i) != 0 && cy(i) != 0) ? S.Pxy : ((cx(i) != 0) ? S.Pxz : S.Pyz);
    const int sgn = (cx(i) != 0 && cy(i) != 0) ? cx(i) * cy(i)
                    : (cx(i) != 0 ? cx(i) * cz<Q>(i) : cy(i) * cz<Q>(i));
    return sgn > 0 ? R(0.25) * p : R(-0.25) * p;
  }
  if (n == 0) return -ts;
  return R(0);
}

// Removes the mass and momentum that rounding left in Delta h: in exact
// arithmetic sum dh = sum c dh = 0; the correction uses the rest and axis
// populations (columns of the inverse moment basis for rho and j).
template <int Q, typename R>
__device__ __forceinline__ void project_conserved(R (&dh)[Q]) {
  R m = R(0), J[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    m += dh[i];
    if (cx(i) > 0) J[0] += dh[i];
    if (cx(i) < 0) J[0] -= dh[i];
    if (cy(i) > 0) J[1] += dh[i];
    if (cy(i) < 0) J[1] -= dh[i];
    if (cz<Q>(i) > 0) J[2] += dh[i];
    if (cz<Q>(i) < 0) J[2] -= dh[i];
  }
  dh[rest<Q>()] -= m;
#pragma unroll
  for (int a = 0; a < dims<Q>(); ++a) {
    dh[axis_pop<Q>(a, +1)] -= R(0.5) * J[a];
    dh[axis_pop<Q>(a, -1)] += R(0.5) * J[a];
  }
}

// ---------------------------------------------------------------------------
// gamma in FP64 for near-equilibrium nodes of the FP32 paths (only the
// deferred FP64 pass calls it, so it holds Delta in registers): Delta in
// FP64 from the stored values, its shear part, the conservation projection
// of Delta h, and the two scalar products with weight 1/f^eq.
// ---------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ double gamma_fp64(const float (&d)[Q], double beta, int trace_in_s) {
  double rt = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double v = d[i];
    rt += v;
    j[0] += cx(i) * v;
    j[1] += cy(i) * v;
    j[2] += cz<Q>(i) * v;
  }
  const double rho = 1.0 + rt, ir = 1.0 / rho;
  AxisEq<double> A[3];
#pragma unroll
  for (int a = 0; a < dims<Q>(); ++a) A[a] = axis_eq(j[a] * ir);
  if (dims<Q>() == 2) A[2] = A[1];   // unused in 2D
  // Delta and its second moments.
  double dl[Q];
  double P[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    dl[i] = (double)d[i] - weight<Q>(i) * (rt + rho * eq_E<Q>(A, i));
    P[0] += cx(i) * cx(i) * dl[i];
    P[1] += cy(i) * cy(i) * dl[i];
    P[2] += cz<Q>(i) * cz<Q>(i) * dl[i];
    P[3] += cx(i) * cy(i) * dl[i];
    P[4] += cx(i) * cz<Q>(i) * dl[i];
    P[5] += cy(i) * cz<Q>(i) * dl[i];
  }
  Shear<Q, double> S;
  S.Pxy = P[3];
  S.Pxz = P[4];
  S.Pyz = P[5];
  if (Q == 27) {
    S.T = P[0] + P[1] + P[2];
    S.Dxx = P[0] - S.T / 3.0;
    S.Dyy = P[1] - S.T / 3.0;
    S.Dzz = -(S.Dxx + S.Dyy);
  } else {
    S.T = P[0] + P[1];
    S.Dxx = 0.5 * (P[0] - P[1]);
    S.Dyy = -S.Dxx;
    S.Dzz = 0.0;
  }
  const double ts = trace_in_s ? S.T : 0.0;
  // Mass and momentum left in Delta h by rounding.
  double m = 0.0, J[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double h = dl[i] - shear_pop<Q>(S, i, ts);
    m += h;
    J[0] += cx(i) * h;
    J[1] += cy(i) * h;
    J[2] += cz<Q>(i) * h;
  }
  // The two scalar products with weight 1/f^eq.
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double s = shear_pop<Q>(S, i, ts);
    double h = dl[i] - s;
    if (i == rest<Q>()) h -= m;
#pragma unroll
    for (int ax = 0; ax < dims<Q>(); ++ax) {
      if (i == axis_pop<Q>(ax, +1)) h -= 0.5 * J[ax];
      if (i == axis_pop<Q>(ax, -1)) h += 0.5 * J[ax];
    }
    double inv = ir * sel_g(A[0], cx(i)) * sel_g(A[1], cy(i));
    if (Q == 27) inv *= sel_g(A[2], cz<Q>(i));
    a += s * h * inv;
    b += h * h * inv;
  }
  if (!(b > 0.0)) return 2.0;
  return 1.0 / beta - (2.0 - 1.0 / beta) * a / b;
}


struct CollideOut {
  float gamma;
  int fp64;
};

// ---------------------------------------------------------------------------
// KBC collision of one node in place (Sec. II.A, Eqs. 1, 3, 6):
//   f' = f - beta (2 Delta s + gamma Delta h),
//   gamma = 1/beta - (2 - 1/beta) <Ds|Dh> / <Dh|Dh>, <X|Y> = sum X_i Y_i / f^eq_i,
// gamma = 2 when <Dh|Dh> = 0 and in LBGK mode.  Returns false (state left
// unchanged) if rho <= 0, |u_a| >= 1 or the state is not finite.
// ---------------------------------------------------------------------------
template <typename R>
struct CollideParams {
  R beta, inv_beta;
  double beta_d;
  int lbgk, trace_in_s;
  float near_eq;
};

// DEFER = true: a near-equilibrium node of an FP32 path keeps the FP32 gamma
// and reports out.fp64 = 1, so that the caller can redo it in FP64 later (the
// bulk kernel does, to keep its register budget); DEFER = false computes the
// FP64 gamma in place.
//
// The arithmetic follows the tensor-product structure of the lattice
// (population index a + 3b + 9c for velocity (a-1, b-1, c-1)):
//   - rho~ and j from 1-D sums along x, then y and z;
//   - f^eq_i - W_i = rho p_x(a) p_y(b) p_z(c) - w_a w_b w_c with the 1-D
//     equilibria p(c) = w(c)(1 + e(c)), built pairwise as deviations
//     (rho folded into the x factor), no cancellation against W_i;
//   - the second moments of Delta and its mass and momentum (for the
//     conservation projection) from one reduction tree along z, y, x.
template <int Q, typename R, bool DEFER = false>
__device__ __forceinline__ bool collide(R (&d)[Q], const CollideParams<R>& P, CollideOut& out) {
  constexpr int D = dims<Q>();
  constexpr int NR = Q / 3;   // x-rows: index b (2D) or b + 3c (3D)
  constexpr int RST = rest<Q>();
  // ---- moments (Eq. 5): sums along x, then over rows -----------------------
  R srow[NR], jrow[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const R pm = d[3 * r + 2] + d[3 * r];
    jrow[r] = d[3 * r + 2] - d[3 * r];
    srow[r] = pm + d[3 * r + 1];
  }
  R rt, j[3];
  if (Q == 27) {
    const R sb0 = srow[0] + srow[3] + srow[6];
    const R sb1 = srow[1] + srow[4] + srow[7];
    const R sb2 = srow[2] + srow[5] + srow[8];
    rt = (sb0 + sb2) + sb1;
    j[1] = sb2 - sb0;
    j[2] = (srow[6] + srow[7] + srow[8]) - (srow[0] + srow[1] + srow[2]);
    j[0] = ((jrow[0] + jrow[1] + jrow[2]) + (jrow[3] + jrow[4] + jrow[5])) +
           (jrow[6] + jrow[7] + jrow[8]);
  } else {
    rt = (srow[0] + srow[2]) + srow[1];
    j[1] = srow[2] - srow[0];
    j[2] = R(0);
    j[0] = (jrow[0] + jrow[2]) + jrow[1];
  }
  const R rho = R(1) + rt;
  const R ir = frcp(rho);
  // Size of the terms that cancel in Delta = d - (f^eq - W): FP32 keeps
  // Delta to ~6e-8 of sqrt(dscale) in the 1/W-weighted norm.
  const R dscale = rt * rt + R(3) * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]);
  const R u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
  const bool ok = rho > R(0) && u[0] < R(1) && u[0] > R(-1) && u[1] < R(1) && u[1] > R(-1) &&
                  u[2] < R(1) && u[2] > R(-1);
  if (!ok) {
    out.gamma = 2.0f;
    out.fp64 = 0;
    return false;
  }
  // ---- per-axis equilibrium factors (Eqs. 4-5) -----------------------------
  AxisEq<R> A[3];
#pragma unroll
  for (int a = 0; a < D; ++a) A[a] = axis_eq(u[a]);
  if (D == 2) A[2] = A[1];   // unused in 2D
  const R wv[3] = {R(1.0 / 6.0), R(2.0 / 3.0), R(1.0 / 6.0)};
  R ex[3] = {A[0].em, A[0].e0, A[0].ep};
  R ey[3] = {A[1].em, A[1].e0, A[1].ep};
  R ez[3] = {A[2].em, A[2].e0, A[2].ep};
  // rho p_x - w, p_y, p_y - w, p_z - w
  R dxr[3], py[3], dy[3], dz[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dxr[k] = wv[k] * (rt + rho * ex[k]);
    dy[k] = wv[k] * ey[k];
    py[k] = wv[k] + dy[k];
    dz[k] = wv[k] * ez[k];
  }
  // ---- Delta = f~ - (f^eq - W) ---------------------------------------------
  // f^eq_i - W_i = dxy p_z + w_a w_b (p_z - w_c) = w_c dxy + pxy (p_z - w_c)
  // with dxy = rho p_x p_y - w_a w_b and pxy = rho p_x p_y.
  R dl[Q];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R dxy = dxr[a] * py[b] + wv[a] * dy[b];   // rho p_x p_y - w_a w_b
      if (Q == 27) {
        const R pxy = dxy + R(w1d(a - 1) * w1d(b - 1));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int i = a + 3 * b + 9 * c;
          dl[i] = (d[i] - wv[c] * dxy) - pxy * dz[c];
        }
      } else {
        const int i = a + 3 * b;
        dl[i] = d[i] - dxy;
      }
    }
  // ---- second moments, mass and momentum of Delta --------------------------
  // m0/m1/m2: zeroth, first and second moment along z of each (a, b) column.
  R m0[9], m1[9], m2[9];
#pragma unroll
  for (int ab = 0; ab < 9; ++ab) {
    if (Q == 27) {
      const R lo = dl[ab], mid = dl[ab + 9], hi = dl[ab + 18];
      m2[ab] = hi + lo;
      m1[ab] = hi - lo;
      m0[ab] = m2[ab] + mid;
    } else {
      m0[ab] = dl[ab];
      m1[ab] = R(0);
      m2[ab] = R(0);
    }
  }
  R n0[3], n1[3], n2[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    n2[a] = m0[a + 6] + m0[a];
    n1[a] = m0[a + 6] - m0[a];
    n0[a] = n2[a] + m0[a + 3];
  }
  const R Rm = (n0[0] + n0[2]) + n0[1];
  const R Jx = n0[2] - n0[0];
  const R Pxx = n0[2] + n0[0];
  const R Jy = (n1[0] + n1[2]) + n1[1];
  const R Pxy = n1[2] - n1[0];
  const R Pyy = (n2[0] + n2[2]) + n2[1];
  R Jz = R(0), Pxz = R(0), Pyz = R(0), Pzz = R(0);
  if (Q == 27) {
    R k0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) k0[a] = (m1[a] + m1[a + 6]) + m1[a + 3];
    Jz = (k0[0] + k0[2]) + k0[1];
    Pxz = k0[2] - k0[0];
    Pyz = (m1[6] + m1[7] + m1[8]) - (m1[0] + m1[1] + m1[2]);
    Pzz = ((m2[0] + m2[1] + m2[2]) + (m2[3] + m2[4] + m2[5])) + (m2[6] + m2[7] + m2[8]);
  }
  // Exact-conservation projection: mass and momentum that rounding left in
  // Delta go to the rest and axis populations (columns of the inverse moment
  // basis for rho and j); the second moments are unchanged by it.
  dl[RST] -= Rm;
  dl[RST + 1] -= R(0.5) * Jx;
  dl[RST - 1] += R(0.5) * Jx;
  dl[RST + 3] -= R(0.5) * Jy;
  dl[RST - 3] += R(0.5) * Jy;
  if (Q == 27) {
    dl[RST + 9] -= R(0.5) * Jz;
    dl[RST - 9] += R(0.5) * Jz;
  }
  // ---- shear part (Eqs. 2-3): deviatoric second moments --------------------
  R T, Dxx, Dyy, Dzz;
  if (Q == 27) {
    T = Pxx + Pyy + Pzz;
    const R t3 = T * R(1.0 / 3.0);
    Dxx = Pxx - t3;
    Dyy = Pyy - t3;
    Dzz = -(Dxx + Dyy);
  } else {
    T = Pxx + Pyy;
    Dxx = R(0.5) * (Pxx - Pyy);
    Dyy = -Dxx;
    Dzz = R(0);
  }
  const R ts = P.trace_in_s ? T : R(0);
  const R tf = ts * R(0.5 / D);
  const R Fx = R(0.5) * Dxx + tf, Fy = R(0.5) * Dyy + tf, Fz = R(0.5) * Dzz + tf;
  const R Exy = R(0.25) * Pxy, Exz = R(0.25) * Pxz, Eyz = R(0.25) * Pyz;
  auto ds_of = [&](int i) -> R {
    const int n = nnz<Q>(i);
    if (n == 1) return cx(i) != 0 ? Fx : (cy(i) != 0 ? Fy : Fz);
    if (n == 2) {
      const R e = (cx(i) != 0 && cy(i) != 0) ? Exy : (cx(i) != 0 ? Exz : Eyz);
      const int sg = cx(i) * cy(i) + cx(i) * cz<Q>(i) + cy(i) * cz<Q>(i);
      return sg > 0 ? e : -e;
    }
    if (n == 0) return -ts;
    return R(0);
  };
  // ---- stabiliser gamma (Eq. 6) --------------------------------------------
  R gamma = R(2);
  out.fp64 = 0;
  if (!P.lbgk) {
    const R gx[3] = {ir * A[0].gm, ir * A[0].g0, ir * A[0].gp};
    const R gy[3] = {A[1].gm, A[1].g0, A[1].gp};
    const R gz[3] = {A[2].gm, A[2].g0, A[2].gp};
    // 1/f^eq_i = gx(a) gy(b) gz(c): the sums over c of each (a, b) column
    // are taken first and weighted by gx gy once per column.
    R a = R(0), b = R(0), ss = R(0);
#pragma unroll
    for (int bb = 0; bb < 3; ++bb)
#pragma unroll
      for (int aa = 0; aa < 3; ++aa) {
        R bc = R(0), ac = R(0), sc = R(0);
#pragma unroll
        for (int cc = 0; cc < (Q == 27 ? 3 : 1); ++cc) {
          const int i = aa + 3 * bb + 9 * cc;
          const int n = nnz<Q>(i);
          const bool has_s = n == 1 || n == 2 || n == 0;
          const R si = ds_of(i);
          const R hi = has_s ? dl[i] - si : dl[i];       // Delta h_i
          const R hz = (Q == 27) ? hi * gz[cc] : hi;
          bc += hz * hi;
          if (has_s) {
            ac += hz * si;
            sc += (Q == 27) ? si * si * gz[cc] : si * si;
          }
        }
        const R gxy = gx[aa] * gy[bb];
        b += gxy * bc;
        a += gxy * ac;
        ss += gxy * sc;
      }
    const R dd = ss + R(2) * a + b;   // <Delta|Delta>
    // FP32 cannot resolve gamma when <Delta|Delta> is small against the
    // terms that cancelled in Delta (relative threshold near_eq on dscale),
    // or when <Dh|Dh> nears the bottom of the normal range (products
    // underflow, the reciprocal overflows): those nodes take gamma from FP64.
    // Not when <Ds|Ds> and <Dh|Dh> are both zero (the rest state, or
    // deviations so small that every product underflows): |gamma Dh| is then
    // of the order of |Ds| + |Dh|, far below the population rounding.
    const bool near_eq = sizeof(R) == 4 && (dd < R(P.near_eq) * dscale || b < R(1e-36)) &&
                         (b > R(0) || ss > R(0));
    if (near_eq && DEFER) {
      out.fp64 = 1;
      if (b > R(1e-36)) gamma = P.inv_beta - (R(2) - P.inv_beta) * a * frcp(b);
    } else if (near_eq) {
      float tmp[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) tmp[i] = (float)d[i];
      gamma = (R)gamma_fp64<Q>(tmp, P.beta_d, P.trace_in_s);
      out.fp64 = 1;
    } else if (b > R(sizeof(R) == 8 ? 1e-300 : 1e-36)) {
      // Below that <Dh|Dh> the reciprocal would overflow; Dh is then
      // negligible and gamma = 2 is kept.
      gamma = P.inv_beta - (R(2) - P.inv_beta) * (sizeof(R) == 8 ? a / b : a * frcp(b));
    }
  }
  // ---- post-collision state (Eqs. 1, 3): f - beta (2 Ds + gamma Dh) --------
  const R bg = P.beta * gamma, b2 = R(2) * P.beta;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R si = ds_of(i);
    const int n = nnz<Q>(i);
    const bool has_s = n == 1 || n == 2 || n == 0;
    const R hi = has_s ? dl[i] - si : dl[i];
    d[i] = has_s ? d[i] - bg * hi - b2 * si : d[i] - bg * hi;
  }
  out.gamma = (float)gamma;
  return true;
}

// ---------------------------------------------------------------------------
// Forced KBC collision in FP64 (Sec. III.B): body force F enters by the exact
// difference method and the stabiliser uses the shifted scalar product,
//   f' = f - beta (2 Delta s + gamma Delta h) + f^eq(rho, u + du) - f^eq(rho, u),
//   gamma = 1/beta - (2 - 1/beta) <Ds|Dh>_s / <Dh|Dh>_s,
//   <X|Y>_s = sum X_i Y_i / f^eq_i(rho, u + du),  du = F / rho,
// with Delta s and Delta h about f^eq(rho, u).  Written as
//   f' - W = (f^eq(rho, u + du) - W) + Delta - beta (2 Delta s + gamma Delta h).
// The state stays in its storage type V (the deviations f - W as stored, so
// FP32 storage keeps 27 single registers); every quantity is formed in FP64,
// Delta_i = d_i - (f^eq_i - W_i) again in each pass from the tensor-product
// factors of the equilibria.  The result is written back into d, rounded to
// V.  FP64 leaves no mass or momentum in Delta worth projecting.
// Returns false (state left unchanged) if rho <= 0, |u_a| >= 1,
// |u_a + du_a| >= 1 or the state is not finite.
// ---------------------------------------------------------------------------
template <int Q, typename V>
__device__ __forceinline__ bool collide_forced(V* p, int64_t stride, const double (&F)[3],
                                               double beta, int lbgk, int trace_in_s,
                                               float& gamma_out) {
  using R = double;
  constexpr int D = dims<Q>();
  // Population i of the node; read again in every pass (from cache), the
  // memory clobbers between passes keep the compiler from holding them all.
  auto ld = [&](int i) -> R { return (R)p[i * stride]; };
  R rt = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R v = ld(i);
    rt += v;
    if (cx(i)) j[0] += R(cx(i)) * v;
    if (cy(i)) j[1] += R(cy(i)) * v;
    if (cz<Q>(i)) j[2] += R(cz<Q>(i)) * v;
  }
  const R rho = R(1) + rt;
  const R ir = R(1) / rho;
  const R u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
  const R us[3] = {u[0] + F[0] * ir, u[1] + F[1] * ir, u[2] + F[2] * ir};
  bool ok = rho > R(0) && isfinite(rho);
#pragma unroll
  for (int a = 0; a < 3; ++a) ok = ok && fabs(u[a]) < R(1) && fabs(us[a]) < R(1) && isfinite(us[a]);
  if (!ok) {
    gamma_out = 2.0f;
    return false;
  }
  const R wv[3] = {R(1.0 / 6.0), R(2.0 / 3.0), R(1.0 / 6.0)};
  // Per-axis factors at (rho, v) (rho folded into x): dxr = rho p_x - w,
  // py = p_y, dy = p_y - w, dz = p_z - w; f^eq_i - W_i from them.
  struct Fac {
    R dxr[3], py[3], dy[3], dz[3];
    R g[3][3];   // 1 / (w (1 + e)) per axis and c, x row times 1/rho
  };
  auto factors = [&](const R (&v)[3], Fac& f) {
    AxisEq<R> A[3];
#pragma unroll
    for (int a = 0; a < D; ++a) A[a] = axis_eq(v[a]);
    if (D == 2) A[2] = A[1];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      f.g[a][0] = A[a].gm;
      f.g[a][1] = A[a].g0;
      f.g[a][2] = A[a].gp;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) f.g[0][k] *= ir;
    const R ex[3] = {A[0].em, A[0].e0, A[0].ep};
    const R ey[3] = {A[1].em, A[1].e0, A[1].ep};
    const R ez[3] = {A[2].em, A[2].e0, A[2].ep};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      f.dxr[k] = wv[k] * (rt + rho * ex[k]);
      f.dy[k] = wv[k] * ey[k];
      f.py[k] = wv[k] + f.dy[k];
      f.dz[k] = wv[k] * ez[k];
    }
  };
  auto eqdev = [&](int i, const Fac& f) -> R {
    const int a = i % 3, b = (i / 3) % 3, c = i / 9;
    const R dxy = f.dxr[a] * f.py[b] + wv[a] * f.dy[b];   // rho p_x p_y - w_a w_b
    if (Q == 27) return wv[c] * dxy + (dxy + R(w1d(a - 1) * w1d(b - 1))) * f.dz[c];
    return dxy;
  };
  Fac fu, fs;
  factors(u, fu);
  factors(us, fs);
  // Second moments of Delta.
  R Pxx = R(0), Pyy = R(0), Pzz = R(0), Pxy = R(0), Pxz = R(0), Pyz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R dl = ld(i) - eqdev(i, fu);
    if (cx(i)) Pxx += dl;
    if (cy(i)) Pyy += dl;
    if (cz<Q>(i)) Pzz += dl;
    if (cx(i) * cy(i)) Pxy += R(cx(i) * cy(i)) * dl;
    if (cx(i) * cz<Q>(i)) Pxz += R(cx(i) * cz<Q>(i)) * dl;
    if (cy(i) * cz<Q>(i)) Pyz += R(cy(i) * cz<Q>(i)) * dl;
  }
  R T, Dxx, Dyy, Dzz;
  if (Q == 27) {
    T = Pxx + Pyy + Pzz;
    const R t3 = T * R(1.0 / 3.0);
    Dxx = Pxx - t3;
    Dyy = Pyy - t3;
    Dzz = -(Dxx + Dyy);
  } else {
    T = Pxx + Pyy;
    Dxx = R(0.5) * (Pxx - Pyy);
    Dyy = -Dxx;
    Dzz = R(0);
  }
  const R ts = trace_in_s ? T : R(0);
  const R tf = ts * R(0.5 / D);
  const R Fx = R(0.5) * Dxx + tf, Fy = R(0.5) * Dyy + tf, Fz = R(0.5) * Dzz + tf;
  const R Exy = R(0.25) * Pxy, Exz = R(0.25) * Pxz, Eyz = R(0.25) * Pyz;
  auto ds_of = [&](int i) -> R {
    const int n = nnz<Q>(i);
    if (n == 1) return cx(i) != 0 ? Fx : (cy(i) != 0 ? Fy : Fz);
    if (n == 2) {
      const R e = (cx(i) != 0 && cy(i) != 0) ? Exy : (cx(i) != 0 ? Exz : Eyz);
      const int sg = cx(i) * cy(i) + cx(i) * cz<Q>(i) + cy(i) * cz<Q>(i);
      return sg > 0 ? e : -e;
    }
    if (n == 0) return -ts;
    return R(0);
  };
  R gamma = R(2);
  if (!lbgk) {
    asm volatile("" ::: "memory");
    // 1/f^eq_i(rho, u + du) = g_x(a) g_y(b) g_z(c).
    R a = R(0), b = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R si = ds_of(i);
      const R hi = (ld(i) - eqdev(i, fu)) - si;
      R g = fs.g[0][i % 3] * fs.g[1][(i / 3) % 3];
      if (Q == 27) g *= fs.g[2][i / 9];
      const R hg = hi * g;
      b += hg * hi;
      a += hg * si;
    }
    if (b != R(0)) gamma = R(1) / beta - (R(2) - R(1) / beta) * a / b;
  }
  const R bg = beta * gamma, b2 = R(2) * beta;
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R si = ds_of(i);
    const R dl = ld(i) - eqdev(i, fu);
    const R hi = dl - si;
    p[i * stride] = (V)(eqdev(i, fs) + dl - bg * hi - b2 * si);
  }
  gamma_out = (float)gamma;
  return true;
}

// Grad's approximation (Sec. II.C.1) as a deviation from W_i, cs^2 = 1/3:
//   f*_i - W_i = W_i [ rho - 1 + 3 rho c.v + (9/2)(Pi - rho/3 I):(c c - I/3) ].
// Pi is given as (xx, yy, zz, xy, xz, yz).
template <int Q, typename R>
__device__ __forceinline__ R grad_dev(int i, R rho, const R (&v)[3], const R (&Pi)[6]) {
  const R c0 = R(cx(i)), c1 = R(cy(i)), c2 = R(cz<Q>(i));
  const R third = R(1.0 / 3.0);
  const R cv = c0 * v[0] + c1 * v[1] + c2 * v[2];
  const R r3 = rho * third;
  R contr = (Pi[0] - r3) * (c0 * c0 - third) + (Pi[1] - r3) * (c1 * c1 - third) +
            R(2) * Pi[3] * c0 * c1;
  if (Q == 27)
    contr += (Pi[2] - r3) * (c2 * c2 - third) + R(2) * Pi[4] * c0 * c2 + R(2) * Pi[5] * c1 * c2;
  return R(weight<Q>(i)) * (rho - R(1) + R(3) * rho * cv + R(4.5) * contr);
}

}  // namespace kbc
