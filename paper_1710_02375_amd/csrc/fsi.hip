// Structure solver and two-way coupling (Sec. II.B and II.C), host code.
//
// The structure is a rectangular beam in plane strain: total-Lagrangian
// Saint Venant-Kirchhoff material (S = lambda tr(E) I + 2 mu E, E = (F^T F - I)/2,
// P = F S), 9-node biquadratic elements with 3 x 3 Gauss points, consistent
// mass, and the two-field (u, v) formulation integrated with the
// one-step-theta scheme:
//   M (v1 - v0)/dt = theta (f_ext1 - f_int(u1)) + (1 - theta)(f_ext0 - f_int(u0)),
//   (u1 - u0)/dt   = theta v1 + (1 - theta) v0.
// With v1 eliminated the step is a nonlinear system in u1, solved by Newton
// with the exact tangent M/(theta dt^2) + theta K_T(u1) in banded storage
// (nodes numbered across the thickness first, so the band is narrow) and an
// LU factorisation without pivoting (the mass term makes the matrix
// diagonally dominant enough).  The structure has ~10^2-10^3 unknowns: it
// runs on the host, between the fluid steps on the GPU.
//
// The coupling is the conventional serial staggered scheme: the fluid steps
// with the body surface of the structure's current state, the traction of
// the fluid on the beam is sampled at the Gauss points of its wet edges
// (lbm_wall_force), the beam takes its step with the consistent nodal loads,
// and the body surface (a closed polygon: the beam's wet edges and a static
// chain closing the outline) is set for the next fluid step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/lbm.h"

struct lbm_fem {
  int nex = 0, ney = 0, nxn = 0, nyn = 0, nn = 0, ndof = 0, bw = 0;
  double x0 = 0, y0 = 0, L = 0, H = 0, rho = 0, lam = 0, mu = 0, dt = 0, theta = 0.5;
  std::vector<double> X;        // reference coordinates, 2 per node
  std::vector<int> conn;        // 9 nodes per element, local (a, b) -> 3 a + b
  double N[9][9], dN[9][2][9], w[9];   // per Gauss point: N_a, dN_a/dX_J, weight
  std::vector<char> fixed;      // per DOF
  std::vector<double> M;        // banded mass, ndof x (2 bw + 1)
  std::vector<double> u, v, fext;
  // Newton scratch.
  std::vector<double> K, R, fi, du;
};

struct lbm_fsi {
  lbm_ctx* ctx = nullptr;
  int inst = 0;
  lbm_fem* fem = nullptr;
  std::vector<double> arc;      // static chain, 2 per point
  std::vector<int> chain;       // wet-boundary node order (bottom, tip, top)
  // Quadrature of the wet edges: 3 nodes and 3 shape values per point.
  std::vector<double> xq, nq, wq, tq, shp;
  std::vector<int> qn;
  std::vector<double> verts, vvel;
  std::vector<int> tris;
};

namespace {

inline double& band(std::vector<double>& A, int bw, int i, int j) {
  return A[(size_t)i * (2 * bw + 1) + (j - i + bw)];
}

void lagrange3(double t, double* l, double* dl) {
  l[0] = 0.5 * t * (t - 1.0);
  l[1] = 1.0 - t * t;
  l[2] = 0.5 * t * (t + 1.0);
  dl[0] = t - 0.5;
  dl[1] = -2.0 * t;
  dl[2] = t + 0.5;
}

// f_int (and, if K is non-null, the tangent d f_int / d u added to K times
// scale) at displacement u.
void element_loop(lbm_fem* s, const double* u, double* f, std::vector<double>* K, double scale) {
  std::memset(f, 0, sizeof(double) * s->ndof);
  const int ne = s->nex * s->ney;
  for (int e = 0; e < ne; ++e) {
    const int* c = &s->conn[9 * e];
    double fe[9][2] = {};
    double ke[18][18];
    if (K) std::memset(ke, 0, sizeof ke);
    for (int g = 0; g < 9; ++g) {
      double F[2][2] = {{1.0, 0.0}, {0.0, 1.0}};
      for (int a = 0; a < 9; ++a)
        for (int i = 0; i < 2; ++i)
          for (int J = 0; J < 2; ++J) F[i][J] += u[2 * c[a] + i] * s->dN[g][J][a];
      double E[2][2];
      for (int I = 0; I < 2; ++I)
        for (int J = 0; J < 2; ++J)
          E[I][J] = 0.5 * (F[0][I] * F[0][J] + F[1][I] * F[1][J] - (I == J ? 1.0 : 0.0));
      const double trE = E[0][0] + E[1][1];
      double S[2][2];
      for (int I = 0; I < 2; ++I)
        for (int J = 0; J < 2; ++J) S[I][J] = (I == J ? s->lam * trE : 0.0) + 2.0 * s->mu * E[I][J];
      double P[2][2];
      for (int i = 0; i < 2; ++i)
        for (int J = 0; J < 2; ++J) P[i][J] = F[i][0] * S[0][J] + F[i][1] * S[1][J];
      const double wg = s->w[g];
      for (int a = 0; a < 9; ++a)
        for (int i = 0; i < 2; ++i)
          fe[a][i] += wg * (P[i][0] * s->dN[g][0][a] + P[i][1] * s->dN[g][1][a]);
      if (!K) continue;
      // Unit displacement k at node b: dF = e_k x grad N_b,
      // dE_IJ = (F_kI dN_b,J + F_kJ dN_b,I)/2, dS = lam tr(dE) I + 2 mu dE,
      // dP_iJ = delta_ik dN_b,L S_LJ + F_iL dS_LJ.
      for (int b = 0; b < 9; ++b) {
        const double gb[2] = {s->dN[g][0][b], s->dN[g][1][b]};
        for (int k = 0; k < 2; ++k) {
          double dE[2][2];
          for (int I = 0; I < 2; ++I)
            for (int J = 0; J < 2; ++J) dE[I][J] = 0.5 * (F[k][I] * gb[J] + F[k][J] * gb[I]);
          const double trd = dE[0][0] + dE[1][1];
          double dS[2][2];
          for (int I = 0; I < 2; ++I)
            for (int J = 0; J < 2; ++J) dS[I][J] = (I == J ? s->lam * trd : 0.0) + 2.0 * s->mu * dE[I][J];
          double dP[2][2];
          for (int i = 0; i < 2; ++i)
            for (int J = 0; J < 2; ++J)
              dP[i][J] = (i == k ? gb[0] * S[0][J] + gb[1] * S[1][J] : 0.0) + F[i][0] * dS[0][J] +
                         F[i][1] * dS[1][J];
          for (int a = 0; a < 9; ++a)
            for (int i = 0; i < 2; ++i)
              ke[2 * a + i][2 * b + k] +=
                  wg * (dP[i][0] * s->dN[g][0][a] + dP[i][1] * s->dN[g][1][a]);
        }
      }
    }
    for (int a = 0; a < 9; ++a)
      for (int i = 0; i < 2; ++i) f[2 * c[a] + i] += fe[a][i];
    if (K)
      for (int a = 0; a < 9; ++a)
        for (int i = 0; i < 2; ++i)
          for (int b = 0; b < 9; ++b)
            for (int k = 0; k < 2; ++k)
              band(*K, s->bw, 2 * c[a] + i, 2 * c[b] + k) += scale * ke[2 * a + i][2 * b + k];
  }
}

// Solves A x = r in place (r becomes x); A banded, destroyed.
bool band_solve(std::vector<double>& A, int n, int bw, double* r) {
  for (int k = 0; k < n; ++k) {
    const double p = band(A, bw, k, k);
    if (!(std::fabs(p) > 0.0)) return false;
    const int iend = std::min(n - 1, k + bw);
    for (int i = k + 1; i <= iend; ++i) {
      const double l = band(A, bw, i, k) / p;
      if (l == 0.0) continue;
      for (int j = k + 1; j <= std::min(n - 1, k + bw); ++j) band(A, bw, i, j) -= l * band(A, bw, k, j);
      r[i] -= l * r[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double sum = r[i];
    for (int j = i + 1; j <= std::min(n - 1, i + bw); ++j) sum -= band(A, bw, i, j) * r[j];
    r[i] = sum / band(A, bw, i, i);
  }
  return true;
}

void band_matvec(const lbm_fem* s, const std::vector<double>& A, const double* x, double* y) {
  for (int i = 0; i < s->ndof; ++i) {
    double sum = 0.0;
    for (int j = std::max(0, i - s->bw); j <= std::min(s->ndof - 1, i + s->bw); ++j)
      sum += A[(size_t)i * (2 * s->bw + 1) + (j - i + s->bw)] * x[j];
    y[i] = sum;
  }
}

// Wet-boundary node chain of the beam: bottom edge from the clamped end to
// the tip, the tip edge upwards, the top edge back (counter-clockwise).
std::vector<int> wet_chain(const lbm_fem* s) {
  std::vector<int> c;
  for (int i = 0; i < s->nxn; ++i) c.push_back(s->nyn * i);
  for (int j = 1; j < s->nyn; ++j) c.push_back(j + s->nyn * (s->nxn - 1));
  for (int i = s->nxn - 2; i >= 0; --i) c.push_back((s->nyn - 1) + s->nyn * i);
  return c;
}

// Body surface of the coupled structure and the wet-edge quadrature, from
// the beam's current state.
void rebuild(lbm_fsi* f) {
  const lbm_fem* s = f->fem;
  const int nw = (int)f->chain.size(), na = (int)f->arc.size() / 2, nv = nw + na;
  f->verts.assign(3 * (size_t)nv, 0.0);
  f->vvel.assign(3 * (size_t)nv, 0.0);
  f->tris.assign(3 * (size_t)nv, 0);
  for (int k = 0; k < nw; ++k) {
    const int n = f->chain[k];
    for (int a = 0; a < 2; ++a) {
      f->verts[3 * k + a] = s->X[2 * n + a] + s->u[2 * n + a];
      f->vvel[3 * k + a] = s->v[2 * n + a];
    }
  }
  for (int k = 0; k < na; ++k)
    for (int a = 0; a < 2; ++a) f->verts[3 * (nw + k) + a] = f->arc[2 * k + a];
  for (int k = 0; k < nv; ++k) {
    f->tris[3 * k] = k;
    f->tris[3 * k + 1] = f->tris[3 * k + 2] = (k + 1) % nv;
  }
  // Gauss points of each quadratic edge element of the chain (three nodes
  // per element, consecutive along the chain): position, outward normal (the
  // tangent turned clockwise, the chain running counter-clockwise), weight.
  static const double gp[3] = {-0.7745966692414834, 0.0, 0.7745966692414834};
  static const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
  f->xq.clear();
  f->nq.clear();
  f->wq.clear();
  f->shp.clear();
  f->qn.clear();
  // Edges: bottom (nxn nodes), tip (nyn), top (nxn), sharing corner nodes.
  const int runs[3][2] = {{0, s->nxn}, {s->nxn - 1, s->nyn}, {s->nxn + s->nyn - 2, s->nxn}};
  for (const auto& r : runs) {
    for (int e = 0; e + 2 < r[1]; e += 2) {
      const int ids[3] = {f->chain[r[0] + e], f->chain[r[0] + e + 1], f->chain[r[0] + e + 2]};
      double x[3][2];
      for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a) x[k][a] = s->X[2 * ids[k] + a] + s->u[2 * ids[k] + a];
      for (int g = 0; g < 3; ++g) {
        double l[3], dl[3];
        lagrange3(gp[g], l, dl);
        double p[2], t[2];
        for (int a = 0; a < 2; ++a) {
          p[a] = l[0] * x[0][a] + l[1] * x[1][a] + l[2] * x[2][a];
          t[a] = dl[0] * x[0][a] + dl[1] * x[1][a] + dl[2] * x[2][a];
        }
        const double len = std::hypot(t[0], t[1]);
        f->xq.push_back(p[0]);
        f->xq.push_back(p[1]);
        f->nq.push_back(t[1] / len);
        f->nq.push_back(-t[0] / len);
        f->wq.push_back(gw[g] * len);
        for (int k = 0; k < 3; ++k) {
          f->qn.push_back(ids[k]);
          f->shp.push_back(l[k]);
        }
      }
    }
  }
}

lbm_status set_surface(lbm_fsi* f) {
  lbm_body b;
  std::memset(&b, 0, sizeof b);
  b.kind = LBM_BODY_MESH;
  b.nverts = (int)f->verts.size() / 3;
  b.ntris = (int)f->tris.size() / 3;
  b.verts = f->verts.data();
  b.vert_vel = f->vvel.data();
  b.tris = f->tris.data();
  return lbm_set_geometry(f->ctx, f->inst, &b);
}

}  // namespace

extern "C" {

lbm_status lbm_fem_create(const lbm_fem_desc* d, lbm_fem** out) {
  if (!d || !out) return LBM_ERR_INVALID;
  *out = nullptr;
  if (d->nex < 1 || d->ney < 1 || !(d->length > 0) || !(d->height > 0) || !(d->rho > 0) ||
      !(d->mu > 0) || !(d->lambda >= 0) || !(d->dt > 0) || !(d->theta > 0 && d->theta <= 1))
    return LBM_ERR_INVALID;
  lbm_fem* s = new lbm_fem;
  s->nex = d->nex;
  s->ney = d->ney;
  s->nxn = 2 * d->nex + 1;
  s->nyn = 2 * d->ney + 1;
  s->nn = s->nxn * s->nyn;
  s->ndof = 2 * s->nn;
  s->x0 = d->x0;
  s->y0 = d->y0;
  s->L = d->length;
  s->H = d->height;
  s->rho = d->rho;
  s->lam = d->lambda;
  s->mu = d->mu;
  s->dt = d->dt;
  s->theta = d->theta;
  // An element couples nodes up to 2 nyn + 2 apart: half band in DOFs.
  s->bw = 2 * (2 * s->nyn + 2) + 1;
  s->X.resize(2 * (size_t)s->nn);
  for (int i = 0; i < s->nxn; ++i)
    for (int j = 0; j < s->nyn; ++j) {
      const int k = j + s->nyn * i;
      s->X[2 * k] = d->x0 + d->length * i / (2.0 * d->nex);
      s->X[2 * k + 1] = d->y0 + d->height * j / (2.0 * d->ney);
    }
  for (int ex = 0; ex < d->nex; ++ex)
    for (int ey = 0; ey < d->ney; ++ey)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s->conn.push_back((2 * ey + b) + s->nyn * (2 * ex + a));
  static const double gp[3] = {-0.7745966692414834, 0.0, 0.7745966692414834};
  static const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
  const double hx = d->length / d->nex, hy = d->height / d->ney;
  for (int gi = 0; gi < 3; ++gi)
    for (int gj = 0; gj < 3; ++gj) {
      const int g = 3 * gi + gj;
      double lx[3], dlx[3], ly[3], dly[3];
      lagrange3(gp[gi], lx, dlx);
      lagrange3(gp[gj], ly, dly);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          s->N[g][3 * a + b] = lx[a] * ly[b];
          s->dN[g][0][3 * a + b] = dlx[a] * ly[b] * 2.0 / hx;
          s->dN[g][1][3 * a + b] = lx[a] * dly[b] * 2.0 / hy;
        }
      s->w[g] = gw[gi] * gw[gj] * hx * hy / 4.0;
    }
  s->M.assign((size_t)s->ndof * (2 * s->bw + 1), 0.0);
  for (size_t e = 0; e < s->conn.size() / 9; ++e) {
    const int* c = &s->conn[9 * e];
    for (int a = 0; a < 9; ++a)
      for (int b = 0; b < 9; ++b) {
        double m = 0.0;
        for (int g = 0; g < 9; ++g) m += s->w[g] * s->N[g][a] * s->N[g][b];
        m *= s->rho;
        for (int k = 0; k < 2; ++k) band(s->M, s->bw, 2 * c[a] + k, 2 * c[b] + k) += m;
      }
  }
  s->fixed.assign(s->ndof, 0);
  for (int j = 0; j < s->nyn; ++j) s->fixed[2 * j] = s->fixed[2 * j + 1] = 1;   // x = x0
  s->u.assign(s->ndof, 0.0);
  s->v.assign(s->ndof, 0.0);
  s->fext.assign(s->ndof, 0.0);
  *out = s;
  return LBM_OK;
}

lbm_status lbm_fem_destroy(lbm_fem* s) {
  delete s;
  return LBM_OK;
}

lbm_status lbm_fem_info(const lbm_fem* s, int* nodes, double* coords) {
  if (!s) return LBM_ERR_INVALID;
  if (nodes) *nodes = s->nn;
  if (coords) std::memcpy(coords, s->X.data(), sizeof(double) * s->X.size());
  return LBM_OK;
}

lbm_status lbm_fem_body_force(const lbm_fem* s, const double b[2], double* f) {
  if (!s || !b || !f) return LBM_ERR_INVALID;
  std::memset(f, 0, sizeof(double) * s->ndof);
  for (size_t e = 0; e < s->conn.size() / 9; ++e)
    for (int a = 0; a < 9; ++a) {
      double m = 0.0;
      for (int g = 0; g < 9; ++g) m += s->w[g] * s->N[g][a];
      for (int k = 0; k < 2; ++k) f[2 * s->conn[9 * e + a] + k] += s->rho * m * b[k];
    }
  return LBM_OK;
}

lbm_status lbm_fem_step(lbm_fem* s, const double* fext1, int* iterations) {
  if (!s || !fext1) return LBM_ERR_INVALID;
  const int n = s->ndof, bw = s->bw;
  const double th = s->theta, dt = s->dt;
  std::vector<double> u0 = s->u, v0 = s->v;
  // (1 - theta)(f_int(u0) - f_ext0), the old time level's share.
  std::vector<double> rhs0(n);
  s->fi.assign(n, 0.0);
  element_loop(s, u0.data(), s->fi.data(), nullptr, 0.0);
  for (int i = 0; i < n; ++i) rhs0[i] = (1.0 - th) * (s->fi[i] - s->fext[i]);
  std::vector<double> u(n), a(n), Ma(n);
  for (int i = 0; i < n; ++i) u[i] = s->fixed[i] ? 0.0 : u0[i] + dt * v0[i];
  int it = 0;
  bool ok = false;
  for (it = 1; it <= 30; ++it) {
    for (int i = 0; i < n; ++i) a[i] = (u[i] - u0[i]) / (th * dt * dt) - v0[i] / (th * dt);
    band_matvec(s, s->M, a.data(), Ma.data());
    s->K.assign(s->M.size(), 0.0);
    element_loop(s, u.data(), s->fi.data(), &s->K, th);
    s->R.resize(n);
    for (int i = 0; i < n; ++i) s->R[i] = Ma[i] + th * (s->fi[i] - fext1[i]) + rhs0[i];
    const double im = 1.0 / (th * dt * dt);
    for (size_t k = 0; k < s->K.size(); ++k) s->K[k] += im * s->M[k];
    // Clamped DOFs: identity rows and columns, zero residual.
    for (int i = 0; i < n; ++i) {
      if (!s->fixed[i]) continue;
      for (int j = std::max(0, i - bw); j <= std::min(n - 1, i + bw); ++j) {
        band(s->K, bw, i, j) = 0.0;
        band(s->K, bw, j, i) = 0.0;
      }
      band(s->K, bw, i, i) = 1.0;
      s->R[i] = 0.0;
    }
    s->du.resize(n);
    for (int i = 0; i < n; ++i) s->du[i] = -s->R[i];
    if (!band_solve(s->K, n, bw, s->du.data())) return LBM_ERR_NONFINITE;
    double dmax = 0.0, umax = 0.0;
    for (int i = 0; i < n; ++i) {
      u[i] += s->du[i];
      dmax = std::max(dmax, std::fabs(s->du[i]));
      umax = std::max(umax, std::fabs(u[i]));
    }
    if (!std::isfinite(dmax)) return LBM_ERR_NONFINITE;
    // Relative to the displacement, with a floor of 1e-14 of the thickness
    // for a beam that has not moved.
    if (dmax <= std::max(1e-10 * umax, 1e-14 * s->H)) {
      ok = true;
      break;
    }
  }
  if (iterations) *iterations = it;
  if (!ok) return LBM_ERR_NONFINITE;
  for (int i = 0; i < n; ++i) {
    s->v[i] = s->fixed[i] ? 0.0 : (u[i] - u0[i]) / (th * dt) - (1.0 - th) / th * v0[i];
    s->u[i] = u[i];
    s->fext[i] = fext1[i];
  }
  return LBM_OK;
}

lbm_status lbm_fem_get_state(const lbm_fem* s, double* u, double* v) {
  if (!s) return LBM_ERR_INVALID;
  if (u) std::memcpy(u, s->u.data(), sizeof(double) * s->ndof);
  if (v) std::memcpy(v, s->v.data(), sizeof(double) * s->ndof);
  return LBM_OK;
}

lbm_status lbm_fem_set_state(lbm_fem* s, const double* u, const double* v) {
  if (!s) return LBM_ERR_INVALID;
  if (u) std::memcpy(s->u.data(), u, sizeof(double) * s->ndof);
  if (v) std::memcpy(s->v.data(), v, sizeof(double) * s->ndof);
  return LBM_OK;
}

lbm_status lbm_fsi_create(lbm_ctx* ctx, int inst, lbm_fem* fem, const double* arc, int n_arc,
                          lbm_fsi** out) {
  if (!ctx || !fem || !out || n_arc < 0 || (n_arc > 0 && !arc)) return LBM_ERR_INVALID;
  *out = nullptr;
  lbm_fsi* f = new lbm_fsi;
  f->ctx = ctx;
  f->inst = inst;
  f->fem = fem;
  f->arc.assign(arc, arc + 2 * (size_t)n_arc);
  f->chain = wet_chain(fem);
  rebuild(f);
  const lbm_status st = set_surface(f);
  if (st != LBM_OK) {
    delete f;
    return st;
  }
  *out = f;
  return LBM_OK;
}

lbm_status lbm_fsi_destroy(lbm_fsi* f) {
  delete f;
  return LBM_OK;
}

lbm_status lbm_fsi_step(lbm_fsi* f, int n_steps, double* beam_force, double* tip) {
  if (!f || n_steps < 0) return LBM_ERR_INVALID;
  lbm_fem* s = f->fem;
  std::vector<double> fext(s->ndof);
  for (int step = 0; step < n_steps; ++step) {
    lbm_status st = lbm_step(f->ctx, 1);
    if (st) return st;
    const int nq = (int)f->wq.size();
    f->tq.assign(2 * (size_t)nq, 0.0);
    double F[3];
    st = lbm_wall_force_noalloc(f->ctx, f->inst, f->xq.data(), f->nq.data(), f->wq.data(), nq,
                                f->tq.data(), F);
    if (st) return st;
    // Gauge pressure: the reference pressure rho_0 c_s^2 (rho_0 = 1) is taken
    // out of the traction.  The beam is only partly wet (its clamped end is
    // not), so a uniform pressure does not cancel on it.
    F[0] = F[1] = F[2] = 0.0;
    for (int q = 0; q < nq; ++q)
      for (int a = 0; a < 2; ++a) {
        f->tq[2 * q + a] += f->nq[2 * q + a] / 3.0;
        F[a] += f->tq[2 * q + a] * f->wq[q];
      }
    std::fill(fext.begin(), fext.end(), 0.0);
    for (int q = 0; q < nq; ++q)
      for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
          fext[2 * f->qn[3 * q + k] + a] += f->shp[3 * q + k] * f->tq[2 * q + a] * f->wq[q];
    st = lbm_fem_step(s, fext.data(), nullptr);
    if (st) return st;
    rebuild(f);
    st = set_surface(f);
    if (st) return st;
    if (beam_force)
      for (int a = 0; a < 3; ++a) beam_force[3 * step + a] = F[a];
    if (tip) {
      const int k = s->ney + s->nyn * (s->nxn - 1);
      tip[2 * step] = s->u[2 * k];
      tip[2 * step + 1] = s->u[2 * k + 1];
    }
  }
  return LBM_OK;
}

}  // extern "C"
