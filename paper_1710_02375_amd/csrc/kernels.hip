// Device kernels of the KBC lattice Boltzmann step for gfx950.
//
//   bulk      fused pull-stream + KBC collide for every node without a special
//             flag: the hot kernel, one thread per node, SoA populations.
//   boundary  nodes on non-periodic faces and nodes with cut links: pull,
//             Grad's approximation for the missing populations, inflow /
//             outflow conditions, then the same collision.
//   geometry  prescribed body motion on the device (solid marks at the next
//             time, fresh-node refill, cut-link marks).
//   init / decode / encode / moments / force / reductions.
#include <math.h>

#include "kbc_node.hpp"
#include "kernels.hpp"

namespace kbc {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
struct Coord {
  int x, y, z;
};

__device__ __forceinline__ Coord node_coord(const InstDev& I, uint32_t node) {
  const uint32_t row = fdiv_u32(node, I.divx);
  const uint32_t z = fdiv_u32(row, I.divy);
  Coord c;
  c.x = (int)(node - row * (uint32_t)I.nx);
  c.y = (int)(row - z * (uint32_t)I.ny);
  c.z = (int)z;
  return c;
}

__device__ __forceinline__ uint32_t node_index(const InstDev& I, int x, int y, int z) {
  return (uint32_t)x + (uint32_t)I.nx * ((uint32_t)y + (uint32_t)I.ny * (uint32_t)z);
}

// Resolves the lattice site (x,y,z) + off for neighbour lookups: periodic
// faces wrap, any other face leaves the domain (returns false).
__device__ __forceinline__ bool resolve_nb(const InstDev& I, int x, int y, int z, int ox, int oy,
                                           int oz, uint32_t& out) {
  int s[3] = {x + ox, y + oy, z + oz};
  const int n[3] = {I.nx, I.ny, I.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (s[a] >= 0 && s[a] < n[a]) continue;
    if (I.face[2 * a + (s[a] < 0 ? 0 : 1)] != LBM_FACE_PERIODIC) return false;
    s[a] = (s[a] % n[a] + n[a]) % n[a];
  }
  out = node_index(I, s[0], s[1], s[2]);
  return true;
}

// ---------------------------------------------------------------------------
// Surface-mesh bodies (Sec. II.C.1): solid test from the column crossings,
// cut links by ray-face intersection over the face cells, velocities by
// linear (barycentric) interpolation of the vertex velocities.  FP64.
// ---------------------------------------------------------------------------
// Solid when the line of the node's column crosses the surface an odd
// number of times before x, or at x (surface points are solid).
__device__ bool mesh_parity(const InstDev& I, int x, int y, int z) {
  const int a = y - I.col_lo[0], b = z - I.col_lo[1];
  if (a < 0 || b < 0 || a >= I.col_n[0] || b >= I.col_n[1]) return false;
  const int k = a + I.col_n[0] * b;
  const double xd = (double)x;
  int below = 0;
  for (int j = I.col_start[k]; j < I.col_start[k + 1]; ++j) {
    const double xc = I.col_x[j];
    if (xc == xd) return true;
    if (xc < xd) ++below;
  }
  return (below & 1) != 0;
}

// Face cells meeting the box [lo, hi] (clamped to the grid): cell ranges.
__device__ __forceinline__ void mesh_cells(const InstDev& I, const double (&lo)[3],
                                           const double (&hi)[3], int (&c0)[3], int (&c1)[3]) {
  for (int a = 0; a < 3; ++a) {
    c0[a] = (int)floor((lo[a] - I.bin_lo[a]) / I.bin_h);
    c1[a] = (int)floor((hi[a] - I.bin_lo[a]) / I.bin_h);
    c0[a] = max(c0[a], 0);
    c1[a] = min(c1[a], I.bin_n[a] - 1);
  }
}

__device__ __forceinline__ void vel_at(const InstDev& I, int f, double l0, double l1, double l2,
                                       double (&v)[3]) {
  const int* fv = I.mesh_f + 3 * f;
  for (int a = 0; a < 3; ++a)
    v[a] = l0 * I.mesh_vel[3 * fv[0] + a] + l1 * I.mesh_vel[3 * fv[1] + a] +
           (I.D == 3 ? l2 * I.mesh_vel[3 * fv[2] + a] : 0.0);
}

// Closest point of face f to p: squared distance and barycentric weights.
// Triangles: the Voronoi region of p (a vertex, an edge or the interior)
// from the signs of the projections on the edges; segments: the clamped
// projection.
__device__ double mesh_closest(const InstDev& I, int f, const double (&p)[3], double (&l)[3]) {
  const int* fv = I.mesh_f + 3 * f;
  const double* A = I.mesh_v + 3 * fv[0];
  const double* B = I.mesh_v + 3 * fv[1];
  if (I.D == 2) {
    const double ex = B[0] - A[0], ey = B[1] - A[1];
    const double len2 = ex * ex + ey * ey;
    double s = len2 > 0.0 ? ((p[0] - A[0]) * ex + (p[1] - A[1]) * ey) / len2 : 0.0;
    s = fmin(fmax(s, 0.0), 1.0);
    const double dx = A[0] + s * ex - p[0], dy = A[1] + s * ey - p[1];
    l[0] = 1.0 - s;
    l[1] = s;
    l[2] = 0.0;
    return dx * dx + dy * dy;
  }
  const double* Cv = I.mesh_v + 3 * fv[2];
  double ab[3], ac[3], ap[3];
  for (int a = 0; a < 3; ++a) {
    ab[a] = B[a] - A[a];
    ac[a] = Cv[a] - A[a];
    ap[a] = p[a] - A[a];
  }
  auto dot = [](const double* u, const double* v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
  auto d2 = [&](double l0, double l1, double l2) {
    double r = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double q = l0 * A[a] + l1 * B[a] + l2 * Cv[a] - p[a];
      r += q * q;
    }
    return r;
  };
  const double d1 = dot(ab, ap), d2v = dot(ac, ap);
  if (d1 <= 0.0 && d2v <= 0.0) {   // vertex A
    l[0] = 1.0; l[1] = 0.0; l[2] = 0.0;
    return d2(1.0, 0.0, 0.0);
  }
  double bp[3], cp[3];
  for (int a = 0; a < 3; ++a) {
    bp[a] = p[a] - B[a];
    cp[a] = p[a] - Cv[a];
  }
  const double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) {   // vertex B
    l[0] = 0.0; l[1] = 1.0; l[2] = 0.0;
    return d2(0.0, 1.0, 0.0);
  }
  const double vc = d1 * d4 - d3 * d2v;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {   // edge AB
    const double v = d1 / (d1 - d3);
    l[0] = 1.0 - v; l[1] = v; l[2] = 0.0;
    return d2(l[0], l[1], 0.0);
  }
  const double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) {   // vertex C
    l[0] = 0.0; l[1] = 0.0; l[2] = 1.0;
    return d2(0.0, 0.0, 1.0);
  }
  const double vb = d5 * d2v - d1 * d6;
  if (vb <= 0.0 && d2v >= 0.0 && d6 <= 0.0) {   // edge AC
    const double w = d2v / (d2v - d6);
    l[0] = 1.0 - w; l[1] = 0.0; l[2] = w;
    return d2(l[0], 0.0, w);
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {   // edge BC
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    l[0] = 0.0; l[1] = 1.0 - w; l[2] = w;
    return d2(0.0, l[1], w);
  }
  const double den = 1.0 / (va + vb + vc);   // interior
  l[1] = vb * den;
  l[2] = vc * den;
  l[0] = 1.0 - l[1] - l[2];
  return d2(l[0], l[1], l[2]);
}

// Velocity at the closest surface point to p: faces of the cells within two
// spacings of p, all faces if none is there.
// Inside or on the surface.  The crossing count decides inside; a node the
// count leaves outside is on the surface if a face of its bin passes within
// 1e-12 of it (a face lying along the node's column, or the half-open tie
// rule at an edge, gives no crossing at the node itself).
__device__ bool mesh_inside(const InstDev& I, int x, int y, int z) {
  if (mesh_parity(I, x, y, z)) return true;
  const double p[3] = {(double)x, (double)y, (double)z};
  const double lo[3] = {p[0] - 1e-9, p[1] - 1e-9, p[2] - 1e-9};
  const double hi[3] = {p[0] + 1e-9, p[1] + 1e-9, p[2] + 1e-9};
  int c0[3], c1[3];
  mesh_cells(I, lo, hi, c0, c1);
  for (int kz = c0[2]; kz <= c1[2]; ++kz)
    for (int ky = c0[1]; ky <= c1[1]; ++ky)
      for (int kx = c0[0]; kx <= c1[0]; ++kx) {
        const int k = kx + I.bin_n[0] * (ky + I.bin_n[1] * kz);
        for (int j = I.bin_start[k]; j < I.bin_start[k + 1]; ++j) {
          double l[3];
          if (mesh_closest(I, I.bin_face[j], p, l) <= 1e-24) return true;
        }
      }
  return false;
}

__device__ void mesh_velocity(const InstDev& I, const double (&p)[3], double (&v)[3]) {
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = p[a] - 2.0;
    hi[a] = p[a] + 2.0;
  }
  int c0[3], c1[3];
  mesh_cells(I, lo, hi, c0, c1);
  double best = 1e300, bl[3] = {1.0, 0.0, 0.0};
  int bf = -1;
  for (int cz_ = c0[2]; cz_ <= c1[2]; ++cz_)
    for (int cy_ = c0[1]; cy_ <= c1[1]; ++cy_)
      for (int cx_ = c0[0]; cx_ <= c1[0]; ++cx_) {
        const int k = cx_ + I.bin_n[0] * (cy_ + I.bin_n[1] * cz_);
        for (int j = I.bin_start[k]; j < I.bin_start[k + 1]; ++j) {
          double l[3];
          const double r = mesh_closest(I, I.bin_face[j], p, l);
          if (r < best) {
            best = r;
            bf = I.bin_face[j];
            bl[0] = l[0]; bl[1] = l[1]; bl[2] = l[2];
          }
        }
      }
  if (bf < 0) {
    for (int f = 0; f < I.mesh_nf; ++f) {
      double l[3];
      const double r = mesh_closest(I, f, p, l);
      if (r < best) {
        best = r;
        bf = f;
        bl[0] = l[0]; bl[1] = l[1]; bl[2] = l[2];
      }
    }
  }
  v[0] = v[1] = v[2] = 0.0;
  if (bf >= 0) vel_at(I, bf, bl[0], bl[1], bl[2], v);
  if (I.D == 2) v[2] = 0.0;
}

// First surface point along the link from node p towards p - c: the
// smallest t in [0, 1] at which p - t c meets a face (triangles:
// Moller-Trumbore; segments: the 2x2 system), q = t, and the interpolated
// velocity there.  Without a hit (the solid test and the intersection
// disagree in the last bits) the wall is taken at the far node.
__device__ void mesh_cut(const InstDev& I, int x, int y, int z, int c0, int c1, int c2,
                         double& q, double (&uw)[3]) {
  const double p[3] = {(double)x, (double)y, (double)z};
  const double dir[3] = {-(double)c0, -(double)c1, -(double)c2};
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = fmin(p[a], p[a] + dir[a]) - 1e-9;
    hi[a] = fmax(p[a], p[a] + dir[a]) + 1e-9;
  }
  int cl[3], ch[3];
  mesh_cells(I, lo, hi, cl, ch);
  const double tol = 1e-12;
  double tbest = 2.0, bl[3] = {1.0, 0.0, 0.0};
  int bf = -1;
  for (int kz = cl[2]; kz <= ch[2]; ++kz)
    for (int ky = cl[1]; ky <= ch[1]; ++ky)
      for (int kx = cl[0]; kx <= ch[0]; ++kx) {
        const int k = kx + I.bin_n[0] * (ky + I.bin_n[1] * kz);
        for (int j = I.bin_start[k]; j < I.bin_start[k + 1]; ++j) {
          const int f = I.bin_face[j];
          const int* fv = I.mesh_f + 3 * f;
          const double* A = I.mesh_v + 3 * fv[0];
          const double* B = I.mesh_v + 3 * fv[1];
          double t, l1, l2;
          if (I.D == 3) {
            const double* Cv = I.mesh_v + 3 * fv[2];
            const double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
            const double e2[3] = {Cv[0] - A[0], Cv[1] - A[1], Cv[2] - A[2]};
            const double pv[3] = {dir[1] * e2[2] - dir[2] * e2[1], dir[2] * e2[0] - dir[0] * e2[2],
                                  dir[0] * e2[1] - dir[1] * e2[0]};
            const double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
            if (fabs(det) < 1e-300) continue;
            const double id = 1.0 / det;
            const double tv[3] = {p[0] - A[0], p[1] - A[1], p[2] - A[2]};
            l1 = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * id;
            if (l1 < -tol || l1 > 1.0 + tol) continue;
            const double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2],
                                  tv[0] * e1[1] - tv[1] * e1[0]};
            l2 = (dir[0] * qv[0] + dir[1] * qv[1] + dir[2] * qv[2]) * id;
            if (l2 < -tol || l1 + l2 > 1.0 + tol) continue;
            t = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * id;
          } else {
            // p + t dir = A + s (B - A): Cramer's rule on the 2x2 system.
            const double ex = B[0] - A[0], ey = B[1] - A[1];
            const double det = ex * dir[1] - ey * dir[0];
            if (fabs(det) < 1e-300) continue;
            const double rx = p[0] - A[0], ry = p[1] - A[1];
            const double sg = (rx * dir[1] - ry * dir[0]) / det;
            if (sg < -tol || sg > 1.0 + tol) continue;
            t = (rx * ey - ry * ex) / det;
            l1 = sg;
            l2 = 0.0;
          }
          if (t < -1e-9 || t > 1.0 + 1e-9) continue;
          if (t < tbest) {
            tbest = t;
            bf = f;
            bl[0] = 1.0 - l1 - l2;
            bl[1] = l1;
            bl[2] = l2;
          }
        }
      }
  if (bf >= 0) {
    q = fmin(fmax(tbest, 1e-12), 1.0);
    for (int a = 0; a < 3; ++a) bl[a] = fmin(fmax(bl[a], 0.0), 1.0);
    vel_at(I, bf, bl[0], bl[1], bl[2], uw);
    if (I.D == 2) uw[2] = 0.0;
  } else {
    q = 1.0;
    const double pf[3] = {p[0] + dir[0], p[1] + dir[1], p[2] + dir[2]};
    mesh_velocity(I, pf, uw);
  }
}

// ---------------------------------------------------------------------------
// Prescribed-motion bodies (FP64).  Time t is the step count.
// ---------------------------------------------------------------------------
// Analytic bodies (sphere, flap, plates) at an arbitrary point.
__device__ bool analytic_inside(const InstDev& I, double x, double y, double z, double t) {
  const double* p = I.body;
  switch (I.body_kind) {
    case LBM_BODY_SPHERE: {
      const double s = sin(p[7] * t + p[8]);
      const double dx = x - (p[0] + p[4] * s);
      const double dy = y - (p[1] + p[5] * s);
      double r2 = dx * dx + dy * dy;
      if (I.D == 3) {
        const double dz = z - (p[2] + p[6] * s);
        r2 += dz * dz;
      }
      return r2 <= p[3] * p[3];
    }
    case LBM_BODY_FLAP: {
      const double sl = y - p[6];
      if (sl < 0.0 || sl > p[1]) return false;
      const double xc = p[0] + p[3] * sin(p[4] * t + p[5]) * (sl / p[1]) * (sl / p[1]);
      return fabs(x - xc) <= 0.5 * p[2];
    }
    case LBM_BODY_PLATES:
      return y < p[0] || y > p[1];
    default:
      return false;
  }
}

// Solid test of a lattice node (meshes by crossings and surface distance).
__device__ bool body_inside(const InstDev& I, double x, double y, double z, double t) {
  if (I.body_kind == LBM_BODY_MESH) return mesh_inside(I, (int)x, (int)y, (int)z);
  return analytic_inside(I, x, y, z, t);
}

__device__ void body_velocity(const InstDev& I, double x, double y, double z, double t,
                              double (&v)[3]) {
  const double* p = I.body;
  v[0] = v[1] = v[2] = 0.0;
  switch (I.body_kind) {
    case LBM_BODY_SPHERE: {
      const double c = cos(p[7] * t + p[8]);
      for (int a = 0; a < I.D; ++a) v[a] = p[4 + a] * p[7] * c;
      break;
    }
    case LBM_BODY_FLAP: {
      double sl = y - p[6];
      sl = fmin(fmax(sl, 0.0), p[1]);
      v[0] = p[3] * p[4] * cos(p[4] * t + p[5]) * (sl / p[1]) * (sl / p[1]);
      break;
    }
    case LBM_BODY_MESH: {
      const double pt[3] = {x, y, z};
      mesh_velocity(I, pt, v);
      break;
    }
    case LBM_BODY_PLATES: {
      const double* u = (y < 0.5 * (p[0] + p[1])) ? &p[2] : &p[5];
      for (int a = 0; a < I.D; ++a) v[a] = u[a];
      break;
    }
    default:
      break;
  }
}

// Wall fraction q in (0,1] of the link from fluid node x towards x - c, whose
// far end is inside the body, and the body velocity at the wall point.
// Sphere: smaller root of |x - lambda c - X_c|^2 = R^2; other bodies:
// bisection to the first inside point.
__device__ void body_cut(const InstDev& I, int x, int y, int z, int c0, int c1, int c2, double t,
                         double& q, double (&uw)[3]) {
  if (I.body_kind == LBM_BODY_MESH) {
    mesh_cut(I, x, y, z, c0, c1, c2, q, uw);
    return;
  }
  if (I.body_kind == LBM_BODY_SPHERE) {
    const double* p = I.body;
    const double s = sin(p[7] * t + p[8]);
    const double d0 = x - (p[0] + p[4] * s), d1 = y - (p[1] + p[5] * s);
    const double d2 = (I.D == 3) ? z - (p[2] + p[6] * s) : 0.0;
    const double cc = (double)(c0 * c0 + c1 * c1 + c2 * c2);
    const double dc = d0 * c0 + d1 * c1 + d2 * c2;
    const double dd = d0 * d0 + d1 * d1 + d2 * d2 - p[3] * p[3];
    const double disc = fmax(dc * dc - cc * dd, 0.0);
    q = (dc - sqrt(disc)) / cc;
    q = fmin(fmax(q, 0.0), 1.0);
  } else {
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (analytic_inside(I, x - mid * c0, y - mid * c1, z - mid * c2, t)) hi = mid; else lo = mid;
    }
    q = hi;
  }
  body_velocity(I, x - q * c0, y - q * c1, z - q * c2, t, uw);
}

__device__ void inflow_velocity(const InstDev& I, int y, int z, double t, double (&u)[3]) {
  double prof = 1.0;
  if (I.inlet_profile == 1) {
    const double yp = y + 0.5, H = I.ny;
    prof = 1.5 * yp * (H - yp) / (0.25 * H * H);
    if (I.D == 3) {
      const double zp = z + 0.5, Z = I.nz;
      prof *= 1.5 * zp * (Z - zp) / (0.25 * Z * Z);
    }
  }
  double r = 1.0;
  if (I.ramp_steps > 0) {
    const double tt = fmin(t, (double)I.ramp_steps);
    r = 0.5 * (1.0 - cos(M_PI * tt / I.ramp_steps));
  }
  for (int a = 0; a < 3; ++a) u[a] = I.u_in[a] * prof * r;
}

// ---------------------------------------------------------------------------
// Lagged moments (post-collision state stored at the node itself), in the
// arithmetic type R.
// ---------------------------------------------------------------------------
template <int Q, int ST, typename R>
__device__ __forceinline__ void lagged(const typename Store<ST>::T* sb, int64_t stride, uint32_t m,
                                       R& rt, R (&u)[3]) {
  R d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = (R)Store<ST>::dec(sb[i * stride + m]);
  R j[3];
  moments_dev<Q>(d, rt, j);
  const R ir = R(1) / (R(1) + rt);
  for (int a = 0; a < 3; ++a) u[a] = j[a] * ir;
}

// ---------------------------------------------------------------------------
// Pre-collision state of one node (any node: bulk, face or cut links) in
// the arithmetic type R: pull streaming f_i(x) = A_i(x - c_i) (Eq. 1),
// missing populations from Grad's approximation (Sec. II.C.1), inflow /
// outflow equilibria.
//   sb   : instance base of the state being streamed (post-collision at t-1)
//   t1   : time of the new state (geometry and inflow ramp)
// Returns the deviations f_i - W_i.  Each neighbour's lagged moments are
// read only where the chosen interpolation or difference uses them.
// WALLONLY: every missing population of the node comes from a wall face
// (q = 1/2, wall at rest), so the body cut-link code is not compiled in.
// MPFILL: compile in the multiphase scaling of the filled populations
// (applied to multiphase instances only).
// ---------------------------------------------------------------------------
template <int Q, int ST, typename R, bool WALLONLY = false, bool MPFILL = false>
__device__ void gather_pre(const InstDev& I, const typename Store<ST>::T* sb, const uint8_t* fl,
                           int x, int y, int z, double t1, R (&f)[Q]) {
  using S = Store<ST>;
  constexpr int D = dims<Q>();
  const int64_t stride = I.stride;
  const int n[3] = {I.nx, I.ny, I.nz};
  uint32_t miss = 0, wallm = 0;
  bool inlet = false, outlet = false;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int s[3] = {x - cx(i), y - cy(i), z - cz<Q>(i)};
    bool w = false, in = false, out = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (s[a] >= 0 && s[a] < n[a]) continue;
      const int fc = I.face[2 * a + (s[a] < 0 ? 0 : 1)];
      if (fc == LBM_FACE_PERIODIC) s[a] = (s[a] + n[a]) % n[a];
      else if (fc == LBM_FACE_WALL) w = true;
      else if (fc == LBM_FACE_INLET) in = true;
      else out = true;
    }
    f[i] = R(0);
    if (w) {
      miss |= 1u << i;
      wallm |= 1u << i;
    } else if (in) {
      inlet = true;
    } else if (out) {
      outlet = true;
    } else {
      const uint32_t m = node_index(I, s[0], s[1], s[2]);
      if (fl && (fl[m] & FLAG_SOLID)) miss |= 1u << i;
      else f[i] = (R)S::dec(sb[i * stride + m]);
    }
  }
  if (inlet) {
    // Equilibrium at the inflow velocity and the lagged density of x + e_x.
    double ud[3];
    inflow_velocity(I, y, z, t1, ud);
    R rt = R(0), uu[3];
    uint32_t m;
    if (resolve_nb(I, x, y, z, 1, 0, 0, m) && !(fl && (fl[m] & FLAG_SOLID)))
      lagged<Q, ST, R>(sb, stride, m, rt, uu);
    const R ui[3] = {(R)ud[0], (R)ud[1], (R)ud[2]};
    feq_dev<Q, R>(rt, ui, f);
    return;
  }
  if (outlet) {
    // Equilibrium at density 1 and the lagged velocity of x - e_x.
    R rt = R(0), uo[3] = {R(0), R(0), R(0)};
    uint32_t m;
    if (resolve_nb(I, x, y, z, -1, 0, 0, m) && !(fl && (fl[m] & FLAG_SOLID)))
      lagged<Q, ST, R>(sb, stride, m, rt, uo);
    feq_dev<Q, R>(R(0), uo, f);
    return;
  }
  if (!miss) return;

  // ---- Grad's approximation for the missing populations ----------------
  const double tq = t1;
  auto link = [&](int i, R& q, R (&uw)[3]) {
    if (WALLONLY || ((wallm >> i) & 1u)) {
      q = R(0.5);
      uw[0] = uw[1] = uw[2] = R(0);
    } else {
      double qd, ud[3];
      body_cut(I, x, y, z, cx(i), cy(i), cz<Q>(i), tq, qd, ud);
      q = (R)qd;
      for (int a = 0; a < 3; ++a) uw[a] = (R)ud[a];
    }
  };
  auto fluid_at = [&](int ox, int oy, int oz, uint32_t& m) -> bool {
    if (!resolve_nb(I, x, y, z, ox, oy, oz, m)) return false;
    return !(fl && (fl[m] & FLAG_SOLID));
  };
  const uint32_t me = node_index(I, x, y, z);
  R rt_x, u_x[3];
  lagged<Q, ST, R>(sb, stride, me, rt_x, u_x);
  const R rho_n = R(1) + rt_x;

  // Target density: bounce-back-implied density plus the wall-motion term.
  R rtt = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (!((miss >> i) & 1u)) {
      rtt += f[i];
    } else {
      R q, uw[3];
      link(i, q, uw);
      const R cu = R(cx(i)) * uw[0] + R(cy(i)) * uw[1] + R(cz<Q>(i)) * uw[2];
      rtt += (R)S::dec(sb[(Q - 1 - i) * stride + me]) + R(6.0 * weight<Q>(i)) * rho_n * cu;
    }
  }
  const R rho_t = R(1) + rtt;

  // Target velocity: interpolation along each missing link through the wall
  // point (s = -q) and the lagged velocities at x + c_i (s = 1), x + 2 c_i
  // (s = 2), averaged over the missing links.
  R ut[3] = {R(0), R(0), R(0)};
  int nm = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (!((miss >> i) & 1u)) continue;
    R q, uw[3];
    link(i, q, uw);
    uint32_t m1, m2;
    R ui[3];
    if (fluid_at(cx(i), cy(i), cz<Q>(i), m1)) {
      R r1, u1[3];
      lagged<Q, ST, R>(sb, stride, m1, r1, u1);
      if (fluid_at(2 * cx(i), 2 * cy(i), 2 * cz<Q>(i), m2)) {
        R r2, u2[3];
        lagged<Q, ST, R>(sb, stride, m2, r2, u2);
        const R a0 = R(2) / ((R(1) + q) * (R(2) + q));
        const R a1 = R(2) * q / (R(1) + q);
        const R a2 = -q / (R(2) + q);
        for (int a = 0; a < 3; ++a) ui[a] = a0 * uw[a] + a1 * u1[a] + a2 * u2[a];
      } else {
        for (int a = 0; a < 3; ++a) ui[a] = (uw[a] + q * u1[a]) / (R(1) + q);
      }
    } else {
      for (int a = 0; a < 3; ++a) ui[a] = uw[a];
    }
    for (int a = 0; a < 3; ++a) ut[a] += ui[a];
    ++nm;
  }
  for (int a = 0; a < 3; ++a) ut[a] /= R(nm);

  // Velocity gradient G[a][b] = d u_a / d x_b: central differences of the
  // lagged velocity, the wall point on a cut side (quadratic through the wall
  // point, x + e, x + 2e; linear if x + 2e is not fluid).  Only the lagged
  // velocities the chosen difference uses are read.
  R G[3][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const int ip = axis_pop<Q>(b, +1);   // link to x - e_b
    const int im = axis_pop<Q>(b, -1);   // link to x + e_b
    const bool cut_m = (miss >> ip) & 1u;
    const bool cut_p = (miss >> im) & 1u;
    const int eb[3] = {b == 0, b == 1, b == 2};
    uint32_t p1, p2, m1, m2;
    const bool fp1 = fluid_at(eb[0], eb[1], eb[2], p1);
    const bool fp2 = fp1 && fluid_at(2 * eb[0], 2 * eb[1], 2 * eb[2], p2);
    const bool fm1 = fluid_at(-eb[0], -eb[1], -eb[2], m1);
    const bool fm2 = fm1 && fluid_at(-2 * eb[0], -2 * eb[1], -2 * eb[2], m2);
    R v1[3] = {R(0), R(0), R(0)}, v2[3] = {R(0), R(0), R(0)}, rr;
    R qq = R(0), w[3] = {R(0), R(0), R(0)};
    int form = 0;   // 0 none, 1 both cut, 2/3 quadratic/linear through the lower
                    // wall, 4/5 through the upper wall, 6 central, 7/8 one-sided
    if (cut_m && cut_p) {
      R qm, wm[3], qp, wp[3];
      link(ip, qm, wm);
      link(im, qp, wp);
      for (int a = 0; a < D; ++a) G[a][b] = (wp[a] - wm[a]) / (qp + qm);
      continue;
    } else if (cut_m) {
      link(ip, qq, w);
      if (fp2) {
        lagged<Q, ST, R>(sb, stride, p1, rr, v1);
        lagged<Q, ST, R>(sb, stride, p2, rr, v2);
        form = 2;
      } else if (fp1) {
        lagged<Q, ST, R>(sb, stride, p1, rr, v1);
        form = 3;
      }
    } else if (cut_p) {
      link(im, qq, w);
      if (fm2) {
        lagged<Q, ST, R>(sb, stride, m1, rr, v1);
        lagged<Q, ST, R>(sb, stride, m2, rr, v2);
        form = 4;
      } else if (fm1) {
        lagged<Q, ST, R>(sb, stride, m1, rr, v1);
        form = 5;
      }
    } else if (fp1 && fm1) {
      lagged<Q, ST, R>(sb, stride, p1, rr, v1);
      lagged<Q, ST, R>(sb, stride, m1, rr, v2);
      form = 6;
    } else if (fp1) {
      lagged<Q, ST, R>(sb, stride, p1, rr, v1);
      form = 7;
    } else if (fm1) {
      lagged<Q, ST, R>(sb, stride, m1, rr, v1);
      form = 8;
    }
    for (int a = 0; a < D; ++a) {
      R g = R(0);
      switch (form) {
        case 2:
          g = R(-3) * w[a] / ((R(1) + qq) * (R(2) + qq)) + v1[a] * (R(2) - qq) / (R(1) + qq) +
              v2[a] * (qq - R(1)) / (R(2) + qq);
          break;
        case 3: g = (v1[a] - w[a]) / (R(1) + qq); break;
        case 4:
          g = R(3) * w[a] / ((R(1) + qq) * (R(2) + qq)) - v1[a] * (R(2) - qq) / (R(1) + qq) -
              v2[a] * (qq - R(1)) / (R(2) + qq);
          break;
        case 5: g = (w[a] - v1[a]) / (R(1) + qq); break;
        case 6: g = R(0.5) * (v1[a] - v2[a]); break;
        case 7: g = v1[a] - u_x[a]; break;
        case 8: g = u_x[a] - v1[a]; break;
        default: break;
      }
      G[a][b] = g;
    }
  }
  // Pi = rho/3 I + rho u u - rho/(6 beta) (G + G^T)   (Pi^eq + Pi^neq, cs^2 = 1/3)
  const R kneq = rho_t / (R(6) * (R)I.beta);
  R Pi[6];
  Pi[0] = rho_t / R(3) + rho_t * ut[0] * ut[0] - kneq * R(2) * G[0][0];
  Pi[1] = rho_t / R(3) + rho_t * ut[1] * ut[1] - kneq * R(2) * G[1][1];
  Pi[2] = rho_t / R(3) + rho_t * ut[2] * ut[2] - kneq * R(2) * G[2][2];
  Pi[3] = rho_t * ut[0] * ut[1] - kneq * (G[0][1] + G[1][0]);
  Pi[4] = rho_t * ut[0] * ut[2] - kneq * (G[0][2] + G[2][0]);
  Pi[5] = rho_t * ut[1] * ut[2] - kneq * (G[1][2] + G[2][1]);
#pragma unroll
  for (int i = 0; i < Q; ++i)
    if ((miss >> i) & 1u) f[i] = grad_dev<Q, R>(i, rho_t, ut, Pi);
  if (MPFILL && I.mp) {
    // Multiphase: the filled populations carry the mass that bounce-back
    // would return, rho_t less the known populations (scaled as full f).
    R sk = R(0), sm = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if ((miss >> i) & 1u) sm += f[i] + R(weight<Q>(i));
      else sk += f[i] + R(weight<Q>(i));
    }
    if (sm > R(0)) {
      const R lam = (rho_t - sk) / sm;
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if ((miss >> i) & 1u) f[i] = lam * (f[i] + R(weight<Q>(i))) - R(weight<Q>(i));
    }
  }
}

// ---------------------------------------------------------------------------
// Statistics reduction within a workgroup (wave64 shuffles + LDS).
// ---------------------------------------------------------------------------
template <int BLOCK>
__device__ void block_stats(float gmin, float gmax, double gsum, uint32_t cnt, uint32_t f64,
                            StatPartial* out) {
  for (int off = 32; off > 0; off >>= 1) {
    gmin = fminf(gmin, __shfl_xor(gmin, off));
    gmax = fmaxf(gmax, __shfl_xor(gmax, off));
    gsum += __shfl_xor(gsum, off);
    cnt += __shfl_xor(cnt, off);
    f64 += __shfl_xor(f64, off);
  }
  constexpr int NW = BLOCK / 64;
  __shared__ StatPartial sh[NW > 0 ? NW : 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = StatPartial{gmin, gmax, gsum, cnt, f64};
  __syncthreads();
  if (threadIdx.x == 0) {
    StatPartial r = sh[0];
    for (int k = 1; k < NW; ++k) {
      r.gmin = fminf(r.gmin, sh[k].gmin);
      r.gmax = fmaxf(r.gmax, sh[k].gmax);
      r.gsum += sh[k].gsum;
      r.count += sh[k].count;
      r.fp64 += sh[k].fp64;
    }
    *out = r;
  }
}

// ---------------------------------------------------------------------------
// Inflow / outflow plane node, computed inside the bulk kernel in its
// arithmetic type R (Sec. III.A.1 inflow with its smooth ramp): every
// population is the entropic equilibrium at the inflow velocity and the
// lagged density of x + e_x, or at density 1 and the lagged velocity of
// x - e_x, all in R (the inflow profile and ramp too).  Its density and
// momentum are exactly those of the state, so
// Delta = 0 and the collision (KBC or LBGK) is the identity (gamma = 2 by the
// <Dh|Dh> = 0 rule): the kernel stores it without colliding.  Takes the
// stored populations of that neighbour on entry (f; the bulk kernel pulls
// them in place of the node's own sources), nb_fluid whether it is fluid;
// ramp is the inflow ramp factor at the new time.  f receives the state
// (deviations).
// Returns false if the state is not valid (rho <= 0 or |u_a| >= 1).
// ---------------------------------------------------------------------------
template <int Q, typename R>
__device__ __forceinline__ bool face_state(const InstDev& I, int y, int z, bool inlet,
                                           bool nb_fluid, R ramp, R (&f)[Q]) {
  R rt = R(0), u[3] = {R(0), R(0), R(0)};
  if (nb_fluid) {
    R r, j[3];
    moments_dev<Q>(f, r, j);
    if (inlet) {
      rt = r;
    } else {
      const R ir = R(1) / (R(1) + r);
      u[0] = j[0] * ir;
      u[1] = j[1] * ir;
      u[2] = j[2] * ir;
    }
  }
  if (inlet) {
    // Parabolic profile 1.5 U y(H - y)/(H/2)^2 (per axis), times the ramp.
    R prof = ramp;
    if (I.inlet_profile == 1) {
      const R yp = R(y) + R(0.5), H = R(I.ny);
      prof *= R(6) * yp * (H - yp) / (H * H);
      if (I.D == 3) {
        const R zp = R(z) + R(0.5), Z = R(I.nz);
        prof *= R(6) * zp * (Z - zp) / (Z * Z);
      }
    }
    for (int a = 0; a < 3; ++a) u[a] = R(I.u_in[a]) * prof;
  }
  const bool ok = R(1) + rt > R(0) && u[0] < R(1) && u[0] > R(-1) && u[1] < R(1) &&
                  u[1] > R(-1) && u[2] < R(1) && u[2] > R(-1);
  feq_dev<Q, R>(rt, u, f);
  return ok;
}

// ---------------------------------------------------------------------------
// Bulk kernel: fused pull-stream + collide, one thread per node.
// ---------------------------------------------------------------------------
// MEM bit 0: non-temporal stores; bit 1: non-temporal loads; bit 2: 32-bit
// byte offsets from one base per instance (every instance's Q population
// arrays span less than 4 GiB), which removes the 64-bit address arithmetic
// and the per-population base registers; bit 3 (with bit 2): buffer loads and
// stores through one resource per instance and buffer, the population offset
// i * stride in the scalar offset, so that a load or store needs no vector
// address arithmetic beyond the node's own offset.
// AUX: cache policy bits of the instruction (2 = non-temporal).
template <typename T, int AUX>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 2)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, AUX));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}

template <typename T, int AUX>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                          uint32_t soff) {
  if constexpr (sizeof(T) == 2)
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, voff, soff, AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, AUX);
}

// Buffer resource word 3 for gfx9-family targets (raw, untyped 32-bit data).
constexpr int kBufferWord3 = 0x00020000;

template <int Q, int ST, int BLOCK, int WAVES, int MEM, bool STATS, bool FACES>
__global__ void __launch_bounds__(BLOCK, WAVES)
    k_bulk(StepBuffers b, const Tile* __restrict__ tiles, int tile0) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  const int ti = tile0 + blockIdx.x;
  const Tile tl = tiles[ti];
  // Local copy: read once, not re-read after every store (the compiler cannot
  // prove the descriptor does not alias the populations).
  const InstDev I = b.insts[tl.inst];
  const int nx = I.nx, ny = I.ny, nz = I.nz;
  // Node offsets of one step along y and z, and of the periodic wrap
  // (n - 1 steps) along each axis.
  const uint32_t sy = (uint32_t)nx, sz = (uint32_t)nx * (uint32_t)ny;
  const uint32_t wx = (uint32_t)(nx - 1), wy = (uint32_t)(ny - 1) * sy,
                 wz = (uint32_t)(nz - 1) * sz;
  const int64_t stride = I.stride;
  const T* __restrict__ sb = static_cast<const T*>(b.src) + I.pop_off;
  T* __restrict__ db = static_cast<T*>(b.dst) + I.pop_off;
  const uint8_t* fl = I.flag_off >= 0 ? b.flags + I.flag_off : nullptr;
  const uint32_t fmask = fl ? uint32_t(FLAG_SPECIAL) : 0u;
  CollideParams<R> P;
  P.beta = (R)I.beta;
  P.inv_beta = (R)(1.0 / I.beta);
  P.beta_d = I.beta;
  P.lbgk = I.collision;
  P.trace_in_s = I.trace_in_s;
  P.near_eq = I.near_eq;
  float gmin = 1e30f, gmax = -1e30f;
  double gsum = 0.0;
  uint32_t cnt = 0, f64 = 0;
  // FACES: inflow ramp factor at the new time, formed once per thread.
  R ramp = R(1);
  if constexpr (FACES) {
    if (I.face[0] == LBM_FACE_INLET && I.ramp_steps > 0) {
      const double tt = fmin((double)(*b.clock + 1), (double)I.ramp_steps);
      ramp = (R)(0.5 * (1.0 - cos(M_PI * tt / I.ramp_steps)));
    }
  }
  // NPI nodes per thread and iteration (lanes on consecutive nodes, the
  // second node BLOCK further on): all their pulls are issued before any is
  // used.  D2Q9 moves only 9 values per node, so one node per wave in flight
  // keeps too little memory traffic outstanding; D3Q27 keeps one.
  constexpr int NPI = Q == 9 ? 2 : 1;
  constexpr bool BUF = (MEM & 8) && sizeof(T) <= 4;
  constexpr uint32_t es = sizeof(T);
  const uint32_t pbytes = (uint32_t)stride * es;
  for (int k0 = threadIdx.x; k0 < tl.count; k0 += BLOCK * NPI) {
    T raw[NPI][Q];
    uint32_t fw[NPI], node[NPI];
    bool valid[NPI], face[NPI], inl[NPI];
    uint32_t fdir[NPI];
    int cy_[NPI], cz_[NPI];
#pragma unroll
    for (int n = 0; n < NPI; ++n) {
      const int k = k0 + n * BLOCK;
      valid[n] = k < tl.count;
      // A lane without a second node loads the first node's sources again.
      node[n] = (uint32_t)(tl.node0 + (valid[n] ? k : k0));
      // The flag is loaded with the pulls and tested after them, so that it
      // adds no memory latency of its own; the pulls of a special node wrap
      // periodically like any other and stay inside the instance.  The load
      // is the aligned 32-bit word holding the node's flag byte (flag slices
      // are padded to 256 bytes); without flags it reads the pool's first
      // word and the mask is zero, so there is no branch before the pulls.
      fw[n] = *reinterpret_cast<const uint32_t*>(fl ? fl + (node[n] & ~3u) : b.flags);
      const Coord c = node_coord(I, node[n]);
      cy_[n] = c.y;
      cz_[n] = c.z;
      // Source of population i is node - c_i, wrapped periodically: per axis
      // the node offset of the neighbour at -1 (dm) and +1 (dp), modulo 2^32,
      // chosen between two per-instance constants (no per-node products).
      const uint32_t dm[3] = {c.x == 0 ? wx : 0u - 1u, c.y == 0 ? wy : 0u - sy,
                              c.z == 0 ? wz : 0u - sz};
      const uint32_t dp[3] = {c.x == nx - 1 ? 0u - wx : 1u, c.y == ny - 1 ? 0u - wy : sy,
                              c.z == nz - 1 ? 0u - wz : sz};
      // Node offset of the source of (cx, cy, cz): the -c part of each axis.
      auto dof = [&](int a, int ci) -> uint32_t { return ci == 0 ? 0u : (ci > 0 ? dm[a] : dp[a]); };
      // FACES: an inflow (outflow) plane node pulls every population of
      // x + e_x (x - e_x) instead, from which it forms its face equilibrium.
      face[n] = false;
      inl[n] = false;
      fdir[n] = 0u;
      if constexpr (FACES) {
        inl[n] = I.face[0] == LBM_FACE_INLET && c.x == 0;
        face[n] = inl[n] || (I.face[1] == LBM_FACE_OUTLET && c.x == nx - 1);
        fdir[n] = inl[n] ? 1u : 0u - 1u;
      }
      if constexpr (BUF || (MEM & 4)) {
        // Byte offsets within the instance's populations: the (cy, cz) part
        // is formed once per pair, then each x neighbour adds its own.
        const uint32_t base = node[n] * es;
        uint32_t yz[3][3];
#pragma unroll
        for (int jy = -1; jy <= 1; ++jy)
#pragma unroll
          for (int jz = -1; jz <= 1; ++jz)
            yz[jy + 1][jz + 1] =
                face[n] ? base : base + (dof(1, jy) + (Q == 27 ? dof(2, jz) : 0u)) * es;
        const uint32_t xf = fdir[n] * es;
        const uint32_t xb[3] = {face[n] ? xf : dp[0] * es, face[n] ? xf : 0u,
                                face[n] ? xf : dm[0] * es};   // by cx + 1
        if constexpr (BUF) {
          // Node part in the vector offset, population part (i * stride) in
          // the scalar offset.
          const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
              const_cast<T*>(sb), (short)0, (int)(uint32_t)(Q * pbytes), kBufferWord3);
#pragma unroll
          for (int i = 0; i < Q; ++i)
            raw[n][i] = buf_load<T, (MEM & 2) ? 2 : 0>(
                rs, yz[cy(i) + 1][cz<Q>(i) + 1] + xb[cx(i) + 1], (uint32_t)i * pbytes);
        } else {
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const uint32_t off =
                (uint32_t)i * pbytes + yz[cy(i) + 1][cz<Q>(i) + 1] + xb[cx(i) + 1];
            const T* p = reinterpret_cast<const T*>(reinterpret_cast<const char*>(sb) + off);
            raw[n][i] = (MEM & 2) ? __builtin_nontemporal_load(p) : *p;
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const uint32_t src =
              face[n] ? node[n] + fdir[n]
                      : node[n] + dof(0, cx(i)) + dof(1, cy(i)) + (Q == 27 ? dof(2, cz<Q>(i)) : 0u);
          const T* p = sb + (i * stride + src);
          raw[n][i] = (MEM & 2) ? __builtin_nontemporal_load(p) : *p;
        }
      }
    }
    // All pulls are issued before the first use: without this fence the
    // scheduler consumes each value right after its load and a wave keeps a
    // single load in flight.
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int n = 0; n < NPI; ++n) {
      // An empty statement that the compiler must assume changes fw: the
      // test cannot be moved above it, to right after the flag load.
      asm volatile("" : "+v"(fw[n]));
      const uint32_t fshift = (node[n] & 3u) * 8u;
      if (!valid[n] || ((fw[n] >> fshift) & (face[n] ? uint32_t(FLAG_SOLID) : fmask))) continue;
      R f[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = S::dec(raw[n][i]);
      CollideOut co;
      bool ok;
      if (FACES && face[n]) {
        ok = face_state<Q, R>(I, cy_[n], cz_[n], inl[n], !(fl[node[n] + fdir[n]] & FLAG_SOLID),
                              ramp, f);
        co.gamma = 2.0f;
        co.fp64 = 0;
      } else {
        ok = collide<Q, R, true>(f, P, co);
      }
      if (!ok) atomicOr(b.err, 1u);
      if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
            db, (short)0, (int)(uint32_t)(Q * pbytes), kBufferWord3);
#pragma unroll
        for (int i = 0; i < Q; ++i)
          buf_store<T, (MEM & 1) ? 2 : 0>(S::enc(f[i]), rd, node[n] * es, (uint32_t)i * pbytes);
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          T* p = (MEM & 4) ? reinterpret_cast<T*>(reinterpret_cast<char*>(db) +
                                                    ((uint32_t)i * (uint32_t)stride + node[n]) *
                                                        (uint32_t)sizeof(T))
                           : db + (i * stride + node[n]);
          if (MEM & 1) __builtin_nontemporal_store(S::enc(f[i]), p); else *p = S::enc(f[i]);
        }
      }
      // Near-equilibrium nodes for the FP64 pass: each wave's 64 consecutive
      // nodes have a mask word of their own, zero unless some node of theirs
      // is deferred (the FP64 pass clears the words it finds set); the
      // lowest deferred lane stores it with a plain store (a shared counter
      // would take one same-address atomic per wave, which serialises when
      // such nodes are spread over the domain).  Skipped lanes defer nothing.
      const uint64_t m = __ballot(co.fp64 != 0);
      if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        if ((int)(threadIdx.x & 63) == leader)
          b.neq_words[(size_t)ti * b.neq_wpt + ((((uint32_t)k0 & ~63u) + (uint32_t)(n * BLOCK)) >> 6)] = m;
      }
      if (STATS && !co.fp64) {
        gmin = fminf(gmin, co.gamma);
        gmax = fmaxf(gmax, co.gamma);
        gsum += co.gamma;
        cnt += 1;
      }
    }
  }
  if (STATS) block_stats<BLOCK>(gmin, gmax, gsum, cnt, f64, b.stats + ti);
}

// Multiphase field helpers (Sec. III.B); the kernels follow the FP64 pass.
template <int ST>
struct MpField {
  using T = float;
};
template <>
struct MpField<LBM_F64> {
  using T = double;
};

// Non-ideal pressure of Sec. III.B, Eq. eos.
__device__ __forceinline__ double eos_p(double r) {
  return r * (5.3e-2 +
              r * (-3.818183621928911e-2 +
                   r * (4.139745482116095e-3 +
                        r * (3.748484095210317e-4 +
                             r * (-1.4552652965531227e-4 + r * 1.2746947442749278e-5)))));
}

template <int ST>
__device__ __forceinline__ void mp_put(const InstDev& I, uint32_t node, double rho) {
  using FT = typename MpField<ST>::T;
  FT* fld = static_cast<FT*>(I.mp_field);
  fld[node] = (FT)rho;
  fld[I.N + node] = (FT)sqrt(rho / 3.0 - eos_p(rho));
}

// ---------------------------------------------------------------------------
// Boundary kernel: special nodes of the scanned regions.
// ---------------------------------------------------------------------------
// Coordinates of a box-local index (x fastest).  A box lies inside one
// instance, so the index is below 2^31 and 32-bit division is exact (64-bit
// division is a long software sequence on this target).
__device__ __forceinline__ bool box_local(const Region& rg, int64_t local, int& x, int& y, int& z) {
  const uint32_t ex = (uint32_t)(rg.hi[0] - rg.lo[0]), ey = (uint32_t)(rg.hi[1] - rg.lo[1]);
  const uint32_t l = (uint32_t)local;
  const uint32_t r = l / ex;
  const uint32_t zz = r / ey;
  x = rg.lo[0] + (int)(l - r * ex);
  y = rg.lo[1] + (int)(r - zz * ey);
  z = rg.lo[2] + (int)zz;
  return z < rg.hi[2];
}

__device__ __forceinline__ bool in_region(const Region& rg, int x, int y, int z) {
  return x >= rg.lo[0] && x < rg.hi[0] && y >= rg.lo[1] && y < rg.hi[1] && z >= rg.lo[2] &&
         z < rg.hi[2];
}

// Boundary node lists: the nodes with missing populations of the scanned
// regions, each once (a node inside an earlier region of its instance
// belongs to that region's tiles), as (instance, node) pairs appended with one
// atomic per list and workgroup.  Nodes with a cut link to a body go to
// list[...] (count[0], one wavefront each); nodes whose missing populations
// all come from wall faces go to list[cap + ...] (count[1], one thread each).
// Inflow and outflow plane nodes are left to the bulk kernel.
template <int Q>
__global__ void __launch_bounds__(256) k_boundary_scan(const InstDev* __restrict__ insts,
                                                       const Region* __restrict__ regions,
                                                       const BoxTile* __restrict__ btiles, int bt0,
                                                       const uint8_t* __restrict__ flags,
                                                       uint2* list, uint32_t cap, uint32_t* count) {
  const BoxTile bt = btiles[bt0 + blockIdx.x];
  const Region rg = regions[bt.region];
  const InstDev& I = insts[rg.inst];
  const int k = threadIdx.x;
  bool take = false, body = false;
  uint32_t node = 0;
  int x, y, z;
  if (k < bt.count && I.flag_off >= 0 && box_local(rg, bt.local0 + k, x, y, z)) {
    bool owned = true;
    for (int r = rg.first; r < bt.region; ++r)
      if (in_region(regions[r], x, y, z)) owned = false;
    node = node_index(I, x, y, z);
    const uint8_t fv = flags[I.flag_off + node];
    const bool face = (x == 0 && I.face[0] == LBM_FACE_INLET) ||
                      (x == I.nx - 1 && I.face[1] == LBM_FACE_OUTLET);
    take = owned && !face && !(fv & FLAG_SOLID) && (fv & (FLAG_STATIC | FLAG_BODY));
    body = (fv & FLAG_BODY) != 0;
  }
  // One atomic per list and workgroup (not per wave): every wave of a wall
  // plane has nodes to append, and same-address atomics serialise.
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ uint32_t s_cnt[2][4];
  __shared__ uint32_t s_base[2];
  uint64_t m[2];
#pragma unroll
  for (int which = 0; which < 2; ++which) {
    m[which] = __ballot(take && (body == (which == 0)));
    if (lane == 0) s_cnt[which][wv] = (uint32_t)__popcll(m[which]);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int which = threadIdx.x;
    const uint32_t tot = s_cnt[which][0] + s_cnt[which][1] + s_cnt[which][2] + s_cnt[which][3];
    s_base[which] = tot ? atomicAdd(count + which, tot) : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int which = 0; which < 2; ++which) {
    if (take && (body == (which == 0))) {
      uint32_t slot = s_base[which] + (uint32_t)__popcll(m[which] & ((1ull << lane) - 1ull));
      for (int w = 0; w < wv; ++w) slot += s_cnt[which][w];
      if (slot < cap) list[which * cap + slot] = make_uint2((uint32_t)rg.inst, node);
    }
  }
}

// Nodes whose missing populations all come from wall faces (resting walls
// half a spacing outside the face, q = 1/2), one thread each: the
// pre-collision state with Grad's approximation for the missing populations
// (Sec. II.C.1) and the KBC collision (Eqs. 1-6), in FP64 except for D3Q27
// with FP32 or 16-bit storage (see RW below).  Consecutive list entries
// are mostly consecutive nodes of a wall row, so the loads coalesce.
template <bool C, typename A, typename B>
struct pick_type {
  using type = A;
};
template <typename A, typename B>
struct pick_type<false, A, B> {
  using type = B;
};

template <int Q, int ST, bool PRE>
__device__ __forceinline__ void boundary_wall_nodes(const StepBuffers& b,
                                                    const uint2* __restrict__ list,
                                                    const uint32_t* __restrict__ count,
                                                    uint32_t cap, int stat_slot, uint32_t bid,
                                                    uint32_t nblk) {
  using S = Store<ST>;
  using T = typename S::T;
  // Arithmetic type: the storage's (FP32 for FP32 and 16-bit storage, with
  // gamma from FP64 near equilibrium, as in the bulk kernel) for D3Q27
  // collisions, whose FP64 form needs 256 VGPRs and spills (one wave per
  // SIMD); FP64 for D2Q9 (its launch is shared with the cut-link kernel,
  // whose registers bound it anyway) and for the multiphase pre-collision
  // state.
  using RW = typename pick_type<(Q == 27 && !PRE), typename S::R, double>::type;
  const double t1 = (double)(*b.clock + 1);
  float gmin = 1e30f, gmax = -1e30f;
  double gsum = 0.0;
  uint32_t cnt = 0, f64 = 0;
  const uint32_t n = min(*count, cap);
  for (uint32_t k = bid * 64 + threadIdx.x; k < n; k += nblk * 64) {
    const uint2 e = list[k];
    const InstDev& I = b.insts[e.x];
    const T* sb = static_cast<const T*>(b.src) + I.pop_off;
    T* db = static_cast<T*>(b.dst) + I.pop_off;
    const uint8_t* fl = b.flags + I.flag_off;
    const Coord c = node_coord(I, e.y);
    RW f[Q];
    // Every missing population of these nodes comes from a wall face (q = 1/2,
    // at rest): the body cut-link code is left out.
    gather_pre<Q, ST, RW, true, PRE>(I, sb, fl, c.x, c.y, c.z, t1, f);
    if constexpr (PRE) {
      // Multiphase: the pre-collision state and its density, for the forced
      // collision that follows.
      double rt = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        db[i * I.stride + e.y] = S::enc_d(f[i]);
        rt += f[i];
      }
      mp_put<ST>(I, e.y, 1.0 + rt);
      continue;
    }
    CollideParams<RW> P;
    P.beta = (RW)I.beta;
    P.inv_beta = (RW)(1.0 / I.beta);
    P.beta_d = I.beta;
    P.lbgk = I.collision;
    P.trace_in_s = I.trace_in_s;
    P.near_eq = sizeof(RW) == 4 ? I.near_eq : 0.0f;
    CollideOut co;
    if (!collide<Q, RW, false>(f, P, co)) atomicOr(b.err, 1u);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if constexpr (sizeof(RW) == 4) db[i * I.stride + e.y] = S::enc(f[i]);
      else db[i * I.stride + e.y] = S::enc_d(f[i]);
    }
    gmin = fminf(gmin, co.gamma);
    gmax = fmaxf(gmax, co.gamma);
    gsum += co.gamma;
    cnt += 1;
    f64 += sizeof(RW) == 4 ? (uint32_t)co.fp64 : 1u;
  }
  if (b.stats) block_stats<64>(gmin, gmax, gsum, cnt, f64, b.stats + stat_slot);
}

template <int Q, int ST, bool PRE>
__global__ void __launch_bounds__(64) k_boundary_wall(StepBuffers b, const uint2* __restrict__ list,
                                                     const uint32_t* __restrict__ count,
                                                     uint32_t cap, int stat0) {
  boundary_wall_nodes<Q, ST, PRE>(b, list, count, cap, stat0 + (int)blockIdx.x, blockIdx.x,
                                  gridDim.x);
}

// One DPP lane exchange of a double (two 32-bit moves); CTRL is the DPP
// control word: 0xB1 / 0x4E swap neighbours / pairs within a quad, 0x141
// mirrors each 8-lane half-row, 0x140 each 16-lane row.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the GL lanes of a group (GL = 32 or 64; all 64 lanes active), the
// same value in every lane of the group, fixed order.  Register-to-register
// DPP exchanges within each 16-lane row (every step adds the same pair in
// both lanes, so the row sum is identical across the row), then the row sums
// are read back as scalars: no LDS round trips.
template <int GL>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(GL == 32 || GL == 64, "group of 32 or 64 lanes");
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
  const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
  if (GL == 64) return (r0 + r1) + (r2 + r3);
  return (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
}

// Value for lattice velocity component c in {0, +1, -1}; the operands are
// plain values so that a per-lane choice stays a register select.
__device__ __forceinline__ double pick3(int c, double v0, double vp, double vm) {
  return c == 0 ? v0 : (c > 0 ? vp : vm);
}

// Lagged-field slot of x + k c_i (k = 1, 2), slot 0 being x itself.
template <int Q>
__device__ __forceinline__ int lag_slot(int i, int k) {
  return 1 + 2 * (i < rest<Q>() ? i : i - 1) + (k - 1);
}

// ---------------------------------------------------------------------------
// Nodes with a cut link to a body (and any wall links they have), one group
// of GL lanes per node (GL = 64 for D3Q27, 32 for D2Q9: two nodes per
// wavefront).
// gather_pre above does the same work in one thread, reading the lagged
// moments of up to 2(Q-1)+1 neighbours one after another; here the lanes take
// them in parallel:
//   lane i < Q            source of population i (pull, wall, solid),
//                         A_opp(i)(x), cut fraction and wall velocity;
//   lane l < 2(Q-1)+1     lagged (rho~, u) of x (l = 0) or x + k c_i where
//                         Grad's target velocity or the velocity gradient
//                         needs it;
//   lane i < Q            its term of the target density and, if missing,
//                         its target velocity (group sums: rho_t, u_t);
//   lane a + 3 b < 9      the target gradient entry G[a][b] (Sec. II.C.1);
//   lane i < Q            f*_i for the missing i, then the KBC collision
//                         (Eqs. 1-6) lane-parallel in FP64 with group sums,
//                         and the store of population i.
// The arithmetic of the cut-link nodes is FP64 for every storage form.
// Workgroups (one wavefront) stride over the node list.
// ---------------------------------------------------------------------------
template <int Q, int ST, bool PRE>
__device__ __forceinline__ void boundary_wave_nodes(const StepBuffers& b,
                                                    const uint2* __restrict__ list,
                                                    const uint32_t* __restrict__ count,
                                                    uint32_t cap, int stat_slot, uint32_t bid,
                                                    uint32_t nblk) {
  using S = Store<ST>;
  using T = typename S::T;
  constexpr int D = dims<Q>();
  constexpr int GL = Q == 27 ? 64 : 32;
  constexpr int NG = 64 / GL;                 // nodes per wavefront
  constexpr int NS = 2 * (Q - 1) + 1;
  static_assert(NS <= GL, "one lane per lagged-field slot");
  __shared__ double s_f[NG][Q], s_opp[NG][Q], s_q[NG][Q], s_uw[NG][Q][3];
  __shared__ double s_lr[NG][NS], s_lu[NG][NS][3];
  __shared__ int s_lf[NG][NS];
  __shared__ uint32_t s_miss[NG];
  __shared__ double s_G[NG][9];    // target velocity gradient G[a + 3 b]
  const int g = threadIdx.x / GL, lane = threadIdx.x % GL;
  const double t1 = (double)(*b.clock + 1);
  float gmin = 1e30f, gmax = -1e30f;
  double gsum = 0.0;
  uint32_t cnt = 0, f64 = 0;
  const uint32_t n = min(*count, cap);
  for (uint32_t base = bid * NG; base < n; base += nblk * NG) {
    const uint32_t k = base + g;
    const bool active = k < n;
    const uint2 e = active ? list[k] : make_uint2(0u, 0u);
    const InstDev& I = b.insts[e.x];
    const T* sb = static_cast<const T*>(b.src) + I.pop_off;
    T* db = static_cast<T*>(b.dst) + I.pop_off;
    const uint8_t* fl = b.flags + (I.flag_off >= 0 ? I.flag_off : 0);
    const int64_t stride = I.stride;
    const Coord c = node_coord(I, e.y);
    const int x = c.x, y = c.y, z = c.z;
    const uint32_t me = e.y;
    if (lane == 0) s_miss[g] = 0u;
    __syncthreads();
    // ---- sources of the populations, cut links --------------------------
    // (Nodes on inflow / outflow planes are on the other list: every source
    // here is a node or a wall.)  The flag and the population are loaded
    // together; a solid source's value is dropped.
    if (active && lane < Q) {
      const int i = lane;
      int sr[3] = {x - cx(i), y - cy(i), z - cz<Q>(i)};
      const int nn[3] = {I.nx, I.ny, I.nz};
      bool w = false;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (sr[a] >= 0 && sr[a] < nn[a]) continue;
        if (I.face[2 * a + (sr[a] < 0 ? 0 : 1)] == LBM_FACE_PERIODIC) sr[a] = (sr[a] + nn[a]) % nn[a];
        else w = true;
      }
      double fi = 0.0;
      bool missing = w;
      const T opp = sb[(Q - 1 - i) * stride + me];
      if (!w) {
        const uint32_t m = node_index(I, sr[0], sr[1], sr[2]);
        const uint8_t fs = fl[m];
        const T v = sb[i * stride + m];
        if (fs & FLAG_SOLID) missing = true;
        else fi = (double)S::dec(v);
      }
      s_f[g][i] = fi;
      if (missing) {
        atomicOr(&s_miss[g], 1u << i);
        s_opp[g][i] = (double)S::dec(opp);
        double q = 0.5, ud[3] = {0.0, 0.0, 0.0};
        if (!w) body_cut(I, x, y, z, cx(i), cy(i), cz<Q>(i), t1, q, ud);
        s_q[g][i] = q;
        for (int a = 0; a < 3; ++a) s_uw[g][i][a] = ud[a];
      }
    }
    __syncthreads();
    const uint32_t miss = s_miss[g];
    // ---- lagged fields of the neighbours needed ---------------------------
    // (x itself; x + c_i and x + 2 c_i for the missing i and for the axis
    // directions.)  The flag and the Q populations are loaded together.
    if (active && lane < NS) {
      bool need;
      int off[3] = {0, 0, 0};
      if (lane == 0) {
        need = miss != 0u;
      } else {
        const int j = (lane - 1) >> 1, kk = ((lane - 1) & 1) + 1;
        const int i = j < rest<Q>() ? j : j + 1;
        off[0] = kk * cx(i);
        off[1] = kk * cy(i);
        off[2] = kk * cz<Q>(i);
        need = miss && (((miss >> i) & 1u) || nnz<Q>(i) == 1);
      }
      int fluid = 0;
      uint32_t m;
      if (need && resolve_nb(I, x, y, z, off[0], off[1], off[2], m)) {
        const uint8_t fs = fl[m];
        T v[Q];
#pragma unroll
        for (int p = 0; p < Q; ++p) v[p] = sb[p * stride + m];
        if (lane == 0 || !(fs & FLAG_SOLID)) {
          double rt = 0.0, j3[3] = {0.0, 0.0, 0.0};
#pragma unroll
          for (int p = 0; p < Q; ++p) {
            const double dv = (double)S::dec(v[p]);
            rt += dv;
            if (cx(p) > 0) j3[0] += dv;
            if (cx(p) < 0) j3[0] -= dv;
            if (cy(p) > 0) j3[1] += dv;
            if (cy(p) < 0) j3[1] -= dv;
            if (cz<Q>(p) > 0) j3[2] += dv;
            if (cz<Q>(p) < 0) j3[2] -= dv;
          }
          const double ir = 1.0 / (1.0 + rt);
          s_lr[g][lane] = rt;
          for (int a = 0; a < 3; ++a) s_lu[g][lane][a] = j3[a] * ir;
          fluid = 1;
        }
      }
      s_lf[g][lane] = fluid;
    }
    __syncthreads();
    // ---- Grad target values (Sec. II.C.1), lane-parallel -------------------
    // Lane i forms the target-density term and the target velocity of its
    // own population (group sums give rho_t and u_t); lanes a + 3 b < 9 form
    // the gradient entry G[a][b] = d u_a / d x_b.
    const int i = lane;
    const bool pop = active && i < Q;
    const bool mi = pop && ((miss >> i) & 1u);
    double tr = 0.0, v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (mi) {
      // Bounce-back-implied density plus the wall-motion term.
      const double rho_n = 1.0 + s_lr[g][0];
      const double w0 = s_uw[g][i][0], w1 = s_uw[g][i][1], w2 = s_uw[g][i][2];
      tr = s_opp[g][i] + 6.0 * weight<Q>(i) * rho_n * (cx(i) * w0 + cy(i) * w1 + cz<Q>(i) * w2);
      // Velocity at x interpolated along c_i through the wall point (s = -q)
      // and the lagged velocities at x + c_i (s = 1), x + 2 c_i (s = 2).
      const double q = s_q[g][i];
      const int l1 = lag_slot<Q>(i, 1), l2 = lag_slot<Q>(i, 2);
      if (s_lf[g][l1] && s_lf[g][l2]) {
        const double a0 = 2.0 / ((1.0 + q) * (2.0 + q));
        const double a1 = 2.0 * q / (1.0 + q);
        const double a2 = -q / (2.0 + q);
        v0 = a0 * w0 + a1 * s_lu[g][l1][0] + a2 * s_lu[g][l2][0];
        v1 = a0 * w1 + a1 * s_lu[g][l1][1] + a2 * s_lu[g][l2][1];
        v2 = a0 * w2 + a1 * s_lu[g][l1][2] + a2 * s_lu[g][l2][2];
      } else if (s_lf[g][l1]) {
        const double iq = 1.0 / (1.0 + q);
        v0 = (w0 + q * s_lu[g][l1][0]) * iq;
        v1 = (w1 + q * s_lu[g][l1][1]) * iq;
        v2 = (w2 + q * s_lu[g][l1][2]) * iq;
      } else {
        v0 = w0;
        v1 = w1;
        v2 = w2;
      }
    } else if (pop) {
      tr = s_f[g][i];
    }
    const double rho_t = 1.0 + group_sum<GL>(tr);
    const double nmi = miss ? 1.0 / (double)__popc(miss) : 0.0;
    const double ut[3] = {group_sum<GL>(v0) * nmi, group_sum<GL>(v1) * nmi,
                          group_sum<GL>(v2) * nmi};
    // G[a][b]: central differences of the lagged velocity; on a cut side the
    // quadratic through the wall point, x + e, x + 2 e (linear if x + 2 e is
    // not fluid); both sides cut: across the two wall points.
    if (active && lane < 9) {
      const int a = lane % 3, bb = lane / 3;
      double gr = 0.0;
      if (miss && a < D && bb < D) {
        const int ip = axis_pop<Q>(bb, +1);   // c = +e_b: slots x + e_b, x + 2 e_b
        const int im = axis_pop<Q>(bb, -1);   // c = -e_b
        const bool cut_m = (miss >> ip) & 1u, cut_p = (miss >> im) & 1u;
        const int p1 = lag_slot<Q>(ip, 1), p2 = lag_slot<Q>(ip, 2);
        const int m1 = lag_slot<Q>(im, 1), m2 = lag_slot<Q>(im, 2);
        const bool fp1 = s_lf[g][p1], fp2 = fp1 && s_lf[g][p2];
        const bool fm1 = s_lf[g][m1], fm2 = fm1 && s_lf[g][m2];
        if (cut_m && cut_p) {
          gr = (s_uw[g][im][a] - s_uw[g][ip][a]) / (s_q[g][im] + s_q[g][ip]);
        } else if (cut_m) {
          const double qm = s_q[g][ip], wm = s_uw[g][ip][a];
          if (fp2)
            gr = -3.0 * wm / ((1.0 + qm) * (2.0 + qm)) + s_lu[g][p1][a] * (2.0 - qm) / (1.0 + qm) +
                 s_lu[g][p2][a] * (qm - 1.0) / (2.0 + qm);
          else if (fp1)
            gr = (s_lu[g][p1][a] - wm) / (1.0 + qm);
        } else if (cut_p) {
          const double qp = s_q[g][im], wp = s_uw[g][im][a];
          if (fm2)
            gr = 3.0 * wp / ((1.0 + qp) * (2.0 + qp)) - s_lu[g][m1][a] * (2.0 - qp) / (1.0 + qp) -
                 s_lu[g][m2][a] * (qp - 1.0) / (2.0 + qp);
          else if (fm1)
            gr = (wp - s_lu[g][m1][a]) / (1.0 + qp);
        } else if (fp1 && fm1) {
          gr = 0.5 * (s_lu[g][p1][a] - s_lu[g][m1][a]);
        } else if (fp1) {
          gr = s_lu[g][p1][a] - s_lu[g][0][a];
        } else if (fm1) {
          gr = s_lu[g][0][a] - s_lu[g][m1][a];
        }
      }
      s_G[g][lane] = gr;
    }
    __syncthreads();
    // ---- f* for the missing populations, then the collision ----------------
    // Pi = rho/3 I + rho u u - rho/(6 beta) (G + G^T)  (Pi^eq + Pi^neq, cs^2 = 1/3)
    double d = 0.0;
    if (pop) {
      d = s_f[g][i];
      if (mi) {
        const double kneq = rho_t / (6.0 * I.beta);
        const double (&G)[9] = s_G[g];   // G[a + 3 b]
        const double Pi[6] = {rho_t / 3.0 + rho_t * ut[0] * ut[0] - kneq * 2.0 * G[0],
                              rho_t / 3.0 + rho_t * ut[1] * ut[1] - kneq * 2.0 * G[4],
                              rho_t / 3.0 + rho_t * ut[2] * ut[2] - kneq * 2.0 * G[8],
                              rho_t * ut[0] * ut[1] - kneq * (G[3] + G[1]),
                              rho_t * ut[0] * ut[2] - kneq * (G[6] + G[2]),
                              rho_t * ut[1] * ut[2] - kneq * (G[7] + G[5])};
        d = grad_dev<Q, double>(i, rho_t, ut, Pi);
      }
    }
    if constexpr (PRE) {
      // Multiphase (only its pre-collision mode needs this): the filled
      // populations carry the mass that bounce-back would return, rho_t less
      // the known populations (scaled as full f).  The sums run on every
      // wavefront so that the lane exchanges stay uniform; only multiphase
      // instances apply them.
      const double fi = pop ? d + weight<Q>(i) : 0.0;
      const double sm = group_sum<GL>(pop && mi ? fi : 0.0);
      const double sk = group_sum<GL>(pop && !mi ? fi : 0.0);
      if (I.mp && pop && mi && sm > 0.0) d = (rho_t - sk) / sm * fi - weight<Q>(i);
    }
    // Moments of the pre-collision state.
    const double rt = group_sum<GL>(pop ? d : 0.0);
    if constexpr (PRE) {
      // Multiphase: the pre-collision state and its density, for the forced
      // collision that follows.
      if (pop) db[i * stride + me] = S::enc_d(d);
      if (active && lane == 0) mp_put<ST>(I, me, 1.0 + rt);
      __syncthreads();
      continue;
    }
    const double jx = group_sum<GL>(pop ? cx(i) * d : 0.0);
    const double jy = group_sum<GL>(pop ? cy(i) * d : 0.0);
    const double jz = group_sum<GL>(pop ? cz<Q>(i) * d : 0.0);
    const double rho = 1.0 + rt, ir = 1.0 / rho;
    const double u[3] = {jx * ir, jy * ir, jz * ir};
    const bool ok = rho > 0.0 && fabs(u[0]) < 1.0 && fabs(u[1]) < 1.0 && fabs(u[2]) < 1.0;
    const int c0 = pop ? cx(i) : 0, c1 = pop ? cy(i) : 0, c2 = pop ? cz<Q>(i) : 0;
    const AxisEq<double> ax = axis_eq(u[0]), ay = axis_eq(u[1]);
    const AxisEq<double> az = Q == 27 ? axis_eq(u[2]) : ay;
    double E = pick3(c0, ax.e0, ax.ep, ax.em);
    {
      const double ey = pick3(c1, ay.e0, ay.ep, ay.em);
      E = E + ey + E * ey;
      if (Q == 27) {
        const double ez = pick3(c2, az.e0, az.ep, az.em);
        E = E + ez + E * ez;
      }
    }
    // Delta = f - f^eq, with the mass and momentum rounding left in it moved
    // to the rest and axis populations (the second moments are unchanged).
    double dl = pop ? d - weight<Q>(i) * (rt + rho * E) : 0.0;
    const double rm = group_sum<GL>(dl);
    const double qx = group_sum<GL>(c0 * dl);
    const double qy = group_sum<GL>(c1 * dl);
    const double qz = group_sum<GL>(c2 * dl);
    const int nz = (c0 != 0) + (c1 != 0) + (c2 != 0);
    if (pop) {
      if (nz == 0) dl -= rm;
      if (nz == 1) dl -= 0.5 * (c0 * qx + c1 * qy + c2 * qz);
    }
    // Second moments and the shear part (closed form, as in the bulk).
    const double Pxx = group_sum<GL>(c0 != 0 ? dl : 0.0);
    const double Pyy = group_sum<GL>(c1 != 0 ? dl : 0.0);
    const double Pzz = group_sum<GL>(c2 != 0 ? dl : 0.0);
    const double Pxy = group_sum<GL>((double)(c0 * c1) * dl);
    const double Pxz = group_sum<GL>((double)(c0 * c2) * dl);
    const double Pyz = group_sum<GL>((double)(c1 * c2) * dl);
    double T, Dxx, Dyy, Dzz;
    if (Q == 27) {
      T = Pxx + Pyy + Pzz;
      Dxx = Pxx - T / 3.0;
      Dyy = Pyy - T / 3.0;
      Dzz = -(Dxx + Dyy);
    } else {
      T = Pxx + Pyy;
      Dxx = 0.5 * (Pxx - Pyy);
      Dyy = -Dxx;
      Dzz = 0.0;
    }
    const double ts = I.trace_in_s ? T : 0.0;
    double si = 0.0;   // Delta s_i (faces: Dev/2 + T/(2D) with the trace; edges: +-P_ab/4)
    if (pop) {
      if (nz == 1) si = 0.5 * (c0 != 0 ? Dxx : (c1 != 0 ? Dyy : Dzz)) + ts * (0.5 / D);
      else if (nz == 2) si = 0.25 * (c0 * c1 * Pxy + c0 * c2 * Pxz + c1 * c2 * Pyz);
      else if (nz == 0) si = -ts;
    }
    const double hi = dl - si;
    double inv = 0.0;   // 1 / f^eq_i
    if (pop) {
      inv = ir * pick3(c0, ax.g0, ax.gp, ax.gm) * pick3(c1, ay.g0, ay.gp, ay.gm);
      if (Q == 27) inv *= pick3(c2, az.g0, az.gp, az.gm);
    }
    const double aa = group_sum<GL>(si * hi * inv);
    const double bb = group_sum<GL>(hi * hi * inv);
    double gamma = 2.0;
    if (!I.collision && bb > 1e-300) gamma = 1.0 / I.beta - (2.0 - 1.0 / I.beta) * aa / bb;
    if (pop) {
      const double outv = ok ? d - I.beta * (2.0 * si + gamma * hi) : d;
      db[i * stride + me] = S::enc_d(outv);
    }
    if (active && lane == 0) {
      if (!ok) atomicOr(b.err, 1u);
      const float gf = ok ? (float)gamma : 2.0f;
      gmin = fminf(gmin, gf);
      gmax = fmaxf(gmax, gf);
      gsum += gf;
      cnt += 1;
      f64 += 1;
    }
    __syncthreads();
  }
  if (b.stats) block_stats<64>(gmin, gmax, gsum, cnt, f64, b.stats + stat_slot);
}

template <int Q, int ST, bool PRE>
__global__ void __launch_bounds__(64) k_boundary_wave(StepBuffers b, const uint2* __restrict__ list,
                                                     const uint32_t* __restrict__ count,
                                                     uint32_t cap, int stat0) {
  boundary_wave_nodes<Q, ST, PRE>(b, list, count, cap, stat0 + (int)blockIdx.x, blockIdx.x,
                                  gridDim.x);
}

// Both node lists in one launch: workgroups [0, nwg) take the cut-link nodes
// one wavefront (group) at a time, the rest the wall-row nodes one thread
// each, so the two run side by side rather than one after the other.  Used
// where the two kernels have the same register budget (D2Q9).
template <int Q, int ST, bool PRE>
__global__ void __launch_bounds__(64) k_boundary_both(StepBuffers b, const uint2* __restrict__ list,
                                                     const uint32_t* __restrict__ count,
                                                     uint32_t cap, int stat0, uint32_t nwg) {
  if (blockIdx.x < nwg)
    boundary_wave_nodes<Q, ST, PRE>(b, list, count, cap, stat0 + (int)blockIdx.x, blockIdx.x, nwg);
  else
    boundary_wall_nodes<Q, ST, PRE>(b, list + cap, count + 1, cap, stat0 + (int)blockIdx.x,
                                    blockIdx.x - nwg, gridDim.x - nwg);
}

// ---------------------------------------------------------------------------
// Geometry kernels over the swept boxes of moving bodies.
// ---------------------------------------------------------------------------
template <int Q, int ST>
__global__ void __launch_bounds__(256) k_geometry(int stage, const InstDev* __restrict__ insts,
                                                  const Region* __restrict__ regions,
                                                  const BoxTile* __restrict__ gtiles, void* src,
                                                  uint8_t* flags, const int64_t* clock, int toff) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  const BoxTile gt = gtiles[blockIdx.x];
  const Region rg = regions[gt.region];
  const InstDev& I = insts[rg.inst];
  uint8_t* fl = flags + I.flag_off;
  const double t = (double)(*clock + toff);
  const int k = threadIdx.x;
  if (k >= gt.count) return;
  int x, y, z;
  if (!box_local(rg, gt.local0 + k, x, y, z)) return;
  const uint32_t node = node_index(I, x, y, z);
  const uint8_t fv = fl[node];
  if (stage == 0) {
    // Solid at the next time; a fresh node (solid now, fluid at the next
    // time) is refilled with the equilibrium at the mean lagged density of
    // the neighbours that are fluid now and the body velocity.  The refill
    // reads only the FLAG_SOLID bits of the neighbours, which this stage
    // does not change, and the populations of nodes that are fluid now,
    // which it does not write.
    const bool in = body_inside(I, x, y, z, t);
    fl[node] = (uint8_t)((fv & ~FLAG_SOLID_NEXT) | (in ? FLAG_SOLID_NEXT : 0));
    if (!((fv & FLAG_SOLID) && !in)) return;
    T* sb = static_cast<T*>(src) + I.pop_off;
    R sum = R(0);
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (i == rest<Q>()) continue;
      uint32_t m;
      if (!resolve_nb(I, x, y, z, cx(i), cy(i), cz<Q>(i), m)) continue;
      if (fl[m] & FLAG_SOLID) continue;
      R rt, uu[3];
      lagged<Q, ST, R>(sb, I.stride, m, rt, uu);
      sum += R(1) + rt;
      ++cnt;
    }
    const R rb = cnt ? sum / R(cnt) : R(1);
    double ub[3];
    body_velocity(I, x, y, z, t, ub);
    const R u[3] = {(R)ub[0], (R)ub[1], (R)ub[2]};
    R fe[Q];
    feq_dev<Q, R>(rb - R(1), u, fe);
#pragma unroll
    for (int i = 0; i < Q; ++i) sb[i * I.stride + node] = S::enc(fe[i]);
  } else {
    // SOLID_NEXT becomes current; fluid nodes with a solid x - c_i are cut.
    const bool solid = fv & FLAG_SOLID_NEXT;
    bool cut = false;
    if (!solid) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        uint32_t m;
        if (resolve_nb(I, x, y, z, -cx(i), -cy(i), -cz<Q>(i), m) && (fl[m] & FLAG_SOLID_NEXT))
          cut = true;
      }
    }
    fl[node] = (uint8_t)((fv & (FLAG_STATIC | FLAG_SOLID_NEXT)) | (solid ? FLAG_SOLID : 0) |
                         (cut ? FLAG_BODY : 0));
  }
}

// ---------------------------------------------------------------------------
// FP64-gamma pass over the near-equilibrium nodes deferred by the bulk kernel:
// the node is streamed and collided again from the same source state, with
// gamma from FP64, and its output overwritten.
// ---------------------------------------------------------------------------
template <int Q, int ST>
__global__ void __launch_bounds__(256) k_neq_fixup(StepBuffers b, int stat0) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // End of the step: the boundary lists were consumed before; only the
    // geometry and boundary kernels, which ran before, read the clock.
    for (int j = 0; j < b.nbcount; ++j) b.bcount[j] = 0u;
    if (b.clock_tick) *b.clock_tick += 1;
  }
  float gmin = 1e30f, gmax = -1e30f;
  double gsum = 0.0;
  uint32_t cnt = 0, f64 = 0;
  // Each wavefront takes 64 mask words at a time, one per lane, and works
  // through their set bits 64 at a time: lane l takes the set bit of rank
  // r + l in lane order, found from the exclusive prefix sum of the words'
  // bit counts (the owner lane by binary search over lanes, then the bit
  // within the owner's word by binary search over popcounts).
  const int lane = threadIdx.x & 63;
  const uint32_t nwaves = gridDim.x * 4u;
  for (uint32_t c0 = (blockIdx.x * 4u + (threadIdx.x >> 6)) * 64u; c0 < b.neq_nwords;
       c0 += nwaves * 64u) {
    const uint32_t wi = c0 + (uint32_t)lane;
    const uint64_t w = wi < b.neq_nwords ? b.neq_words[wi] : 0ull;
    if (__ballot(w != 0ull) == 0ull) continue;
    // Every word is zero again for the next step's bulk kernel.
    if (w != 0ull) b.neq_words[wi] = 0ull;
    const uint32_t pc = (uint32_t)__popcll(w);
    uint32_t incl = pc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t t = (uint32_t)__shfl_up((int)incl, d);
      if (lane >= d) incl += t;
    }
    const uint32_t excl = incl - pc;
    const uint32_t total = (uint32_t)__shfl((int)incl, 63);
    for (uint32_t r = 0; r < total; r += 64u) {
      const uint32_t g = r + (uint32_t)lane;
      // Owner: the last lane o with excl[o] <= g (it has bits: a lane
      // without bits shares its prefix with the lane after it).
      int o = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        const int cand = o + step;
        const uint32_t v = (uint32_t)__shfl((int)excl, cand & 63);
        if (cand < 64 && v <= g) o = cand;
      }
      const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)w, o);
      const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(w >> 32), o);
      uint64_t wo = ((uint64_t)hi << 32) | lo;
      uint32_t rank = g - (uint32_t)__shfl((int)excl, o);
      if (g >= total) continue;
      int bit = 0;
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) {
        const uint32_t cl = (uint32_t)__popcll(wo & ((1ull << sh) - 1ull));
        if (rank >= cl) {
          rank -= cl;
          wo >>= sh;
          bit += sh;
        }
      }
      const uint32_t gw = c0 + (uint32_t)o;
      const uint32_t ti = gw / b.neq_wpt;
      const uint32_t loc = (gw - ti * b.neq_wpt) * 64u + (uint32_t)bit;
      const Tile tl = b.tiles[ti];
      // A bit beyond the tile's nodes names no node (the bulk kernel sets
      // bits of its own nodes only): skipped.
      if (loc >= (uint32_t)tl.count) continue;
      const InstDev& I = b.insts[tl.inst];
      const uint32_t node = (uint32_t)(tl.node0 + loc);
      const T* sb = static_cast<const T*>(b.src) + I.pop_off;
      T* db = static_cast<T*>(b.dst) + I.pop_off;
      const Coord c = node_coord(I, node);
      R f[Q];
      // Deferred nodes come from the bulk kernel, whose nodes have every
      // source inside the instance (face planes and cut-link nodes are
      // flagged and never deferred); a source that does not resolve means a
      // corrupt mask word: the node is left as the bulk kernel wrote it and
      // the error word is set.
      bool resolved = true;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        uint32_t m = node;
        if (!resolve_nb(I, c.x, c.y, c.z, -cx(i), -cy(i), -cz<Q>(i), m)) {
          resolved = false;
          m = node;
        }
        f[i] = S::dec(sb[i * I.stride + m]);
      }
      if (!resolved) {
        atomicOr(b.err, 2u);
        continue;
      }
      CollideParams<R> P;
      P.beta = (R)I.beta;
      P.inv_beta = (R)(1.0 / I.beta);
      P.beta_d = I.beta;
      P.lbgk = I.collision;
      P.trace_in_s = I.trace_in_s;
      P.near_eq = I.near_eq;
      CollideOut co;
      if (!collide<Q, R, false>(f, P, co)) atomicOr(b.err, 1u);
#pragma unroll
      for (int i = 0; i < Q; ++i) db[i * I.stride + node] = S::enc(f[i]);
      gmin = fminf(gmin, co.gamma);
      gmax = fmaxf(gmax, co.gamma);
      gsum += co.gamma;
      cnt += 1;
      f64 += 1;
    }
  }
  if (b.stats) block_stats<256>(gmin, gmax, gsum, cnt, f64, b.stats + stat0 + blockIdx.x);
}


// ---------------------------------------------------------------------------
// Multiphase step (Sec. III.B).  After the boundary kernels have written the
// pre-collision state of their nodes (their pre-collision mode), three
// passes over the tiles:
//   stage 0 (k_mp_stream): every node with no special flag pulls its
//     populations into dst unchanged and writes its density and
//     phi = sqrt(rho cs^2 - p(rho)) to the instance's fields;
//   stage 1 (k_mp_lap): the lattice Laplacian of the density at every fluid
//     node, lap X = (2/cs^2) sum_i W_i (X(x + c_i) - X(x));
//   stage 2 (k_mp_collide): the body force
//       F = 2 phi grad(phi) + kappa rho grad(lap rho) + kappa_w rho sum_i W_i s(x + c_i) c_i,
//     with grad_a X = (1/cs^2) sum_i W_i c_ia X(x + c_i) (the kappa term's
//     sign is the one the divergence of the Korteweg tensor gives; a
//     neighbour that is not fluid gives the node's own value and s = 1),
//     then the KBC collision in FP64 with the exact difference method: the
//     post-collision state gains f^eq(rho, u + F/rho) - f^eq(rho, u), and
//     gamma uses the scalar product weighted by 1 / f^eq(rho, u + F/rho).
//     In place in dst.
// Field element type: FP64 for FP64 storage, FP32 otherwise; an instance's
// fields hold rho at [node], phi at [N + node] and lap at [2N + node].
// An instance with multiphase off gets F = 0 (the plain KBC collision, in
// FP64).
// ---------------------------------------------------------------------------
template <int Q, int ST>
__global__ void __launch_bounds__(256) k_mp_stream(StepBuffers b, const Tile* __restrict__ tiles,
                                                   int tile0) {
  using S = Store<ST>;
  using T = typename S::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& I = b.insts[tl.inst];
  if (!I.mp_field) return;
  const T* __restrict__ sb = static_cast<const T*>(b.src) + I.pop_off;
  T* __restrict__ db = static_cast<T*>(b.dst) + I.pop_off;
  const uint8_t* fl = I.flag_off >= 0 ? b.flags + I.flag_off : nullptr;
  const int nx = I.nx, ny = I.ny, nz = I.nz;
  const uint32_t sy = (uint32_t)nx, sz = (uint32_t)nx * (uint32_t)ny;
  const uint32_t wx = (uint32_t)(nx - 1), wy = (uint32_t)(ny - 1) * sy,
                 wz = (uint32_t)(nz - 1) * sz;
  for (int k = threadIdx.x; k < tl.count; k += 256) {
    const uint32_t node = (uint32_t)(tl.node0 + k);
    // Special nodes are the boundary kernels' (or solid); every source of
    // any other node lies inside the instance, wrapping periodically.
    if (fl && (fl[node] & FLAG_SPECIAL)) continue;
    const Coord c = node_coord(I, node);
    const uint32_t dm[3] = {c.x == 0 ? wx : 0u - 1u, c.y == 0 ? wy : 0u - sy,
                            c.z == 0 ? wz : 0u - sz};
    const uint32_t dp[3] = {c.x == nx - 1 ? 0u - wx : 1u, c.y == ny - 1 ? 0u - wy : sy,
                            c.z == nz - 1 ? 0u - wz : sz};
    auto dof = [&](int a, int ci) -> uint32_t { return ci == 0 ? 0u : (ci > 0 ? dm[a] : dp[a]); };
    T v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      // Source node index, formed modulo 2^32 (the -1 offsets are stored as
      // their 32-bit complements) before it is widened.
      const uint32_t src = node + dof(0, cx(i)) + dof(1, cy(i)) + (Q == 27 ? dof(2, cz<Q>(i)) : 0u);
      v[i] = sb[i * I.stride + (int64_t)src];
    }
    double rt = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      db[i * I.stride + node] = v[i];
      rt += (double)S::dec(v[i]);
    }
    mp_put<ST>(I, node, 1.0 + rt);
  }
}

template <int Q, int ST>
__global__ void __launch_bounds__(256) k_mp_lap(StepBuffers b, const Tile* __restrict__ tiles,
                                                int tile0) {
  using FT = typename MpField<ST>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& I = b.insts[tl.inst];
  if (!I.mp_field) return;
  FT* fld = static_cast<FT*>(I.mp_field);
  const uint8_t* fl = I.flag_off >= 0 ? b.flags + I.flag_off : nullptr;
  const int nx = I.nx, ny = I.ny, nz = I.nz;
  const uint32_t sy = (uint32_t)nx, sz = (uint32_t)nx * (uint32_t)ny;
  const uint32_t wx = (uint32_t)(nx - 1), wy = (uint32_t)(ny - 1) * sy,
                 wz = (uint32_t)(nz - 1) * sz;
  for (int k = threadIdx.x; k < tl.count; k += 256) {
    const uint32_t node = (uint32_t)(tl.node0 + k);
    const uint8_t fv = fl ? fl[node] : 0;
    if (fv & FLAG_SOLID) continue;
    const Coord c = node_coord(I, node);
    // Neighbours as in the collision pass: wrap offsets for nodes with no
    // face or body flag, resolved and flag-tested otherwise.
    const bool edge = fv & (FLAG_STATIC | FLAG_BODY);
    const uint32_t dn[3] = {c.x == 0 ? wx : 0u - 1u, c.y == 0 ? wy : 0u - sy,
                            c.z == 0 ? wz : 0u - sz};
    const uint32_t up[3] = {c.x == nx - 1 ? 0u - wx : 1u, c.y == ny - 1 ? 0u - wy : sy,
                            c.z == nz - 1 ? 0u - wz : sz};
    auto off = [&](int a, int ci) -> uint32_t { return ci == 0 ? 0u : (ci > 0 ? up[a] : dn[a]); };
    const double r0 = (double)fld[node];
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      uint32_t m = node + off(0, cx(i)) + off(1, cy(i)) + (Q == 27 ? off(2, cz<Q>(i)) : 0u);
      if (edge && !(resolve_nb(I, c.x, c.y, c.z, cx(i), cy(i), cz<Q>(i), m) &&
                    !(fl[m] & FLAG_SOLID)))
        m = node;
      s += weight<Q>(i) * ((double)fld[m] - r0);
    }
    fld[2 * I.N + node] = (FT)(6.0 * s);
  }
}

template <int Q, int ST>
__global__ void __launch_bounds__(256, 2) k_mp_collide(StepBuffers b, const Tile* __restrict__ tiles,
                                                    int tile0) {
  using S = Store<ST>;
  using T = typename S::T;
  using FT = typename MpField<ST>::T;
  constexpr int D = dims<Q>();
  const int ti = tile0 + blockIdx.x;
  const Tile tl = tiles[ti];
  const InstDev& I = b.insts[tl.inst];
  float gmin = 1e30f, gmax = -1e30f;
  double gsum = 0.0;
  uint32_t cnt = 0;
  if (I.mp_field) {
    T* __restrict__ db = static_cast<T*>(b.dst) + I.pop_off;
    const FT* __restrict__ fld = static_cast<const FT*>(I.mp_field);
    const uint8_t* fl = I.flag_off >= 0 ? b.flags + I.flag_off : nullptr;
    const int64_t N = I.N, stride = I.stride;
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const uint32_t sy = (uint32_t)nx, sz = (uint32_t)nx * (uint32_t)ny;
    const uint32_t wx = (uint32_t)(nx - 1), wy = (uint32_t)(ny - 1) * sy,
                   wz = (uint32_t)(nz - 1) * sz;
    for (int k = threadIdx.x; k < tl.count; k += 256) {
      const uint32_t node = (uint32_t)(tl.node0 + k);
      const uint8_t fv = fl ? fl[node] : 0;
      if (fv & FLAG_SOLID) continue;
      const Coord c = node_coord(I, node);
      // ---- body force, before the populations are loaded -------------------
      double F[3] = {0.0, 0.0, 0.0};
      if (I.mp) {
        // A node with no face or body flag has only fluid neighbours, inside
        // the instance or across periodic faces (32-bit wrap offsets as in
        // the stream pass); the others resolve each neighbour and read its
        // flag.  A neighbour that is not fluid reads the node's own values.
        const bool edge = fv & (FLAG_STATIC | FLAG_BODY);
        const uint32_t dn[3] = {c.x == 0 ? wx : 0u - 1u, c.y == 0 ? wy : 0u - sy,
                                c.z == 0 ? wz : 0u - sz};
        const uint32_t up[3] = {c.x == nx - 1 ? 0u - wx : 1u, c.y == ny - 1 ? 0u - wy : sy,
                                c.z == nz - 1 ? 0u - wz : sz};
        auto off = [&](int a, int ci) -> uint32_t { return ci == 0 ? 0u : (ci > 0 ? up[a] : dn[a]); };
        const double rho0 = (double)fld[node];
        const double p0 = (double)fld[N + node];
        double gp[3] = {0.0, 0.0, 0.0}, gl[3] = {0.0, 0.0, 0.0}, wt[3] = {0.0, 0.0, 0.0};
        if (!edge) {
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            if (i == rest<Q>()) continue;
            const uint32_t m =
                node + off(0, cx(i)) + off(1, cy(i)) + (Q == 27 ? off(2, cz<Q>(i)) : 0u);
            const double vp = (double)fld[N + m];
            const double vl = (double)fld[2 * N + m];
            const double w = weight<Q>(i);
#pragma unroll
            for (int a = 0; a < D; ++a) {
              const int ca = comp<Q>(i, a);
              if (ca == 0) continue;
              gp[a] += w * ca * vp;
              gl[a] += w * ca * vl;
            }
          }
        } else {
#pragma unroll 1
          for (int i = 0; i < Q; ++i) {
            const int c0 = i % 3 - 1, c1 = (i / 3) % 3 - 1, c2 = Q == 27 ? i / 9 - 1 : 0;
            if (c0 == 0 && c1 == 0 && c2 == 0) continue;
            uint32_t m = node;
            const bool f = resolve_nb(I, c.x, c.y, c.z, c0, c1, c2, m) && !(fl[m] & FLAG_SOLID);
            if (!f) m = node;
            const double vp = (double)fld[N + m];
            const double vl = (double)fld[2 * N + m];
            const double w = w1d(c0) * w1d(c1) * (Q == 27 ? w1d(c2) : 1.0);
            const int cc[3] = {c0, c1, c2};
            for (int a = 0; a < D; ++a) {
              gp[a] += w * cc[a] * vp;
              gl[a] += w * cc[a] * vl;
              if (!f) wt[a] += w * cc[a];
            }
          }
        }
#pragma unroll
        for (int a = 0; a < D; ++a)
          F[a] = 2.0 * p0 * (3.0 * gp[a]) + I.mp_kappa * rho0 * (3.0 * gl[a]) +
                 I.mp_kappa_w * rho0 * wt[a];
      }
      // ---- forced collision (FP64) ---------------------------------------------
      // The state in its storage type (FP32 or FP64; multiphase needs one of
      // the two), in place; the arithmetic in FP64.
      float g;
      if (!collide_forced<Q, T>(db + node, stride, F, I.beta, I.collision, I.trace_in_s, g)) {
        atomicOr(b.err, 1u);
        continue;
      }
      gmin = fminf(gmin, g);
      gmax = fmaxf(gmax, g);
      gsum += g;
      cnt += 1;
    }
  }
  if (b.stats) block_stats<256>(gmin, gmax, gsum, cnt, cnt, b.stats + ti);
}

// ---------------------------------------------------------------------------
// Initialisation, checkpoint encode/decode, moments.
// ---------------------------------------------------------------------------
template <int Q, int ST>
__global__ void k_init_eq(const InstDev* __restrict__ insts, int inst, int64_t N,
                          const double* __restrict__ rho, const double* __restrict__ u, void* buf) {
  using S = Store<ST>;
  using T = typename S::T;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const InstDev& I = insts[inst];
  const double uu[3] = {u[n], u[N + n], dims<Q>() == 3 ? u[2 * N + n] : 0.0};
  double fe[Q];
  feq_dev<Q, double>(rho[n] - 1.0, uu, fe);
  T* db = static_cast<T*>(buf) + I.pop_off;
#pragma unroll
  for (int i = 0; i < Q; ++i) db[i * I.stride + n] = S::enc_d(fe[i]);
}

template <int Q, int ST>
__global__ void k_decode(const InstDev* __restrict__ insts, int inst, int64_t N, const void* buf,
                         double* __restrict__ f) {
  using S = Store<ST>;
  using T = typename S::T;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const InstDev& I = insts[inst];
  const T* sb = static_cast<const T*>(buf) + I.pop_off;
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i * N + n] = weight<Q>(i) + (double)S::dec(sb[i * I.stride + n]);
}

// Populations of the box [lo, lo + ext) of one instance (box-local node
// order x-fastest, population-major, full f_i in FP64); lo may be negative or
// lo + ext exceed the size along periodic axes (wrapped once; the host
// checks that).
template <int Q, int ST>
__global__ void k_decode_box(const InstDev* __restrict__ insts, int inst, int3 lo, int3 ext,
                             const void* buf, double* __restrict__ f) {
  using S = Store<ST>;
  using T = typename S::T;
  const int64_t Nb = (int64_t)ext.x * ext.y * ext.z;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= Nb) return;
  const InstDev& I = insts[inst];
  const int lx = (int)(n % ext.x), ly = (int)((n / ext.x) % ext.y), lz = (int)(n / ((int64_t)ext.x * ext.y));
  int x = lo.x + lx, y = lo.y + ly, z = lo.z + lz;
  x += x < 0 ? I.nx : (x >= I.nx ? -I.nx : 0);
  y += y < 0 ? I.ny : (y >= I.ny ? -I.ny : 0);
  z += z < 0 ? I.nz : (z >= I.nz ? -I.nz : 0);
  const T* sb = static_cast<const T*>(buf) + I.pop_off;
  const uint32_t m = node_index(I, x, y, z);
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i * Nb + n] = weight<Q>(i) + (double)S::dec(sb[i * I.stride + m]);
}

template <int Q, int ST>
__global__ void k_encode(const InstDev* __restrict__ insts, int inst, int64_t N,
                         const double* __restrict__ f, void* buf) {
  using S = Store<ST>;
  using T = typename S::T;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const InstDev& I = insts[inst];
  T* db = static_cast<T*>(buf) + I.pop_off;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    db[i * I.stride + n] = S::enc_d(f[i * N + n] - weight<Q>(i));
}

template <int BLOCK, int W>
__device__ void block_sum_doubles(double (&v)[W], double* out) {
  for (int off = 32; off > 0; off >>= 1)
    for (int k = 0; k < W; ++k) v[k] += __shfl_xor(v[k], off);
  constexpr int NW = BLOCK / 64;
  __shared__ double sh[NW][W];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < W; ++k) sh[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < W; ++k) {
      double s = 0.0;
      for (int j = 0; j < NW; ++j) s += sh[j][k];
      out[k] = s;
    }
}

template <int Q, int ST>
__global__ void __launch_bounds__(256) k_moments(const InstDev* __restrict__ insts, int inst,
                                                 int64_t N, const void* buf,
                                                 const uint8_t* flags, double* rho, double* u,
                                                 double* partials) {
  using S = Store<ST>;
  using T = typename S::T;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const InstDev& I = insts[inst];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (n < N) {
    const T* sb = static_cast<const T*>(buf) + I.pop_off;
    const bool solid = I.flag_off >= 0 && (flags[I.flag_off + n] & FLAG_SOLID);
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    if (!solid) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double d = (double)S::dec(sb[i * I.stride + n]);
        r += d;
        j[0] += cx(i) * d;
        j[1] += cy(i) * d;
        j[2] += cz<Q>(i) * d;
      }
      r += 1.0;
    }
    const double ir = solid ? 0.0 : 1.0 / r;
    if (rho) rho[n] = r;
    if (u)
      for (int a = 0; a < dims<Q>(); ++a) u[a * N + n] = j[a] * ir;
    acc[0] = r;
    acc[1] = j[0];
    acc[2] = j[1];
    acc[3] = j[2];
  }
  block_sum_doubles<256, 4>(acc, partials + 4 * blockIdx.x);
}

// ---------------------------------------------------------------------------
// Wall force (Sec. II.C.2).
// ---------------------------------------------------------------------------
// Pre-collision stress sigma = -p I - (1 - beta) Pi^(1) of node m in FP64
// (Sec. II.C.2), Pi^(1) = sum_i (f_i - f^eq_i) c_i c_i, from the state the
// last step streamed (sb) with the same boundary fill.  Order xx, yy, zz,
// xy, xz, yz.
template <int Q, int ST>
__device__ void node_stress(const InstDev& I, const typename Store<ST>::T* sb, const uint8_t* fl,
                            uint32_t m, double t, double (&sig)[6]) {
  const Coord c = node_coord(I, m);
  double f[Q];
  gather_pre<Q, ST, double>(I, sb, fl, c.x, c.y, c.z, t, f);
  double rt, j[3];
  moments_dev<Q>(f, rt, j);
  const double rho = 1.0 + rt;
  const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  double fe[Q];
  feq_dev<Q, double>(rt, u, fe);
  double P[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double dl = f[i] - fe[i];
    P[0] += (double)(cx(i) * cx(i)) * dl;
    P[1] += (double)(cy(i) * cy(i)) * dl;
    P[2] += (double)(cz<Q>(i) * cz<Q>(i)) * dl;
    P[3] += (double)(cx(i) * cy(i)) * dl;
    P[4] += (double)(cx(i) * cz<Q>(i)) * dl;
    P[5] += (double)(cy(i) * cz<Q>(i)) * dl;
  }
  const double k = 1.0 - I.beta, p = rho / 3.0;
  for (int e = 0; e < 6; ++e) sig[e] = -k * P[e] - (e < 3 ? p : 0.0);
  if (dims<Q>() == 2) sig[2] = sig[4] = sig[5] = 0.0;
}

// Probe stress when no stencil corner of the probe p is fluid: the nearest
// fluid node in the 5^D box around floor(p) (Euclidean distance, first in z,
// y, x order on ties).  Returns false if the box holds no fluid node.
template <int Q, int ST>
__device__ bool nearest_fluid_stress(const InstDev& I, const typename Store<ST>::T* sb,
                                     const uint8_t* fl, const double (&p)[3], double t,
                                     double (&sig)[6]) {
  constexpr int D = dims<Q>();
  int base[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) base[a] = (int)floor(p[a]);
  double best = 1e300;
  int64_t bestm = -1;
  const int zr = D == 3 ? 2 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        uint32_t m;
        if (!resolve_nb(I, base[0], base[1], base[2], dx, dy, dz, m)) continue;
        if (fl && (fl[m] & FLAG_SOLID)) continue;
        const double q[3] = {(double)(base[0] + dx), (double)(base[1] + dy), (double)(base[2] + dz)};
        double r2 = 0.0;
        for (int a = 0; a < D; ++a) r2 += (q[a] - p[a]) * (q[a] - p[a]);
        if (r2 < best) {
          best = r2;
          bestm = m;
        }
      }
  if (bestm < 0) {
    for (int e = 0; e < 6; ++e) sig[e] = 0.0;
    return false;
  }
  node_stress<Q, ST>(I, sb, fl, (uint32_t)bestm, t, sig);
  return true;
}

// Wall force (Sec. II.C.2).  For quadrature point q the stress is sampled at
// the probes p_k = x_q + k n_q (k = 1, 2): multilinear over the 2^D stencil
// corners that are fluid, weights renormalised, else the nearest fluid node
// (nearest_fluid_stress); sigma_q = 2 sigma(p_1) - sigma(p_2), t_q = sigma_q
// n_q, and the workgroup's partial sum of w_q t_q.  One lane per (point,
// probe, corner): each reconstructs one node's pre-collision stress, so the
// 2 * 2^D reconstructions of a point run in parallel; lane 0 of the point
// sums its corners in corner order and forms the traction.  64 / (2 * 2^D)
// points per workgroup.  partials[4 * block] = (sum w t, count of probes
// that found no fluid node).
template <int Q, int ST>
__global__ void __launch_bounds__(64) k_force(const InstDev* __restrict__ insts, int inst,
                                              const void* prev, const uint8_t* flags,
                                              const int64_t* clock, const double* xq,
                                              const double* nq, const double* wq, int nqp,
                                              double* traction, double* partials) {
  constexpr int D = dims<Q>();
  constexpr int NC = 1 << D;    // stencil corners of a probe
  constexpr int SL = 2 * NC;    // lanes per point
  constexpr int PPW = 64 / SL;  // points per workgroup
  __shared__ double s_sig[64][6];
  __shared__ double s_w[64];
  const InstDev& I = insts[inst];
  const typename Store<ST>::T* sb = static_cast<const typename Store<ST>::T*>(prev) + I.pop_off;
  const uint8_t* fl = I.flag_off >= 0 ? flags + I.flag_off : nullptr;
  const double t = (double)(*clock);
  const int lane = threadIdx.x, slot = lane % SL;
  const int q = blockIdx.x * PPW + lane / SL;
  const int k = slot / NC, corner = slot % NC;
  double sig[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double w = 0.0;
  double nv[3] = {0.0, 0.0, 0.0}, p[3] = {0.0, 0.0, 0.0};
  if (q < nqp) {
    for (int a = 0; a < D; ++a) {
      nv[a] = nq[q * D + a];
      p[a] = xq[q * D + a] + (k + 1) * nv[a];
    }
    int base[3] = {0, 0, 0}, off[3] = {0, 0, 0};
    w = 1.0;
    for (int a = 0; a < D; ++a) {
      base[a] = (int)floor(p[a]);
      const double fr = p[a] - base[a];
      off[a] = (corner >> a) & 1;
      w *= off[a] ? fr : 1.0 - fr;
    }
    uint32_t m;
    if (w > 0.0 && resolve_nb(I, base[0], base[1], base[2], off[0], off[1], off[2], m) &&
        !(fl && (fl[m] & FLAG_SOLID))) {
      node_stress<Q, ST>(I, sb, fl, m, t, sig);
      for (int e = 0; e < 6; ++e) sig[e] *= w;
    } else {
      w = 0.0;
    }
  }
  for (int e = 0; e < 6; ++e) s_sig[lane][e] = sig[e];
  s_w[lane] = w;
  __syncthreads();
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (slot == 0 && q < nqp) {
    double S[2][6];
    int missing = 0;
    for (int kk = 0; kk < 2; ++kk) {
      double a6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, wsum = 0.0;
      for (int cc = 0; cc < NC; ++cc) {
        const int l = lane + kk * NC + cc;
        if (s_w[l] <= 0.0) continue;
        for (int e = 0; e < 6; ++e) a6[e] += s_sig[l][e];
        wsum += s_w[l];
      }
      if (wsum > 0.0) {
        for (int e = 0; e < 6; ++e) S[kk][e] = a6[e] / wsum;
      } else {
        double pk[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < D; ++a) pk[a] = xq[q * D + a] + (kk + 1) * nv[a];
        if (!nearest_fluid_stress<Q, ST>(I, sb, fl, pk, t, S[kk])) ++missing;
      }
    }
    const int ix[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    for (int a = 0; a < D; ++a) {
      double ta = 0.0;
      for (int c = 0; c < D; ++c) ta += (2.0 * S[0][ix[a][c]] - S[1][ix[a][c]]) * nv[c];
      if (traction) traction[q * D + a] = ta;
      acc[a] = wq[q] * ta;
    }
    acc[3] = (double)missing;
  }
  block_sum_doubles<64, 4>(acc, partials + 4 * blockIdx.x);
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_reduce(const double* partials, int n, int width,
                                                double* out) {
  // Fixed order: thread t sums partials t, t+256, ... sequentially, then a
  // fixed tree over the threads.
  __shared__ double sh[256];
  for (int k = 0; k < width; ++k) {
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) s += partials[(int64_t)j * width + k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
    __syncthreads();
  }
}

__global__ void k_reduce_stats(const StatPartial* parts, int n, StatPartial* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  StatPartial r{1e30f, -1e30f, 0.0, 0u, 0u};
  for (int j = 0; j < n; ++j) {
    const StatPartial p = parts[j];
    if (p.count == 0) continue;
    r.gmin = fminf(r.gmin, p.gmin);
    r.gmax = fmaxf(r.gmax, p.gmax);
    r.gsum += p.gsum;
    r.count += p.count;
    r.fp64 += p.fp64;
  }
  *out = r;
}

// ---------------------------------------------------------------------------
// Launchers and variant table
// ---------------------------------------------------------------------------
struct BulkVariant {
  const char* name;
  int block, tile, waves, mem;
};

// Workgroup size, nodes per tile (a workgroup loops over its tile), minimum
// waves per SIMD requested from the register allocator, non-temporal access.
static const BulkVariant kVariants[] = {
    {"b256_t256_w1", 256, 256, 1, 0},         {"b256_t512_w1", 256, 512, 1, 0},
    {"b128_t128_w1", 128, 128, 1, 0},         {"b512_t512_w1", 512, 512, 1, 0},
    {"b256_t256_w2", 256, 256, 2, 0},         {"b256_t1024_w2", 256, 1024, 2, 0},
    {"b512_t512_w1_nts", 512, 512, 1, 1},     {"b256_t256_w2_nts", 256, 256, 2, 1},
    {"b256_t1024_w2_nts", 256, 1024, 2, 1},   {"b512_t512_w1_ntls", 512, 512, 1, 3},
    {"b256_t1024_w2_ntls", 256, 1024, 2, 3},  {"b512_t512_w1_nts_o32", 512, 512, 1, 5},
    {"b256_t256_w2_nts_o32", 256, 256, 2, 5}, {"b256_t1024_w2_nts_o32", 256, 1024, 2, 5},
    {"b256_t256_w1_o32", 256, 256, 1, 4},     {"b512_t512_w1_buf", 512, 512, 1, 12},
    {"b512_t512_w1_nts_buf", 512, 512, 1, 13}, {"b256_t256_w2_nts_buf", 256, 256, 2, 13},
    {"b256_t1024_w2_nts_buf", 256, 1024, 2, 13},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int bulk_variant_count() { return kNumVariants; }
const char* bulk_variant_name(int v) { return (v >= 0 && v < kNumVariants) ? kVariants[v].name : "?"; }
int bulk_variant_tile(int v) { return kVariants[(v >= 0 && v < kNumVariants) ? v : 0].tile; }
bool bulk_variant_off32(int v) { return (kVariants[(v >= 0 && v < kNumVariants) ? v : 0].mem & 4) != 0; }

template <int Q, int ST, int BLOCK, int WAVES, int MEM>
static hipError_t launch_bulk_v(const StepBuffers& b, const Tile* tiles, int tile0, int ntiles,
                                bool faces, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (b.stats) {
    if (faces)
      hipLaunchKernelGGL((k_bulk<Q, ST, BLOCK, WAVES, MEM, true, true>), dim3(ntiles), dim3(BLOCK),
                         0, s, b, tiles, tile0);
    else
      hipLaunchKernelGGL((k_bulk<Q, ST, BLOCK, WAVES, MEM, true, false>), dim3(ntiles),
                         dim3(BLOCK), 0, s, b, tiles, tile0);
  } else {
    if (faces)
      hipLaunchKernelGGL((k_bulk<Q, ST, BLOCK, WAVES, MEM, false, true>), dim3(ntiles),
                         dim3(BLOCK), 0, s, b, tiles, tile0);
    else
      hipLaunchKernelGGL((k_bulk<Q, ST, BLOCK, WAVES, MEM, false, false>), dim3(ntiles),
                         dim3(BLOCK), 0, s, b, tiles, tile0);
  }
  return hipGetLastError();
}

template <int Q, int ST>
static hipError_t launch_bulk(int v, const StepBuffers& b, const Tile* tiles, int tile0,
                              int ntiles, bool faces, hipStream_t s) {
  switch (v) {
    case 1: return launch_bulk_v<Q, ST, 256, 1, 0>(b, tiles, tile0, ntiles, faces, s);
    case 2: return launch_bulk_v<Q, ST, 128, 1, 0>(b, tiles, tile0, ntiles, faces, s);
    case 3: return launch_bulk_v<Q, ST, 512, 1, 0>(b, tiles, tile0, ntiles, faces, s);
    case 4: return launch_bulk_v<Q, ST, 256, 2, 0>(b, tiles, tile0, ntiles, faces, s);
    case 5: return launch_bulk_v<Q, ST, 256, 2, 0>(b, tiles, tile0, ntiles, faces, s);
    case 6: return launch_bulk_v<Q, ST, 512, 1, 1>(b, tiles, tile0, ntiles, faces, s);
    case 7: return launch_bulk_v<Q, ST, 256, 2, 1>(b, tiles, tile0, ntiles, faces, s);
    case 8: return launch_bulk_v<Q, ST, 256, 2, 1>(b, tiles, tile0, ntiles, faces, s);
    case 9: return launch_bulk_v<Q, ST, 512, 1, 3>(b, tiles, tile0, ntiles, faces, s);
    case 10: return launch_bulk_v<Q, ST, 256, 2, 3>(b, tiles, tile0, ntiles, faces, s);
    case 11: return launch_bulk_v<Q, ST, 512, 1, 5>(b, tiles, tile0, ntiles, faces, s);
    case 12: return launch_bulk_v<Q, ST, 256, 2, 5>(b, tiles, tile0, ntiles, faces, s);
    case 13: return launch_bulk_v<Q, ST, 256, 2, 5>(b, tiles, tile0, ntiles, faces, s);
    case 14: return launch_bulk_v<Q, ST, 256, 1, 4>(b, tiles, tile0, ntiles, faces, s);
    case 15: return launch_bulk_v<Q, ST, 512, 1, 12>(b, tiles, tile0, ntiles, faces, s);
    case 16: return launch_bulk_v<Q, ST, 512, 1, 13>(b, tiles, tile0, ntiles, faces, s);
    case 17: return launch_bulk_v<Q, ST, 256, 2, 13>(b, tiles, tile0, ntiles, faces, s);
    case 18: return launch_bulk_v<Q, ST, 256, 2, 13>(b, tiles, tile0, ntiles, faces, s);
    default: return launch_bulk_v<Q, ST, 256, 1, 0>(b, tiles, tile0, ntiles, faces, s);
  }
}

template <int Q, int ST>
static hipError_t launch_boundary(const StepBuffers& b, const Region* regions,
                                  const BoxTile* btiles, int bt0, int nbt, uint2* list,
                                  uint32_t cap, uint32_t* count, int nwg, int nwall, int stat0,
                                  bool pre, hipStream_t s) {
  if (nbt <= 0 || (nwg <= 0 && nwall <= 0)) return hipSuccess;
  hipLaunchKernelGGL((k_boundary_scan<Q>), dim3(nbt), dim3(256), 0, s, b.insts, regions, btiles,
                     bt0, b.flags, list, cap, count);
  if (Q == 9 && nwg > 0 && nwall > 0) {
    if (pre)
      hipLaunchKernelGGL((k_boundary_both<Q, ST, true>), dim3(nwg + nwall), dim3(64), 0, s, b, list,
                         count, cap, stat0, (uint32_t)nwg);
    else
      hipLaunchKernelGGL((k_boundary_both<Q, ST, false>), dim3(nwg + nwall), dim3(64), 0, s, b,
                         list, count, cap, stat0, (uint32_t)nwg);
    return hipGetLastError();
  }
  if (nwg > 0) {
    if (pre)
      hipLaunchKernelGGL((k_boundary_wave<Q, ST, true>), dim3(nwg), dim3(64), 0, s, b, list,
                         count, cap, stat0);
    else
      hipLaunchKernelGGL((k_boundary_wave<Q, ST, false>), dim3(nwg), dim3(64), 0, s, b, list,
                         count, cap, stat0);
  }
  if (nwall > 0) {
    if (pre)
      hipLaunchKernelGGL((k_boundary_wall<Q, ST, true>), dim3(nwall), dim3(64), 0, s, b,
                         list + cap, count + 1, cap, stat0 + nwg);
    else
      hipLaunchKernelGGL((k_boundary_wall<Q, ST, false>), dim3(nwall), dim3(64), 0, s, b,
                         list + cap, count + 1, cap, stat0 + nwg);
  }
  return hipGetLastError();
}

template <int Q, int ST>
static hipError_t launch_mp(int stage, const StepBuffers& b, const Tile* tiles, int tile0,
                            int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (stage == 0)
    hipLaunchKernelGGL((k_mp_stream<Q, ST>), dim3(ntiles), dim3(256), 0, s, b, tiles, tile0);
  else if (stage == 1)
    hipLaunchKernelGGL((k_mp_lap<Q, ST>), dim3(ntiles), dim3(256), 0, s, b, tiles, tile0);
  else
    hipLaunchKernelGGL((k_mp_collide<Q, ST>), dim3(ntiles), dim3(256), 0, s, b, tiles, tile0);
  return hipGetLastError();
}

int boundary_nodes_per_workgroup(int Q) { return Q == 27 ? 1 : 2; }

int force_points_per_workgroup(int Q) { return Q == 27 ? 4 : 8; }

template <int Q, int ST>
static hipError_t launch_geometry(int stage, const InstDev* insts, const Region* regions,
                                  const BoxTile* gtiles, int ngt, void* src, uint8_t* flags,
                                  const int64_t* clock, int toff, hipStream_t s) {
  if (ngt <= 0) return hipSuccess;
  if (stage == 1) return hipSuccess;   // the fresh-node refill runs in stage 0
  hipLaunchKernelGGL((k_geometry<Q, ST>), dim3(ngt), dim3(256), 0, s, stage, insts, regions,
                     gtiles, src, flags, clock, toff);
  return hipGetLastError();
}

static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

template <int Q, int ST>
static hipError_t launch_init(const InstDev* insts, int inst, int64_t N, const double* rho,
                              const double* u, void* buf, hipStream_t s) {
  hipLaunchKernelGGL((k_init_eq<Q, ST>), dim3(grid_for(N, 256)), dim3(256), 0, s, insts, inst, N,
                     rho, u, buf);
  return hipGetLastError();
}

template <int Q, int ST>
static hipError_t launch_decode(const InstDev* insts, int inst, int64_t N, const void* buf,
                                double* f, hipStream_t s) {
  hipLaunchKernelGGL((k_decode<Q, ST>), dim3(grid_for(N, 256)), dim3(256), 0, s, insts, inst, N,
                     buf, f);
  return hipGetLastError();
}

template <int Q, int ST>
static hipError_t launch_decode_box(const InstDev* insts, int inst, const int* lo, const int* ext,
                                    const void* buf, double* f, hipStream_t s) {
  const int64_t Nb = (int64_t)ext[0] * ext[1] * ext[2];
  hipLaunchKernelGGL((k_decode_box<Q, ST>), dim3(grid_for(Nb, 256)), dim3(256), 0, s, insts, inst,
                     make_int3(lo[0], lo[1], lo[2]), make_int3(ext[0], ext[1], ext[2]), buf, f);
  return hipGetLastError();
}

template <int Q, int ST>
static hipError_t launch_encode(const InstDev* insts, int inst, int64_t N, const double* f,
                                void* buf, hipStream_t s) {
  hipLaunchKernelGGL((k_encode<Q, ST>), dim3(grid_for(N, 256)), dim3(256), 0, s, insts, inst, N,
                     f, buf);
  return hipGetLastError();
}

template <int Q, int ST>
static hipError_t launch_moments(const InstDev* insts, int inst, int64_t N, const void* buf,
                                 const uint8_t* flags, double* rho, double* u, double* partials,
                                 int* nparts, hipStream_t s) {
  const unsigned g = grid_for(N, 256);
  *nparts = (int)g;
  hipLaunchKernelGGL((k_moments<Q, ST>), dim3(g), dim3(256), 0, s, insts, inst, N, buf, flags,
                     rho, u, partials);
  return hipGetLastError();
}

template <int Q, int ST>
static hipError_t launch_force(const InstDev* insts, int inst, const void* prev,
                               const uint8_t* flags, const int64_t* clock, const double* xq,
                               const double* nq, const double* wq, int nqp, double* traction,
                               double* partials, int* nparts, hipStream_t s) {
  const unsigned g = (unsigned)((nqp + force_points_per_workgroup(Q) - 1) /
                                force_points_per_workgroup(Q));
  *nparts = (int)g;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL((k_force<Q, ST>), dim3(g), dim3(64), 0, s, insts, inst, prev, flags, clock,
                     xq, nq, wq, nqp, traction, partials);
  return hipGetLastError();
}

template <int Q, int ST>
static hipError_t launch_fixup(const StepBuffers& b, int nblocks, int stat0, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_neq_fixup<Q, ST>), dim3(nblocks), dim3(256), 0, s, b, stat0);
  return hipGetLastError();
}

template <int Q, int ST>
static const Ops* ops_for() {
  static const Ops o = {launch_bulk<Q, ST>,    launch_boundary<Q, ST>, launch_geometry<Q, ST>,
                        launch_init<Q, ST>,    launch_decode<Q, ST>,   launch_encode<Q, ST>,
                        launch_moments<Q, ST>, launch_fixup<Q, ST>,    launch_force<Q, ST>,
                        launch_decode_box<Q, ST>, launch_mp<Q, ST>};
  return &o;
}

const Ops* get_ops(int Q, int storage) {
  if (Q == 9) {
    switch (storage) {
      case LBM_F64: return ops_for<9, LBM_F64>();
      case LBM_F32: return ops_for<9, LBM_F32>();
      case LBM_F16_SHIFTED: return ops_for<9, LBM_F16_SHIFTED>();
      case LBM_BF16_SHIFTED: return ops_for<9, LBM_BF16_SHIFTED>();
    }
  } else if (Q == 27) {
    switch (storage) {
      case LBM_F64: return ops_for<27, LBM_F64>();
      case LBM_F32: return ops_for<27, LBM_F32>();
      case LBM_F16_SHIFTED: return ops_for<27, LBM_F16_SHIFTED>();
      case LBM_BF16_SHIFTED: return ops_for<27, LBM_BF16_SHIFTED>();
    }
  }
  return nullptr;
}

hipError_t launch_reduce(const double* partials, int n, int width, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, n, width, out);
  return hipGetLastError();
}

hipError_t launch_reduce_stats(const StatPartial* parts, int n, StatPartial* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(64), 0, s, parts, n, out);
  return hipGetLastError();
}

}  // namespace kbc
