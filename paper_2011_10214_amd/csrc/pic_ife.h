// Immersed finite elements on the PIC mesh (the paper's discretisation of the
// object's interface, §2.3; §3.1.1: every cubic PIC cell is cut into five
// tetrahedra). Host and device code: the library's host side evaluates the
// stencil of an interior node with the same functions the assembly kernel
// uses, so both give the same bits.
//
// The elements:
//   * cube corners are numbered c = a + 2b + 4c for the offset (a, b, c); a
//     cube of parity p = (i + j + k) mod 2 has the central tetrahedron on its
//     four corners whose offset parity is p, and for each of the other four
//     corners the tetrahedron of that corner and its three axis neighbours
//     (c ^ 1, c ^ 2, c ^ 4), so that the face diagonals of neighbouring cubes
//     coincide (all of them join nodes of even global parity);
//   * the interface in a tetrahedron is the plane where the linear
//     interpolant psi_h of the level set's vertex values vanishes; the part
//     with psi_h < 0 is inside the object (eps_in), the rest outside (eps_out);
//     a tetrahedron with vertex values of both signs (psi < 0 against
//     psi >= 0) is cut;
//   * in a cut tetrahedron a basis function is linear on each side, equal on
//     the plane, and eps grad phi . n is the same on both sides: with
//     g = grad psi_h, phi_out = phi_in + tau psi_h and
//     tau = (eps_in / eps_out - 1) (grad phi_in . g) / |g|^2;
//   * element matrix K_ij = eps_in V_in grad phi_i,in . grad phi_j,in
//     + eps_out V_out grad phi_i,out . grad phi_j,out (upper triangle,
//     mirrored); an uncut tetrahedron gives eps times the linear element's
//     matrix V grad lambda_i . grad lambda_j.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// Links of a node in the five-tetrahedra mesh: the 6 axis neighbours, then
// the 12 face diagonals.
constexpr int kIfeLinks = 18;
__host__ __device__ inline void ife_link_offset(int l, int o[3]) {
  const int8_t t[kIfeLinks][3] = {{-1, 0, 0},  {1, 0, 0},  {0, -1, 0}, {0, 1, 0},
                                  {0, 0, -1},  {0, 0, 1},  {-1, -1, 0}, {1, -1, 0},
                                  {-1, 1, 0},  {1, 1, 0},  {-1, 0, -1}, {1, 0, -1},
                                  {-1, 0, 1},  {1, 0, 1},  {0, -1, -1}, {0, 1, -1},
                                  {0, -1, 1},  {0, 1, 1}};
  o[0] = t[l][0];
  o[1] = t[l][1];
  o[2] = t[l][2];
}

// Link index of an offset (each component in -1..1), or -1 (itself, or a
// body diagonal, which is no edge of the mesh).
__host__ __device__ inline int ife_link_of(int dx, int dy, int dz) {
  const int nz = (dx != 0) + (dy != 0) + (dz != 0);
  if (nz == 1) return dx ? (dx < 0 ? 0 : 1) : dy ? (dy < 0 ? 2 : 3) : (dz < 0 ? 4 : 5);
  if (nz != 2) return -1;
  if (dz == 0) return 6 + (dx > 0) + 2 * (dy > 0);
  if (dy == 0) return 10 + (dx > 0) + 2 * (dz > 0);
  return 14 + (dy > 0) + 2 * (dz > 0);
}

// The four corners of tetrahedron t (0: central, 1..4: corner tetrahedra in
// increasing order of their lone corner) of a cube of parity p.
__host__ __device__ inline void ife_tet(int p, int t, int v[4]) {
  // corners of offset parity 0: 0, 3, 5, 6; of parity 1: 1, 2, 4, 7
  const int8_t par[2][4] = {{0, 3, 5, 6}, {1, 2, 4, 7}};
  if (t == 0) {
    for (int r = 0; r < 4; ++r) v[r] = par[p][r];
    return;
  }
  const int lone = par[1 - p][t - 1];
  v[0] = lone;
  v[1] = lone ^ 1;
  v[2] = lone ^ 2;
  v[3] = lone ^ 4;
}

__host__ __device__ inline void ife_corner_xyz(int c, double x[3]) {
  x[0] = (double)(c & 1);
  x[1] = (double)((c >> 1) & 1);
  x[2] = (double)((c >> 2) & 1);
}

// grad lambda_i = N / (N . (x_i - x_j)), N the normal of the face opposite
// vertex i (vertices j, k, l): lambda_i vanishes on that face and is 1 at x_i.
__host__ __device__ inline void ife_gradients(const double X[4][3], double G[4][3], double *vol) {
  for (int i = 0; i < 4; ++i) {
    const int j = (i + 1) & 3, k = (i + 2) & 3, l = (i + 3) & 3;
    double u[3], w[3], N[3];
    for (int d = 0; d < 3; ++d) {
      u[d] = X[k][d] - X[j][d];
      w[d] = X[l][d] - X[j][d];
    }
    N[0] = u[1] * w[2] - u[2] * w[1];
    N[1] = u[2] * w[0] - u[0] * w[2];
    N[2] = u[0] * w[1] - u[1] * w[0];
    const double h = N[0] * (X[i][0] - X[j][0]) + N[1] * (X[i][1] - X[j][1]) +
                     N[2] * (X[i][2] - X[j][2]);
    for (int d = 0; d < 3; ++d) G[i][d] = N[d] / h;
    if (i == 0) *vol = (h < 0.0 ? -h : h) / 6.0;
  }
}

__host__ __device__ inline double ife_tet_vol(const double *A, const double *B, const double *C,
                                              const double *D) {
  const double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  const double v[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
  const double w[3] = {D[0] - A[0], D[1] - A[1], D[2] - A[2]};
  const double t = u[0] * (v[1] * w[2] - v[2] * w[1]) + u[1] * (v[2] * w[0] - v[0] * w[2]) +
                   u[2] * (v[0] * w[1] - v[1] * w[0]);
  return (t < 0.0 ? -t : t) / 6.0;
}

// Volume of the part of the tetrahedron where psi_h < 0.
__host__ __device__ inline double ife_inside_volume(const double X[4][3], const double psi[4],
                                                    double vol) {
  int in[4], out[4], ni = 0, no = 0;
  for (int r = 0; r < 4; ++r) {
    if (psi[r] < 0.0) in[ni++] = r;
    else out[no++] = r;
  }
  if (no == 0) return vol;
  if (ni == 0) return 0.0;
  auto cross_pt = [&](int a, int b, double P[3]) {  // psi_h = 0 on the edge a-b
    const double t = psi[a] / (psi[a] - psi[b]);
    for (int d = 0; d < 3; ++d) P[d] = X[a][d] + t * (X[b][d] - X[a][d]);
  };
  if (ni == 1 || no == 1) {  // the corner at the lone vertex is a small tetrahedron
    const int lone = ni == 1 ? in[0] : out[0];
    const int *rest = ni == 1 ? out : in;
    double P0[3], P1[3], P2[3];
    cross_pt(lone, rest[0], P0);
    cross_pt(lone, rest[1], P1);
    cross_pt(lone, rest[2], P2);
    const double corner = ife_tet_vol(X[lone], P0, P1, P2);
    return ni == 1 ? corner : vol - corner;
  }
  // two inside (a, b), two outside (c, d): a prism; coned from a over its
  // faces that do not contain a
  const int a = in[0], b = in[1], c = out[0], d = out[1];
  double Pac[3], Pad[3], Pbc[3], Pbd[3];
  cross_pt(a, c, Pac);
  cross_pt(a, d, Pad);
  cross_pt(b, c, Pbc);
  cross_pt(b, d, Pbd);
  return ife_tet_vol(X[a], X[b], Pbc, Pbd) + ife_tet_vol(X[a], Pac, Pbc, Pbd) +
         ife_tet_vol(X[a], Pac, Pbd, Pad);
}

// Element matrix K (vertex order of X) of the IFE basis of a tetrahedron in
// the unit cells of the mesh.
__host__ __device__ inline void ife_element_matrix(const double X[4][3], const double psi[4],
                                                   double ein, double eout, double K[4][4]) {
  double G[4][3], vol;
  ife_gradients(X, G, &vol);
  bool has_in = false, has_out = false;
  for (int r = 0; r < 4; ++r) {
    if (psi[r] < 0.0) has_in = true;
    else has_out = true;
  }
  if (!(has_in && has_out)) {  // uncut: the linear element
    const double e = has_in ? ein : eout;
    for (int i = 0; i < 4; ++i)
      for (int j = i; j < 4; ++j) {
        const double gg = G[i][0] * G[j][0] + G[i][1] * G[j][1] + G[i][2] * G[j][2];
        K[i][j] = e * (vol * gg);
        K[j][i] = K[i][j];
      }
    return;
  }
  double g[3] = {0.0, 0.0, 0.0};
  for (int r = 0; r < 4; ++r)
    for (int d = 0; d < 3; ++d) g[d] += psi[r] * G[r][d];
  const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  const double kap = (ein / eout - 1.0) / g2;
  // vertex values v = c + tau d with d_r = psi_r outside, 0 inside, and
  // tau = kap (grad phi_in . g) = kap sum_r c_r wg_r, wg_r = grad lambda_r . g:
  // c = v - kap d (wg . v) / (1 + kap wg . d) (a rank-one inverse)
  double wg[4], dd[4], wd = 0.0;
  for (int r = 0; r < 4; ++r) {
    wg[r] = G[r][0] * g[0] + G[r][1] * g[1] + G[r][2] * g[2];
    dd[r] = psi[r] < 0.0 ? 0.0 : psi[r];
    wd += wg[r] * dd[r];
  }
  const double inv = 1.0 / (1.0 + kap * wd);
  double gin[4][3], gout[4][3];
  for (int i = 0; i < 4; ++i) {
    // basis function i: v = e_i, so wg . v = wg_i
    const double s = kap * wg[i] * inv;
    double tau_num = 0.0;
    for (int d = 0; d < 3; ++d) {
      double a = G[i][d];
      for (int r = 0; r < 4; ++r) a -= s * dd[r] * G[r][d];
      gin[i][d] = a;
      tau_num += a * g[d];
    }
    const double tau = kap * tau_num;
    for (int d = 0; d < 3; ++d) gout[i][d] = gin[i][d] + tau * g[d];
  }
  const double vin = ife_inside_volume(X, psi, vol), vout = vol - vin;
  for (int i = 0; i < 4; ++i)
    for (int j = i; j < 4; ++j) {
      const double ai = gin[i][0] * gin[j][0] + gin[i][1] * gin[j][1] + gin[i][2] * gin[j][2];
      const double ao = gout[i][0] * gout[j][0] + gout[i][1] * gout[j][1] + gout[i][2] * gout[j][2];
      K[i][j] = ein * vin * ai + eout * vout * ao;
      K[j][i] = K[i][j];
    }
}

// Element matrix of tetrahedron t of a cube of parity p whose corners have
// the level-set values cpsi[8] (the unit-cube vertex coordinates); the
// tetrahedron's corner numbers go to v.
__host__ __device__ inline void ife_cube_element(int p, int t, const double cpsi[8], double ein,
                                                 double eout, int v[4], double K[4][4]) {
  ife_tet(p, t, v);
  double X[4][3], ps[4];
  for (int r = 0; r < 4; ++r) {
    ife_corner_xyz(v[r], X[r]);
    ps[r] = cpsi[v[r]];
  }
  ife_element_matrix(X, ps, ein, eout, K);
}

// Link coefficients c_l = -A_pq (unit cells, eps = 1: the reference) of a
// node of parity par whose cubes all lie in the mesh, every tetrahedron
// uncut, summed over cubes in increasing global order and over tetrahedra
// in order (the order of the assembly kernel). rl[kIfeLinks].
__host__ __device__ inline void ife_reference_links(int par, double rl[kIfeLinks]) {
  for (int l = 0; l < kIfeLinks; ++l) rl[l] = 0.0;
  const double ones[8] = {1, 1, 1, 1, 1, 1, 1, 1};
  for (int dc = -1; dc <= 0; ++dc)
    for (int db = -1; db <= 0; ++db)
      for (int da = -1; da <= 0; ++da) {
        // the node is corner (-da, -db, -dc) of the cube; cube parity
        const int p = (par + da + db + dc) & 1;
        const int lp = -da - 2 * db - 4 * dc;
        for (int t = 0; t < 5; ++t) {
          int v[4];
          double K[4][4];
          ife_cube_element(p, t, ones, 1.0, 1.0, v, K);
          int rp = -1;
          for (int r = 0; r < 4; ++r)
            if (v[r] == lp) rp = r;
          if (rp < 0) continue;
          for (int r = 0; r < 4; ++r) {
            if (r == rp) continue;
            const int l = ife_link_of((v[r] & 1) - (lp & 1), ((v[r] >> 1) & 1) - ((lp >> 1) & 1),
                                      ((v[r] >> 2) & 1) - ((lp >> 2) & 1));
            rl[l] -= K[rp][r];
          }
        }
      }
}

}  // namespace pic
