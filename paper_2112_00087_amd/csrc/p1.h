// P1 (linear tetrahedron / linear triangle) element integrals for the
// Galerkin form of the Helmholtz equation.  The shape functions are the
// barycentric coordinates l_a, whose gradients are constant on the element,
// so every integral is exact in closed form:
//   stiffness  int grad(l_a).grad(l_b) = V G_a . G_b
//   mass       int l_a l_b             = V (1 + delta_ab) / 20
//   face mass  int_face l_a l_b        = A (1 + delta_ab) / 12
// with V the volume, A the face area, and G_a the gradients: with the edge
// matrix D (columns x_a - x_0, a = 1..3) the gradients of l_1..l_3 are the
// rows of D^-1 and G_0 = -(G_1 + G_2 + G_3).
// Used by the host assembly and by the device gradient kernels.
#pragma once

#include "common.h"

namespace p1 {

// Barycentric gradients G[4][3] and volume of the tetrahedron X[4][3].
HD void tet_grad(const double X[4][3], double G[4][3], double* vol) {
  double D[3][3];   // D[i][c] = x_{c+1,i} - x_{0,i}
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) D[i][c] = X[c + 1][i] - X[0][i];
  const double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  const double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  const double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  const double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
  const double inv = 1.0 / det;
  // row c of D^-1 = gradient of l_{c+1}
  G[1][0] = c00 * inv;
  G[1][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * inv;
  G[1][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * inv;
  G[2][0] = c01 * inv;
  G[2][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * inv;
  G[2][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * inv;
  G[3][0] = c02 * inv;
  G[3][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * inv;
  G[3][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * inv;
  for (int i = 0; i < 3; ++i) G[0][i] = -((G[1][i] + G[2][i]) + G[3][i]);
  *vol = fabs(det) / 6.0;
}

// Row a of the element stiffness and mass matrices; entries (a,b) and (b,a)
// come from the same products in the same order (bitwise symmetric assembly).
HD void tet_rows(const double X[4][3], int a, double Krow[4], double Mrow[4]) {
  double G[4][3], vol;
  tet_grad(X, G, &vol);
  for (int b = 0; b < 4; ++b) {
    const double gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
    Krow[b] = gg * vol;
    Mrow[b] = (a == b ? 2.0 : 1.0) * (vol / 20.0);
  }
}

// Full element mass matrix (used by the absorption-field gradient).
HD void tet_mass(const double X[4][3], double Me[4][4]) {
  double G[4][3], vol;
  tet_grad(X, G, &vol);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) Me[a][b] = (a == b ? 2.0 : 1.0) * (vol / 20.0);
}

// Boundary-face mass of a triangle embedded in 3-D.
HD void tri_mass(const double X[3][3], double Fe[3][3]) {
  const double u0 = X[1][0] - X[0][0], u1 = X[1][1] - X[0][1], u2 = X[1][2] - X[0][2];
  const double v0 = X[2][0] - X[0][0], v1 = X[2][1] - X[0][1], v2 = X[2][2] - X[0][2];
  const double nx = u1 * v2 - u2 * v1, ny = u2 * v0 - u0 * v2, nz = u0 * v1 - u1 * v0;
  const double area = 0.5 * sqrt(nx * nx + ny * ny + nz * nz);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Fe[a][b] = (a == b ? 2.0 : 1.0) * (area / 12.0);
}

}  // namespace p1
