// Q1 (trilinear hexahedron / bilinear quad) element integrals for the
// Galerkin form of the Helmholtz equation: stiffness int grad(phi_a).grad(phi_b),
// mass int phi_a phi_b, boundary-face mass int_face phi_a phi_b.
// 2-point Gauss-Legendre rule per axis (exact for Q1 on parallelepipeds).
// Used by the host assembly and by the device gradient kernels.
//
// Local node a of a hexahedron sits at reference corner
// (2 bit0(a) - 1, 2 bit1(a) - 1, 2 bit2(a) - 1); of a quad at
// (2 bit0(a) - 1, 2 bit1(a) - 1).
#pragma once

#include "common.h"

namespace q1 {

HD double corner_sign(int a, int d) { return double(2 * ((a >> d) & 1) - 1); }

// Shape values N[8] and reference gradients dN[8][3] at reference point p.
HD void hex_shape(const double p[3], double N[8], double dN[8][3]) {
  for (int a = 0; a < 8; ++a) {
    double f0 = 1.0 + corner_sign(a, 0) * p[0];
    double f1 = 1.0 + corner_sign(a, 1) * p[1];
    double f2 = 1.0 + corner_sign(a, 2) * p[2];
    N[a] = f0 * f1 * f2 * 0.125;
    dN[a][0] = corner_sign(a, 0) * f1 * f2 * 0.125;
    dN[a][1] = corner_sign(a, 1) * f0 * f2 * 0.125;
    dN[a][2] = corner_sign(a, 2) * f0 * f1 * 0.125;
  }
}

HD double gauss_point(int q) { return (q ? 1.0 : -1.0) * 0.57735026918962576451; }  // 1/sqrt(3)

// Physical gradients G[8][3] and |J| at Gauss point (qx, qy, qz).
HD void hex_point(const double X[8][3], int qx, int qy, int qz, double N[8], double G[8][3],
                  double* detJ) {
  double p[3] = {gauss_point(qx), gauss_point(qy), gauss_point(qz)};
  double dN[8][3];
  hex_shape(p, N, dN);
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // J[i][d] = dx_i / dxi_d
  for (int a = 0; a < 8; ++a)
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 3; ++d) J[i][d] += X[a][i] * dN[a][d];
  // inverse by cofactors: Jinv[d][i] = dxi_d / dx_i
  double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  double inv = 1.0 / det;
  double Ji[3][3];
  Ji[0][0] = c00 * inv;
  Ji[1][0] = c01 * inv;
  Ji[2][0] = c02 * inv;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * inv;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * inv;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * inv;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * inv;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * inv;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * inv;
  for (int a = 0; a < 8; ++a)
    for (int i = 0; i < 3; ++i)
      G[a][i] = dN[a][0] * Ji[0][i] + dN[a][1] * Ji[1][i] + dN[a][2] * Ji[2][i];
  *detJ = det;
}

// Row a of the element stiffness and mass matrices.  Entry (a,b) and (b,a)
// are formed from the same products in the same order, so assembling rows
// independently gives bitwise symmetric matrices.
HD void hex_rows(const double X[8][3], int a, double Krow[8], double Mrow[8]) {
  for (int b = 0; b < 8; ++b) Krow[b] = Mrow[b] = 0.0;
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        double N[8], G[8][3], dj;
        hex_point(X, qx, qy, qz, N, G, &dj);
        for (int b = 0; b < 8; ++b) {
          double gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
          Krow[b] += gg * dj;
          Mrow[b] += (N[a] * N[b]) * dj;
        }
      }
}

// Full element mass matrix (used by the absorption-field gradient).
HD void hex_mass(const double X[8][3], double Me[8][8]) {
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) Me[a][b] = 0.0;
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        double N[8], G[8][3], dj;
        hex_point(X, qx, qy, qz, N, G, &dj);
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b) Me[a][b] += (N[a] * N[b]) * dj;
      }
}

// Boundary-face mass of a bilinear quad embedded in 3-D (area element
// |dx/dxi x dx/deta|).
HD void quad_mass(const double X[4][3], double Fe[4][4]) {
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) Fe[a][b] = 0.0;
  for (int qy = 0; qy < 2; ++qy)
    for (int qx = 0; qx < 2; ++qx) {
      double p0 = gauss_point(qx), p1 = gauss_point(qy);
      double N[4], t0[3] = {0, 0, 0}, t1[3] = {0, 0, 0};
      for (int a = 0; a < 4; ++a) {
        double s0 = corner_sign(a, 0), s1 = corner_sign(a, 1);
        double f0 = 1.0 + s0 * p0, f1 = 1.0 + s1 * p1;
        N[a] = f0 * f1 * 0.25;
        for (int i = 0; i < 3; ++i) {
          t0[i] += X[a][i] * s0 * f1 * 0.25;
          t1[i] += X[a][i] * s1 * f0 * 0.25;
        }
      }
      double nx = t0[1] * t1[2] - t0[2] * t1[1];
      double ny = t0[2] * t1[0] - t0[0] * t1[2];
      double nz = t0[0] * t1[1] - t0[1] * t1[0];
      double area = sqrt(nx * nx + ny * ny + nz * nz);
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) Fe[a][b] += (N[a] * N[b]) * area;
    }
}

}  // namespace q1
