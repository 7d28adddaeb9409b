// Device-side FP64 3x3 linear algebra and the isotropic constitutive models
// of the implicit step (Sec. 4.3 of the paper), written for gfx950.
//
// Conventions: 3x3 matrices are row-major double[9]; symmetric 3x3 tensors
// are stored as 6 entries (xx, yy, zz, xy, yz, xz).
//
// Routes taken on the GPU:
//   * polar F = R S_F by Higham's scaled Newton iteration X <- (g X + X^{-T}/g)/2
//     (det F > 0; near the identity it converges in 3-4 steps);
//   * the principal frame F = U diag(s) V^T from the symmetric stretch
//     S_F = R^T F by cyclic Jacobi, U = R V;
//   * the projected tangent [dP/dF]_+ from the analytic eigensystem of an
//     isotropic energy in the principal frame: the 3x3 Hessian of psi_hat
//     (scaling modes) and, for each pair (i, j), the two modes
//     (E_ij + E_ji)/sqrt2 with eigenvalue (psi_i - psi_j)/(s_i - s_j) and
//     (E_ij - E_ji)/sqrt2 with eigenvalue (psi_i + psi_j)/(s_i + s_j),
//     each difference quotient written in a form that stays exact as s_i -> s_j.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#define MPL_DEV __host__ __device__ __forceinline__

namespace mpl {

// SplitMix64 (Steele, Lea and Flood 2014) of counter q: the state
// (q + 1) * golden gamma through the published finaliser (the multigrid
// power iterations draw their start signs from it).
MPL_DEV uint64_t splitmix64(uint64_t q) {
  uint64_t z = (q + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Two-level reduction of partial-sum arrays of up to nm entries: the number
// of workgroups (one per 256 entries, at most gmax) and the contiguous range
// [lo, hi) of entries that workgroup g of G sums.  The ranges of g = 0..G-1
// cover [0, nm) in order, each entry once.
MPL_DEV int red2_groups(int nm, int gmax) {
  const int g = (nm + 255) / 256;
  return g < 1 ? 1 : (g > gmax ? gmax : g);
}
MPL_DEV void red2_range(int g, int G, int nm, int& lo, int& hi) {
  const int chunk = (nm + G - 1) / G;
  const long long l = (long long)g * chunk;
  lo = l < nm ? (int)l : nm;
  hi = lo + chunk < nm ? lo + chunk : nm;
}

enum { NEOHOOKEAN = 0, FIXED_COROTATED = 1, HENCKY = 2, WATER = 3 };
enum { PLASTIC_NONE = 0, PLASTIC_VON_MISES = 1, PLASTIC_DRUCKER_PRAGER = 2 };

struct MatParams {
  int model, plastic;
  double mu, lambda, kappa;   // kappa: split Neo-Hookean 2 mu / 3 + lambda; water: the bulk modulus
  double yield_stress, alpha_f;
};

// ---------------------------------------------------------------- 3x3 basics
MPL_DEV void eye(double* A) {
#pragma unroll
  for (int i = 0; i < 9; ++i) A[i] = (i % 4 == 0) ? 1.0 : 0.0;
}
MPL_DEV void mul(const double* A, const double* B, double* C) {  // C = A B (C != A, B)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
}
MPL_DEV void mul_tn(const double* A, const double* B, double* C) {  // C = A^T B
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}
MPL_DEV void mul_nt(const double* A, const double* B, double* C) {  // C = A B^T
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = A[i * 3] * B[j * 3] + A[i * 3 + 1] * B[j * 3 + 1] + A[i * 3 + 2] * B[j * 3 + 2];
}
MPL_DEV double det(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}
// cof(A) = det(A) A^{-T}
// Inverse of the symmetric 3x3 matrix h = (xx, yy, zz, xy, yz, xz) by its
// adjugate over its determinant, same storage.  Returns false (and inv = 0)
// unless the determinant is finite and positive (h positive definite when
// also its leading 1x1 and 2x2 minors are, which a block of an SPD matrix
// satisfies).
MPL_DEV bool sym3_inverse(const double h[6], double inv[6]) {
  const double xx = h[0], yy = h[1], zz = h[2], xy = h[3], yz = h[4], xz = h[5];
  const double c00 = yy * zz - yz * yz, c11 = xx * zz - xz * xz, c22 = xx * yy - xy * xy;
  const double c01 = xz * yz - xy * zz, c12 = xy * xz - xx * yz, c02 = xy * yz - yy * xz;
  const double d = xx * c00 + xy * c01 + xz * c02;
  const bool ok = d > 0.0 && isfinite(d) && xx > 0.0 && c22 > 0.0;
  const double id = ok ? 1.0 / d : 0.0;
  inv[0] = ok ? c00 * id : 0.0;
  inv[1] = ok ? c11 * id : 0.0;
  inv[2] = ok ? c22 * id : 0.0;
  inv[3] = ok ? c01 * id : 0.0;
  inv[4] = ok ? c12 * id : 0.0;
  inv[5] = ok ? c02 * id : 0.0;
  return ok;
}

MPL_DEV void cofactor(const double* A, double* C) {
  C[0] = A[4] * A[8] - A[5] * A[7];
  C[1] = A[5] * A[6] - A[3] * A[8];
  C[2] = A[3] * A[7] - A[4] * A[6];
  C[3] = A[2] * A[7] - A[1] * A[8];
  C[4] = A[0] * A[8] - A[2] * A[6];
  C[5] = A[1] * A[6] - A[0] * A[7];
  C[6] = A[1] * A[5] - A[2] * A[4];
  C[7] = A[2] * A[3] - A[0] * A[5];
  C[8] = A[0] * A[4] - A[1] * A[3];
}
MPL_DEV double frob2(const double* A) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) s += A[i] * A[i];
  return s;
}
MPL_DEV void sym_to_full(const double* s, double* A) {
  A[0] = s[0]; A[4] = s[1]; A[8] = s[2];
  A[1] = A[3] = s[3];
  A[5] = A[7] = s[4];
  A[2] = A[6] = s[5];
}
MPL_DEV void full_to_sym(const double* A, double* s) {
  s[0] = A[0]; s[1] = A[4]; s[2] = A[8];
  s[3] = 0.5 * (A[1] + A[3]);
  s[4] = 0.5 * (A[5] + A[7]);
  s[5] = 0.5 * (A[2] + A[6]);
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi: A = Q diag(w) Q^T,
// columns of Q (row-major Q[r*3+c]) are the eigenvectors; det Q = +1.
MPL_DEV void jacobi_rotate(double (&a)[3][3], double (&q)[3][3], int p, int r) {
  double apr = a[p][r];
  if (apr == 0.0) return;
  double theta = (a[r][r] - a[p][p]) / (2.0 * apr);
  double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
  a[p][p] -= t * apr;
  a[r][r] += t * apr;
  a[p][r] = a[r][p] = 0.0;
  int o = 3 - p - r;
  double aop = a[o][p], aor = a[o][r];
  a[o][p] = a[p][o] = c * aop - s * aor;
  a[o][r] = a[r][o] = s * aop + c * aor;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double qp = q[k][p], qr = q[k][r];
    q[k][p] = c * qp - s * qr;
    q[k][r] = s * qp + c * qr;
  }
}
MPL_DEV void eig_sym3(const double* A, double* w, double* Q) {
  double a[3][3], q[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      a[i][j] = 0.5 * (A[i * 3 + j] + A[j * 3 + i]);
      q[i][j] = (i == j) ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off == 0.0 || off <= 1e-36 * dia) break;
    jacobi_rotate(a, q, 0, 1);
    jacobi_rotate(a, q, 0, 2);
    jacobi_rotate(a, q, 1, 2);
  }
  w[0] = a[0][0]; w[1] = a[1][1]; w[2] = a[2][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Q[i * 3 + j] = q[i][j];
}

// Rotation factor of F (det F > 0) by the scaled Newton iteration.  Returns
// false if det F <= 0 or the iteration did not settle.
MPL_DEV bool polar_rotation(const double* F, double* R) {
  double X[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) X[i] = F[i];
  if (!(det(F) > 0.0)) return false;
  bool scale = true;
  for (int it = 0; it < 40; ++it) {
    double C[9];
    cofactor(X, C);
    double d = det(X);
    double n2 = frob2(X);
    // X^{-T} = cof(X)/det(X)
    double ni2 = frob2(C) / (d * d);
    double g = scale ? sqrt(sqrt(ni2 / n2)) : 1.0;
    double diff = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      double xn = 0.5 * (g * X[i] + C[i] / (d * g));
      double dd = xn - X[i];
      diff += dd * dd;
      X[i] = xn;
    }
    if (diff < 1e-6) scale = false;
    if (diff <= 1e-30) break;
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = X[i];
  return true;
}

// Principal frame F = U diag(s) V^T (det F > 0): R from the polar iteration,
// S_F = sym(R^T F) = V diag(s) V^T by Jacobi, U = R V.
MPL_DEV bool principal_frame(const double* F, double* U, double* s, double* V, double* R) {
  if (!polar_rotation(F, R)) return false;
  double SF[9];
  mul_tn(R, F, SF);
  eig_sym3(SF, s, V);
  if (det(V) < 0.0) {
    V[2] = -V[2]; V[5] = -V[5]; V[8] = -V[8];
  }
  mul(R, V, U);
  return true;
}

// ---------------------------------------------------------------- models
// Principal derivatives of psi_hat for the three models:
//   d[i] = d psi_hat / d s_i,  H[i][j] = d^2 psi_hat / d s_i d s_j,
//   tw[p] = (d_i - d_j)/(s_i - s_j),  fl[p] = (d_i + d_j)/(s_i + s_j)
// for the pairs p = (0,1), (1,2), (0,2).
MPL_DEV void principal_derivs(const MatParams& m, const double* s, double* d, double (&H)[3][3],
                              double* tw, double* fl) {
  const int pi[3] = {0, 1, 0}, pj[3] = {1, 2, 2};
  const double J = s[0] * s[1] * s[2];
  if (m.model == WATER) {
    // psi = kappa/2 (J - 1)^2: d_i = kappa (J - 1) J / s_i,
    // H_ii = kappa J^2 / s_i^2, H_ij = kappa J (2J - 1) / (s_i s_j); both pair
    // quotients are closed forms, -+ kappa (J - 1) J / (s_i s_j)
    const double k = m.kappa;
    for (int i = 0; i < 3; ++i) {
      d[i] = k * (J - 1.0) * J / s[i];
      for (int j = 0; j < 3; ++j)
        H[i][j] = (i == j) ? k * J * J / (s[i] * s[i]) : k * J * (2.0 * J - 1.0) / (s[i] * s[j]);
    }
    for (int p = 0; p < 3; ++p) {
      const double q = k * (J - 1.0) * J / (s[pi[p]] * s[pj[p]]);
      tw[p] = -q;
      fl[p] = q;
    }
  } else if (m.model == FIXED_COROTATED) {
    // psi = mu sum (s_i - 1)^2 + lambda/2 (J - 1)^2
    for (int i = 0; i < 3; ++i) {
      double sjk = J / s[i];
      d[i] = 2.0 * m.mu * (s[i] - 1.0) + m.lambda * (J - 1.0) * sjk;
      for (int j = 0; j < 3; ++j) {
        if (i == j) H[i][i] = 2.0 * m.mu + m.lambda * sjk * sjk;
        else {
          int k = 3 - i - j;
          H[i][j] = m.lambda * s[k] * (2.0 * J - 1.0);
        }
      }
    }
    for (int p = 0; p < 3; ++p) {
      int i = pi[p], j = pj[p], k = 3 - i - j;
      tw[p] = 2.0 * m.mu - m.lambda * (J - 1.0) * s[k];
      fl[p] = 2.0 * m.mu * (1.0 - 2.0 / (s[i] + s[j])) + m.lambda * (J - 1.0) * s[k];
    }
  } else if (m.model == NEOHOOKEAN) {
    // psi = mu/2 (J^{-2/3} I - 3) + kappa/4 (J^2 - 1 - 2 log J), I = sum s^2
    const double c = pow(J, -2.0 / 3.0);
    const double I = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
    const double vol = 0.5 * m.kappa * (J * J - 1.0);
    for (int i = 0; i < 3; ++i) {
      d[i] = m.mu * c * (s[i] - I / (3.0 * s[i])) + vol / s[i];
      for (int j = 0; j < 3; ++j) {
        if (i == j)
          H[i][i] = m.mu * c * (-1.0 / 3.0 + 5.0 * I / (9.0 * s[i] * s[i])) +
                    0.5 * m.kappa * (J * J + 1.0) / (s[i] * s[i]);
        else
          H[i][j] = m.mu * c * (-2.0 * s[i] / (3.0 * s[j]) - 2.0 * s[j] / (3.0 * s[i]) +
                                2.0 * I / (9.0 * s[i] * s[j])) +
                    m.kappa * J * J / (s[i] * s[j]);
      }
    }
    for (int p = 0; p < 3; ++p) {
      int i = pi[p], j = pj[p];
      double sij = s[i] * s[j];
      tw[p] = m.mu * c * (1.0 + I / (3.0 * sij)) - vol / sij;
      fl[p] = m.mu * c * (1.0 - I / (3.0 * sij)) + vol / sij;
    }
  } else {  // HENCKY: psi = mu sum e_i^2 + lambda/2 (sum e)^2, e = log s
    double e[3] = {log(s[0]), log(s[1]), log(s[2])};
    double tr = e[0] + e[1] + e[2];
    double t[3];
    for (int i = 0; i < 3; ++i) {
      t[i] = 2.0 * m.mu * e[i] + m.lambda * tr;
      d[i] = t[i] / s[i];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        H[i][j] = (i == j) ? (2.0 * m.mu + m.lambda - t[i]) / (s[i] * s[i])
                           : m.lambda / (s[i] * s[j]);
    for (int p = 0; p < 3; ++p) {
      int i = pi[p], j = pj[p];
      // (d_i - d_j)/(s_i - s_j) = [2 mu (h/expm1(h) - e_j) - lambda tr]/(s_i s_j), h = e_i - e_j
      double h = e[i] - e[j];
      double q = (h == 0.0) ? 1.0 : h / expm1(h);
      tw[p] = (2.0 * m.mu * (q - e[j]) - m.lambda * tr) / (s[i] * s[j]);
      fl[p] = (d[i] + d[j]) / (s[i] + s[j]);
    }
  }
}

// Energy density psi(F); +inf outside the domain (det F <= 0).
MPL_DEV double psi(const MatParams& m, const double* F) {
  const double J = det(F);
  if (!(J > 0.0)) return INFINITY;
  if (m.model == WATER) return 0.5 * m.kappa * (J - 1.0) * (J - 1.0);
  if (m.model == NEOHOOKEAN) {
    double I = frob2(F);
    return 0.5 * m.mu * (pow(J, -2.0 / 3.0) * I - 3.0) + 0.25 * m.kappa * (J * J - 1.0 - 2.0 * log(J));
  }
  double R[9];
  if (!polar_rotation(F, R)) return INFINITY;
  if (m.model == FIXED_COROTATED) {
    double D[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) D[i] = F[i] - R[i];
    return m.mu * frob2(D) + 0.5 * m.lambda * (J - 1.0) * (J - 1.0);
  }
  // HENCKY from the singular values of the symmetric stretch
  double SF[9], s[3], V[9];
  mul_tn(R, F, SF);
  eig_sym3(SF, s, V);
  double e0 = log(s[0]), e1 = log(s[1]), e2 = log(s[2]);
  double tr = e0 + e1 + e2;
  return m.mu * (e0 * e0 + e1 * e1 + e2 * e2) + 0.5 * m.lambda * tr * tr;
}

// First Piola stress P(F).  Returns false outside the domain.
MPL_DEV bool piola(const MatParams& m, const double* F, double* P) {
  const double J = det(F);
  if (!(J > 0.0)) return false;
  double C[9];
  cofactor(F, C);
  if (m.model == WATER) {  // P = kappa (J - 1) cof F
#pragma unroll
    for (int i = 0; i < 9; ++i) P[i] = m.kappa * (J - 1.0) * C[i];
    return true;
  }
  if (m.model == NEOHOOKEAN) {
    // P = mu J^{-2/3} (F - I1/3 F^{-T}) + kappa/2 (J^2 - 1) F^{-T}, F^{-T} = cof F / J
    double c = pow(J, -2.0 / 3.0), I1 = frob2(F), vol = 0.5 * m.kappa * (J * J - 1.0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      double fit = C[i] / J;
      P[i] = m.mu * c * (F[i] - I1 / 3.0 * fit) + vol * fit;
    }
    return true;
  }
  if (m.model == FIXED_COROTATED) {
    double R[9];
    if (!polar_rotation(F, R)) return false;
#pragma unroll
    for (int i = 0; i < 9; ++i) P[i] = 2.0 * m.mu * (F[i] - R[i]) + m.lambda * (J - 1.0) * C[i];
    return true;
  }
  double U[9], s[3], V[9], R[9];
  if (!principal_frame(F, U, s, V, R)) return false;
  double e[3] = {log(s[0]), log(s[1]), log(s[2])};
  double tr = e[0] + e[1] + e[2];
  double ph[3];
  for (int i = 0; i < 3; ++i) ph[i] = (2.0 * m.mu * e[i] + m.lambda * tr) / s[i];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      P[i * 3 + j] = U[i * 3] * ph[0] * V[j * 3] + U[i * 3 + 1] * ph[1] * V[j * 3 + 1] +
                     U[i * 3 + 2] * ph[2] * V[j * 3 + 2];
  return true;
}

// Kirchhoff stress tau = P F^T (symmetric, 6 entries).
MPL_DEV bool kirchhoff(const MatParams& m, const double* F, double* tau6) {
  const double J = det(F);
  if (!(J > 0.0)) return false;
  double T[9];
  if (m.model == WATER) {
    // tau = pi I with the pressure pi = kappa J (J - 1)
    const double pr = m.kappa * J * (J - 1.0);
#pragma unroll
    for (int i = 0; i < 9; ++i) T[i] = (i % 4 == 0) ? pr : 0.0;
  } else if (m.model == NEOHOOKEAN) {
    // tau = mu J^{-2/3} dev(F F^T) + kappa/2 (J^2 - 1) I
    double B[9];
    mul_nt(F, F, B);
    double c = pow(J, -2.0 / 3.0), tr3 = (B[0] + B[4] + B[8]) / 3.0, vol = 0.5 * m.kappa * (J * J - 1.0);
#pragma unroll
    for (int i = 0; i < 9; ++i) T[i] = m.mu * c * B[i];
    T[0] += -m.mu * c * tr3 + vol;
    T[4] += -m.mu * c * tr3 + vol;
    T[8] += -m.mu * c * tr3 + vol;
  } else if (m.model == FIXED_COROTATED) {
    // tau = 2 mu (F - R) F^T + lambda J (J - 1) I
    double R[9], D[9];
    if (!polar_rotation(F, R)) return false;
#pragma unroll
    for (int i = 0; i < 9; ++i) D[i] = F[i] - R[i];
    mul_nt(D, F, T);
#pragma unroll
    for (int i = 0; i < 9; ++i) T[i] *= 2.0 * m.mu;
    double v = m.lambda * J * (J - 1.0);
    T[0] += v; T[4] += v; T[8] += v;
  } else {
    // tau = U diag(2 mu e_i + lambda tr e) U^T
    double U[9], s[3], V[9], R[9];
    if (!principal_frame(F, U, s, V, R)) return false;
    double e[3] = {log(s[0]), log(s[1]), log(s[2])};
    double tr = e[0] + e[1] + e[2];
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = 2.0 * m.mu * e[i] + m.lambda * tr;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        T[i * 3 + j] = U[i * 3] * t[0] * U[j * 3] + U[i * 3 + 1] * t[1] * U[j * 3 + 1] +
                       U[i * 3 + 2] * t[2] * U[j * 3 + 2];
  }
  full_to_sym(T, tau6);
  return true;
}

// ---------------------------------------------------------------- inverse
// Largest real root of m^3 + p m + q = 0 (p <= 0 for deviatoric offsets):
// Cardano with the second cube root from the product identity A B = -p/3,
// or the trigonometric form (largest root, k = 0) when three roots are real.
MPL_DEV double cubic_largest_root(double p, double q) {
  double p3 = p / 3.0;
  double disc = 0.25 * q * q + p3 * p3 * p3;
  if (disc >= 0.0) {
    double h = -0.5 * q;
    double A = cbrt(h + copysign(sqrt(disc), h));
    return (A == 0.0) ? 0.0 : A - p3 / A;
  }
  double r = 2.0 * sqrt(-p3);
  double arg = (1.5 * q / p) * sqrt(-3.0 / p);
  arg = fmin(1.0, fmax(-1.0, arg));
  return r * cos(acos(arg) / 3.0);
}

// Principal stretches from principal Kirchhoff stresses (tau_i = s_i dpsi/ds_i).
// Returns 0 on success, 1 when the stress lies outside the model's range
// (the result is then clamped and flagged).
MPL_DEV int stretch_from_principal(const MatParams& m, const double* t, double* s) {
  if (m.model == WATER) {
    // pressure pi = mean principal stress = kappa J (J - 1), inverted on J > 0:
    // J = (1 + sqrt(1 + 4 pi / kappa)) / 2 (no root below pi = -kappa/4: J = 1/2,
    // flagged); isotropic base s_i = J^{1/3}
    const double pr = (t[0] + t[1] + t[2]) / 3.0;
    double r = 1.0 + 4.0 * pr / m.kappa;
    int flag = 0;
    if (r < 0.0) { r = 0.0; flag = 1; }
    const double c = cbrt(0.5 * (1.0 + sqrt(r)));
    s[0] = s[1] = s[2] = c;
    return flag;
  }
  if (m.model == HENCKY) {
    double lsum = (t[0] + t[1] + t[2]) / (2.0 * m.mu + 3.0 * m.lambda);
    for (int i = 0; i < 3; ++i) s[i] = exp((t[i] - m.lambda * lsum) / (2.0 * m.mu));
    return 0;
  }
  if (m.model == NEOHOOKEAN) {
    int flag = 0;
    double alpha = (t[0] + t[1] + t[2]) / 3.0;
    double r = 1.0 + 2.0 * alpha / m.kappa;
    double J = (r > 1e-12) ? sqrt(r) : (flag = 1, 1e-6);
    double sc = m.mu * pow(J, -2.0 / 3.0);
    double d0 = (t[0] - alpha) / sc, d1 = (t[1] - alpha) / sc, d2 = (t[2] - alpha) / sc;
    double mm = cubic_largest_root(d0 * d1 + d1 * d2 + d2 * d0, d0 * d1 * d2 - J * J);
    double b[3] = {mm + d0, mm + d1, mm + d2};
    for (int i = 0; i < 3; ++i) {
      if (!(b[i] > 0.0)) { b[i] = 1e-12; flag = 1; }
      s[i] = sqrt(b[i]);
    }
    return flag;
  }
  // FIXED_COROTATED: tau_i = 2 mu s_i (s_i - 1) + a(J), a = lambda J (J - 1);
  // s_i(J) = (1 + sqrt(1 + 2 (tau_i - a)/mu))/2 on the branch s_i >= 1/2;
  // h(J) = prod s_i(J) - J is strictly decreasing for J >= 1/2: safeguarded
  // Newton on [1/2, J_max].
  const double mu = m.mu, la = m.lambda;
  double tmin = fmin(t[0], fmin(t[1], t[2]));
  double amax = tmin + 0.5 * mu;
  double lo = 0.5, hi;
  if (la > 0.0) {
    double disc = 1.0 + 4.0 * amax / la;
    if (disc < 0.0) { s[0] = s[1] = s[2] = 0.5; return 1; }
    hi = 0.5 * (1.0 + sqrt(disc));
  } else {
    hi = 1e6;
  }
  if (!(hi > lo)) { s[0] = s[1] = s[2] = 0.5; return 1; }
  auto eval = [&](double J, double* sv, double* dh) {
    double a = la * J * (J - 1.0), da = la * (2.0 * J - 1.0);
    double prod = 1.0, rs[3];
    for (int i = 0; i < 3; ++i) {
      double rad = fmax(1.0 + 2.0 * (t[i] - a) / mu, 0.0);
      rs[i] = sqrt(rad);
      sv[i] = 0.5 * (1.0 + rs[i]);
      prod *= sv[i];
    }
    double dp = 0.0;
    for (int i = 0; i < 3; ++i) {
      double dsi = (rs[i] > 0.0) ? -da / (2.0 * mu * rs[i]) : -INFINITY;
      dp += dsi * (prod / sv[i]);
    }
    *dh = dp - 1.0;
    return prod - J;
  };
  double sv[3], dh;
  if (eval(lo, sv, &dh) < 0.0) { s[0] = sv[0]; s[1] = sv[1]; s[2] = sv[2]; return 1; }
  double hh = eval(hi, sv, &dh);
  if (hh > 0.0) { s[0] = sv[0]; s[1] = sv[1]; s[2] = sv[2]; return 1; }
  double J = fmin(fmax(1.0 + (t[0] + t[1] + t[2]) / (2.0 * mu + 3.0 * la), lo), hi);
  for (int it = 0; it < 100; ++it) {
    double h = eval(J, sv, &dh);
    if (h == 0.0) break;
    if (h > 0.0) lo = J; else hi = J;
    double Jn = (dh < 0.0 && isfinite(dh)) ? J - h / dh : 0.5 * (lo + hi);
    if (!(Jn > lo && Jn < hi)) Jn = 0.5 * (lo + hi);
    if (fabs(Jn - J) <= 1e-16 * J || hi - lo <= 1e-16 * J) { J = Jn; break; }
    J = Jn;
  }
  eval(J, sv, &dh);
  s[0] = sv[0]; s[1] = sv[1]; s[2] = sv[2];
  return 0;
}

// Plastic projection of an elastic F (Hencky strain e = log s):
// von Mises caps 2 mu |dev e| at the yield stress; Drucker-Prager projects
// to the cone |dev e| + (3 lambda + 2 mu)/(2 mu) tr(e) alpha_f <= 0 and to
// the tip e = 0 under expansion.  Returns the plastic increment (0 = none).
MPL_DEV double plastic_project(const MatParams& m, double* F) {
  if (m.plastic == PLASTIC_NONE) return 0.0;
  double U[9], s[3], V[9], R[9];
  if (!principal_frame(F, U, s, V, R)) return 0.0;
  double e[3] = {log(s[0]), log(s[1]), log(s[2])};
  double tr = e[0] + e[1] + e[2];
  double dv[3] = {e[0] - tr / 3.0, e[1] - tr / 3.0, e[2] - tr / 3.0};
  double nd = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  double dg = 0.0;
  if (m.plastic == PLASTIC_VON_MISES) {
    if (2.0 * m.mu * nd > m.yield_stress && nd > 0.0) {
      dg = nd - m.yield_stress / (2.0 * m.mu);
      for (int i = 0; i < 3; ++i) e[i] -= dg * dv[i] / nd;
    }
  } else {
    if (tr > 0.0) {
      dg = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
      e[0] = e[1] = e[2] = 0.0;
    } else {
      double g = nd + (3.0 * m.lambda + 2.0 * m.mu) / (2.0 * m.mu) * tr * m.alpha_f;
      if (g > 0.0 && nd > 0.0) {
        dg = g;
        for (int i = 0; i < 3; ++i) e[i] -= g * dv[i] / nd;
      }
    }
  }
  if (dg > 0.0) {
    double se[3] = {exp(e[0]), exp(e[1]), exp(e[2])};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        F[i * 3 + j] = U[i * 3] * se[0] * V[j * 3] + U[i * 3 + 1] * se[1] * V[j * 3 + 1] +
                       U[i * 3 + 2] * se[2] * V[j * 3 + 2];
  }
  return dg;
}

}  // namespace mpl
