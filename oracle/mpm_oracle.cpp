// FP64 CPU oracle for the MPM Lite implicit step — TEST INFRASTRUCTURE ONLY.
//
// Only tests, the smoke check and the benchmark's CPU-baseline leg may load
// this file's library.  It shares no code with the HIP product path.
//
// Plain, slow and written for reading against the paper:
//   * every formula is written out once, in the paper's notation;
//   * no blocking, fusion or reordering beyond what the paper states;
//   * 3x3 / 9x9 symmetric eigenproblems use textbook cyclic Jacobi;
//   * sums over particles and cells run in index order (serial), except
//     independent per-cell work, which may run in OpenMP threads but writes
//     into per-cell slots that are then summed serially.
//
// Readings of the paper where it is silent are listed next to the code that
// takes them (grid origin 0, active cell = positive mass, projected Newton,
// Armijo backtracking, fixed-corotated inverse, plasticity formulas).

#include "oracle.h"

#include <cmath>
#include <cstring>
#include <vector>
#include <algorithm>
#include <limits>

namespace {

// ---------------------------------------------------------------------------
// Small dense helpers (row-major 3x3).
// ---------------------------------------------------------------------------
inline void m3_mul(const double* A, const double* B, double* C) {
  double T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      T[i * 3 + j] = s;
    }
  std::memcpy(C, T, sizeof(T));
}
inline void m3_transpose(const double* A, double* B) {
  double T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[i * 3 + j] = A[j * 3 + i];
  std::memcpy(B, T, sizeof(T));
}
inline double m3_det(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}
// Cofactor matrix: columns of F are f0,f1,f2; cof(F) = [f1 x f2, f2 x f0, f0 x f1]
// (as columns).  cof(F) = det(F) F^{-T} for invertible F.
inline void m3_cofactor(const double* F, double* C) {
  double f[3][3];
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) f[c][r] = F[r * 3 + c];
  auto cross = [](const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
  };
  double c0[3], c1[3], c2[3];
  cross(f[1], f[2], c0);
  cross(f[2], f[0], c1);
  cross(f[0], f[1], c2);
  for (int r = 0; r < 3; ++r) {
    C[r * 3 + 0] = c0[r];
    C[r * 3 + 1] = c1[r];
    C[r * 3 + 2] = c2[r];
  }
}
// Directional derivative of cof(F) along E.
inline void m3_cofactor_deriv(const double* F, const double* E, double* dC) {
  double f[3][3], e[3][3];
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) {
      f[c][r] = F[r * 3 + c];
      e[c][r] = E[r * 3 + c];
    }
  auto cross = [](const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
  };
  const int nxt[3][2] = {{1, 2}, {2, 0}, {0, 1}};
  for (int col = 0; col < 3; ++col) {
    double a[3], b[3];
    cross(e[nxt[col][0]], f[nxt[col][1]], a);
    cross(f[nxt[col][0]], e[nxt[col][1]], b);
    for (int r = 0; r < 3; ++r) dC[r * 3 + col] = a[r] + b[r];
  }
}
inline bool m3_inverse(const double* A, double* Ai) {
  double C[9];
  m3_cofactor(A, C);  // C = det(A) A^{-T}
  double d = m3_det(A);
  if (d == 0.0) return false;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ai[i * 3 + j] = C[j * 3 + i] / d;
  return true;
}
inline double m3_ddot(const double* A, const double* B) {
  double s = 0.0;
  for (int i = 0; i < 9; ++i) s += A[i] * B[i];
  return s;
}

// Cyclic Jacobi for a symmetric n x n matrix.  On return w holds the
// eigenvalues and the columns of Q the eigenvectors (Q[r*n+c] = comp r of vec c).
void jacobi_eigen(int n, const double* Ain, double* w, double* Q) {
  std::vector<double> A(Ain, Ain + n * n);
  for (int i = 0; i < n * n; ++i) Q[i] = 0.0;
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a2 = A[i * n + j] * A[i * n + j];
        tot += a2;
        if (i != j) off += a2;
      }
    if (off == 0.0 || off <= 1e-34 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        A[p * n + q] = A[q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {  // Q <- Q J
          double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - s * qkq;
          Q[k * n + q] = s * qkp + c * qkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

// Signed SVD F = U diag(sig) V^T with U, V rotations (det +1), |sig| sorted
// descending; sig[2] carries the sign of det F.
void svd3(const double* F, double* U, double* sig, double* V) {
  double C[9], Ft[9];
  m3_transpose(F, Ft);
  m3_mul(Ft, F, C);
  double w[3], Q[9];
  jacobi_eigen(3, C, w, Q);
  int order[3] = {0, 1, 2};
  std::sort(order, order + 3, [&](int a, int b) { return w[a] > w[b]; });
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) V[r * 3 + c] = Q[r * 3 + order[c]];
  if (m3_det(V) < 0.0)
    for (int r = 0; r < 3; ++r) V[r * 3 + 2] = -V[r * 3 + 2];
  double fv[3][3];  // fv[c] = F v_c
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += F[r * 3 + k] * V[k * 3 + c];
      fv[c][r] = s;
    }
  double u[3][3];
  double scale = std::sqrt(std::max(w[order[0]], 0.0));
  double n0 = std::sqrt(fv[0][0] * fv[0][0] + fv[0][1] * fv[0][1] + fv[0][2] * fv[0][2]);
  if (n0 > 1e-300) {
    for (int r = 0; r < 3; ++r) u[0][r] = fv[0][r] / n0;
  } else {
    u[0][0] = 1.0; u[0][1] = 0.0; u[0][2] = 0.0;
  }
  double d = u[0][0] * fv[1][0] + u[0][1] * fv[1][1] + u[0][2] * fv[1][2];
  double t[3];
  for (int r = 0; r < 3; ++r) t[r] = fv[1][r] - d * u[0][r];
  double n1 = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  if (n1 > 1e-14 * std::max(scale, 1e-300)) {
    for (int r = 0; r < 3; ++r) u[1][r] = t[r] / n1;
  } else {
    // pick any unit vector orthogonal to u0
    double a[3] = {1.0, 0.0, 0.0};
    if (std::fabs(u[0][0]) > 0.9) { a[0] = 0.0; a[1] = 1.0; }
    double dd = a[0] * u[0][0] + a[1] * u[0][1] + a[2] * u[0][2];
    for (int r = 0; r < 3; ++r) t[r] = a[r] - dd * u[0][r];
    double nn = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int r = 0; r < 3; ++r) u[1][r] = t[r] / nn;
  }
  u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
  u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
  u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
  for (int c = 0; c < 3; ++c) {
    for (int r = 0; r < 3; ++r) U[r * 3 + c] = u[c][r];
    sig[c] = u[c][0] * fv[c][0] + u[c][1] * fv[c][1] + u[c][2] * fv[c][2];
  }
}

// Polar F = R S with R a rotation (R = U V^T from the signed SVD).
void polar(const double* F, double* R, double* S) {
  double U[9], sig[3], V[9], Vt[9];
  svd3(F, U, sig, V);
  m3_transpose(V, Vt);
  m3_mul(U, Vt, R);
  double D[9] = {sig[0], 0, 0, 0, sig[1], 0, 0, 0, sig[2]}, T[9];
  m3_mul(V, D, T);
  m3_mul(T, Vt, S);
}

// Clamp negative eigenvalues of a symmetric n x n matrix at zero.
void project_psd(int n, double* A) {
  std::vector<double> w(n), Q(n * n), S(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) S[i * n + j] = 0.5 * (A[i * n + j] + A[j * n + i]);
  jacobi_eigen(n, S.data(), w.data(), Q.data());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k)
        if (w[k] > 0.0) s += Q[i * n + k] * w[k] * Q[j * n + k];
      A[i * n + j] = s;
    }
}

constexpr double kInf = std::numeric_limits<double>::infinity();

// ---------------------------------------------------------------------------
// Constitutive models (Sec. 4.3).
// ---------------------------------------------------------------------------
double nh_kappa(const or_material* m) { return 2.0 * m->mu / 3.0 + m->lambda; }

// Split Neo-Hookean energy, Sec. 4.3.2 (deviatoric part on J^{-1/3}F,
// volumetric part kappa/2((J^2-1)/2 - log J)).
double psi_nh(const or_material* m, const double* F) {
  double J = m3_det(F);
  if (!(J > 0.0)) return kInf;
  double I1 = m3_ddot(F, F);
  double k = nh_kappa(m);
  return 0.5 * m->mu * (std::pow(J, -2.0 / 3.0) * I1 - 3.0) +
         0.5 * k * (0.5 * (J * J - 1.0) - std::log(J));
}
// P = mu J^{-2/3} (F - I1/3 F^{-T}) + kappa/2 (J^2 - 1) F^{-T}.
int piola_nh(const or_material* m, const double* F, double* P) {
  double J = m3_det(F);
  if (!(J > 0.0)) return OR_ERR_DOMAIN;
  double C[9];
  m3_cofactor(F, C);
  double FiT[9];
  for (int i = 0; i < 9; ++i) FiT[i] = C[i] / J;
  double I1 = m3_ddot(F, F), k = nh_kappa(m), c = std::pow(J, -2.0 / 3.0);
  for (int i = 0; i < 9; ++i)
    P[i] = m->mu * c * (F[i] - I1 / 3.0 * FiT[i]) + 0.5 * k * (J * J - 1.0) * FiT[i];
  return OR_OK;
}
// Directional derivative of piola_nh, written term by term.
int dpdf_nh(const or_material* m, const double* F, double* A) {
  double J = m3_det(F);
  if (!(J > 0.0)) return OR_ERR_DOMAIN;
  double Cf[9], FiT[9];
  m3_cofactor(F, Cf);
  for (int i = 0; i < 9; ++i) FiT[i] = Cf[i] / J;
  double I1 = m3_ddot(F, F), k = nh_kappa(m), c = std::pow(J, -2.0 / 3.0);
  for (int e = 0; e < 9; ++e) {
    double E[9] = {0};
    E[e] = 1.0;
    double trFiE = m3_ddot(FiT, E);      // tr(F^{-1} E)
    double dJ = J * trFiE;
    double dc = -2.0 / 3.0 * c * trFiE;
    double dI1 = 2.0 * m3_ddot(F, E);
    // d(F^{-T}) = -F^{-T} E^T F^{-T}
    double Et[9], T1[9], dFiT[9];
    m3_transpose(E, Et);
    m3_mul(FiT, Et, T1);
    m3_mul(T1, FiT, dFiT);
    for (int i = 0; i < 9; ++i) dFiT[i] = -dFiT[i];
    for (int i = 0; i < 9; ++i) {
      double dP = m->mu * (dc * (F[i] - I1 / 3.0 * FiT[i]) +
                           c * (E[i] - dI1 / 3.0 * FiT[i] - I1 / 3.0 * dFiT[i])) +
                  0.5 * k * (2.0 * J * dJ * FiT[i] + (J * J - 1.0) * dFiT[i]);
      A[i * 9 + e] = dP;  // A[(P index), (F index)]
    }
  }
  return OR_OK;
}

// Fixed-corotated: psi = mu |F - R|^2 + lambda/2 (J-1)^2.
double psi_fcr(const or_material* m, const double* F) {
  double R[9], S[9];
  polar(F, R, S);
  double s = 0.0;
  for (int i = 0; i < 9; ++i) s += (F[i] - R[i]) * (F[i] - R[i]);
  double J = m3_det(F);
  return m->mu * s + 0.5 * m->lambda * (J - 1.0) * (J - 1.0);
}
// P = 2 mu (F - R) + lambda (J - 1) cof(F).
int piola_fcr(const or_material* m, const double* F, double* P) {
  double R[9], S[9], C[9];
  polar(F, R, S);
  m3_cofactor(F, C);
  double J = m3_det(F);
  for (int i = 0; i < 9; ++i) P[i] = 2.0 * m->mu * (F[i] - R[i]) + m->lambda * (J - 1.0) * C[i];
  return OR_OK;
}
// dP = 2 mu (E - dR) + lambda (cof F : E) cof F + lambda (J - 1) d cof F.
// dR = R [w]x where (tr(S) I - S) w = axial(R^T E - E^T R)  (from F = R S,
// R^T dF - dF^T R = W S + S W with W = R^T dR skew).
int dpdf_fcr(const or_material* m, const double* F, double* A) {
  double R[9], S[9], C[9], Rt[9];
  polar(F, R, S);
  m3_cofactor(F, C);
  m3_transpose(R, Rt);
  double J = m3_det(F);
  double trS = S[0] + S[4] + S[8];
  double Mw[9];
  for (int i = 0; i < 9; ++i) Mw[i] = -S[i];
  Mw[0] += trS; Mw[4] += trS; Mw[8] += trS;
  double Mwi[9];
  bool inv = m3_inverse(Mw, Mwi);
  for (int e = 0; e < 9; ++e) {
    double E[9] = {0};
    E[e] = 1.0;
    double RtE[9], Et[9], EtR[9], K[9];
    m3_mul(Rt, E, RtE);
    m3_transpose(E, Et);
    m3_mul(Et, R, EtR);
    for (int i = 0; i < 9; ++i) K[i] = RtE[i] - EtR[i];
    double ax[3] = {K[7], K[2], K[3]};  // (K_32, K_13, K_21)
    double w[3] = {0, 0, 0};
    if (inv)
      for (int r = 0; r < 3; ++r) w[r] = Mwi[r * 3 + 0] * ax[0] + Mwi[r * 3 + 1] * ax[1] + Mwi[r * 3 + 2] * ax[2];
    double W[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    double dR[9];
    m3_mul(R, W, dR);
    double dC[9];
    m3_cofactor_deriv(F, E, dC);
    double cE = m3_ddot(C, E);
    for (int i = 0; i < 9; ++i)
      A[i * 9 + e] = 2.0 * m->mu * (E[i] - dR[i]) + m->lambda * cE * C[i] +
                     m->lambda * (J - 1.0) * dC[i];
  }
  return inv ? OR_OK : OR_ERR_DOMAIN;
}

// StVK with Hencky strain, Sec. 4.3.1: psi = mu sum (log s_i)^2 + lambda/2 (sum log s_i)^2.
double psi_hencky(const or_material* m, const double* F) {
  double U[9], s[3], V[9];
  svd3(F, U, s, V);
  if (!(s[2] > 0.0)) return kInf;
  double e[3] = {std::log(s[0]), std::log(s[1]), std::log(s[2])};
  double tr = e[0] + e[1] + e[2];
  return m->mu * (e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) + 0.5 * m->lambda * tr * tr;
}
// P = U diag(tau_i / s_i) V^T, tau_i = 2 mu e_i + lambda sum e.
int piola_hencky(const or_material* m, const double* F, double* P) {
  double U[9], s[3], V[9];
  svd3(F, U, s, V);
  if (!(s[2] > 0.0)) return OR_ERR_DOMAIN;
  double e[3] = {std::log(s[0]), std::log(s[1]), std::log(s[2])};
  double tr = e[0] + e[1] + e[2];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k)
        acc += U[i * 3 + k] * ((2.0 * m->mu * e[k] + m->lambda * tr) / s[k]) * V[j * 3 + k];
      P[i * 3 + j] = acc;
    }
  return OR_OK;
}
// Isotropic tangent in the principal frame F = U diag(s) V^T:
//   dP^_ii = sum_j psi_ij dF^_jj,
//   (dP^_ij, dP^_ji) = [[a, b], [b, a]] (dF^_ij, dF^_ji),
// with a + b = (psi_i - psi_j)/(s_i - s_j), a - b = (psi_i + psi_j)/(s_i + s_j).
// For Hencky psi_i = tau_i / s_i, psi_ii = (2mu + lambda - tau_i)/s_i^2,
// psi_ij = lambda/(s_i s_j); the divided difference is written with
// log1p so that it stays exact as s_i -> s_j.
int dpdf_hencky(const or_material* m, const double* F, double* A) {
  double U[9], s[3], V[9];
  svd3(F, U, s, V);
  if (!(s[2] > 0.0)) return OR_ERR_DOMAIN;
  const double mu = m->mu, la = m->lambda;
  double e[3] = {std::log(s[0]), std::log(s[1]), std::log(s[2])};
  double tr = e[0] + e[1] + e[2];
  double tau[3], ps[3];
  for (int i = 0; i < 3; ++i) {
    tau[i] = 2.0 * mu * e[i] + la * tr;
    ps[i] = tau[i] / s[i];
  }
  double H[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      H[i][j] = (i == j) ? (2.0 * mu + la - tau[i]) / (s[i] * s[i]) : la / (s[i] * s[j]);
  double apb[3][3], amb[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      if (i == j) continue;
      // (psi_i - psi_j)/(s_i - s_j) = 2mu (e_i/s_i - e_j/s_j)/(s_i-s_j) - la tr/(s_i s_j)
      double x = (s[i] - s[j]) / s[j];
      double l1 = (x == 0.0) ? 1.0 : std::log1p(x) / x;      // (e_i-e_j)/(s_i-s_j) * s_j
      double dd = (l1 - e[j]) / (s[i] * s[j]);                 // (e_i/s_i-e_j/s_j)/(s_i-s_j)
      apb[i][j] = 2.0 * mu * dd - la * tr / (s[i] * s[j]);
      amb[i][j] = (ps[i] + ps[j]) / (s[i] + s[j]);
    }
  for (int e2 = 0; e2 < 9; ++e2) {
    double E[9] = {0};
    E[e2] = 1.0;
    double Eh[9];  // U^T E V
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) acc += U[k * 3 + i] * E[k * 3 + l] * V[l * 3 + j];
        Eh[i * 3 + j] = acc;
      }
    double Ph[9] = {0};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Ph[i * 3 + i] += H[i][j] * Eh[j * 3 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        if (i == j) continue;
        double a = 0.5 * (apb[i][j] + amb[i][j]), b = 0.5 * (apb[i][j] - amb[i][j]);
        Ph[i * 3 + j] = a * Eh[i * 3 + j] + b * Eh[j * 3 + i];
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) acc += U[i * 3 + k] * Ph[k * 3 + l] * V[j * 3 + l];
        A[(i * 3 + j) * 9 + e2] = acc;
      }
  }
  return OR_OK;
}

// J-based water (Sec. 3, Water): psi = kappa/2 (J - 1)^2 with kappa in
// m->lambda.  P = dpsi/dJ dJ/dF = kappa (J - 1) cof F, and
// dP[E] = kappa (cof F : E) cof F + kappa (J - 1) d(cof F)[E].
double psi_water(const or_material* m, const double* F) {
  double J = m3_det(F);
  if (!(J > 0.0)) return kInf;
  return 0.5 * m->lambda * (J - 1.0) * (J - 1.0);
}
int piola_water(const or_material* m, const double* F, double* P) {
  double J = m3_det(F);
  if (!(J > 0.0)) return OR_ERR_DOMAIN;
  double C[9];
  m3_cofactor(F, C);
  for (int i = 0; i < 9; ++i) P[i] = m->lambda * (J - 1.0) * C[i];
  return OR_OK;
}
int dpdf_water(const or_material* m, const double* F, double* A) {
  double J = m3_det(F);
  if (!(J > 0.0)) return OR_ERR_DOMAIN;
  double C[9];
  m3_cofactor(F, C);
  for (int e = 0; e < 9; ++e) {
    double E[9] = {0};
    E[e] = 1.0;
    double dC[9];
    m3_cofactor_deriv(F, E, dC);
    double cE = m3_ddot(C, E);
    for (int i = 0; i < 9; ++i) A[i * 9 + e] = m->lambda * (cE * C[i] + (J - 1.0) * dC[i]);
  }
  return OR_OK;
}

// ---------------------------------------------------------------------------
// Stress -> stretch inverses (Sec. 4.3, App. C).
// ---------------------------------------------------------------------------
inline double cbrt_signed(double z) { return z >= 0.0 ? std::cbrt(z) : -std::cbrt(-z); }

// Largest real root of m^3 + p m + q = 0 (App. C): Cardano when the
// discriminant is non-negative, the trigonometric form (k = 0) otherwise.
// In the Cardano branch the two real cube roots A, B satisfy A B = -p/3, so
// the smaller one is taken as -p/(3A) with A from the radicand of larger
// magnitude; this is the same root as the printed sum of cube roots, without
// the cancellation of -q/2 - sqrt(disc) when p is near 0.
double cardano_largest(double p, double q) {
  double disc = 0.25 * q * q + (p / 3.0) * (p / 3.0) * (p / 3.0);
  if (disc >= 0.0) {
    double sd = std::sqrt(disc);
    double h = -0.5 * q;
    double A = cbrt_signed(h >= 0.0 ? h + sd : h - sd);
    if (A == 0.0) return 0.0;
    return A - p / (3.0 * A);
  }
  double r = 2.0 * std::sqrt(-p / 3.0);
  double arg = (3.0 * q / (2.0 * p)) * std::sqrt(-3.0 / p);
  arg = std::min(1.0, std::max(-1.0, arg));
  double theta = std::acos(arg) / 3.0;
  return r * std::cos(theta);
}

int stretch_from_principal(const or_material* m, const double* t, double* sig) {
  const double mu = m->mu, la = m->lambda;
  int st = OR_OK;
  if (m->model == OR_WATER) {
    // Sec. 3, Water: pressure pi = mean principal stress, pi = kappa J (J - 1)
    // inverted on J > 0 as J = (1 + sqrt(1 + 4 pi / kappa)) / 2 (below
    // pi = -kappa/4 there is no root: J = 1/2 and a domain flag), and the
    // base is isotropic, sigma_i = J^{1/3}.
    double pi_c = (t[0] + t[1] + t[2]) / 3.0;
    double r = 1.0 + 4.0 * pi_c / m->lambda;
    if (r < 0.0) {
      r = 0.0;
      st = OR_ERR_DOMAIN;
    }
    double J = 0.5 * (1.0 + std::sqrt(r));
    for (int i = 0; i < 3; ++i) sig[i] = std::cbrt(J);
  } else if (m->model == OR_HENCKY) {
    // Sec. 4.3.1: s = tr tau/(2mu + 3 lambda), e_i = (tau_i - lambda s)/(2 mu).
    double s = (t[0] + t[1] + t[2]) / (2.0 * mu + 3.0 * la);
    for (int i = 0; i < 3; ++i) sig[i] = std::exp((t[i] - la * s) / (2.0 * mu));
  } else if (m->model == OR_NEOHOOKEAN) {
    // Sec. 4.3.2: J from the spherical part, offsets delta_i, cubic for m.
    double k = nh_kappa(m);
    double alpha = (t[0] + t[1] + t[2]) / 3.0;
    double r = 1.0 + 2.0 * alpha / k;
    double J;
    if (r <= 1e-12) {
      J = 1e-6;
      st = OR_ERR_DOMAIN;
    } else {
      J = std::sqrt(r);
    }
    double sc = mu * std::pow(J, -2.0 / 3.0);
    double d[3] = {(t[0] - alpha) / sc, (t[1] - alpha) / sc, (t[2] - alpha) / sc};
    double S2 = d[0] * d[1] + d[1] * d[2] + d[2] * d[0];
    double S3 = d[0] * d[1] * d[2];
    double mm = cardano_largest(S2, S3 - J * J);
    for (int i = 0; i < 3; ++i) {
      double b = mm + d[i];
      if (!(b > 0.0)) {
        b = 1e-12;
        st = OR_ERR_DOMAIN;
      }
      sig[i] = std::sqrt(b);
    }
  } else if (m->model == OR_FIXED_COROTATED) {
    // tau_i = 2 mu s_i (s_i - 1) + a,  a = lambda J (J - 1).  For a trial J the
    // stretch branch s_i >= 1/2 is s_i(J) = (1 + sqrt(1 + 2 (tau_i - a)/mu))/2.
    // For J >= 1/2, a(J) increases, so prod s_i(J) - J strictly decreases;
    // bisection on [1/2, J_max] (J_max: the smallest radicand reaches 0).
    double tmin = std::min(t[0], std::min(t[1], t[2]));
    double amax = tmin + 0.5 * mu;  // radicand >= 0  <=>  a <= amax
    double hi;
    if (la > 0.0) {
      double disc = 1.0 + 4.0 * amax / la;
      if (disc < 0.0) return OR_ERR_DOMAIN;
      hi = 0.5 * (1.0 + std::sqrt(disc));
    } else {
      hi = 1e6;
    }
    double lo = 0.5;
    if (!(hi > lo)) return OR_ERR_DOMAIN;
    auto resid = [&](double J, double* s) {
      double a = la * J * (J - 1.0);
      double p = 1.0;
      for (int i = 0; i < 3; ++i) {
        double rad = 1.0 + 2.0 * (t[i] - a) / mu;
        s[i] = 0.5 * (1.0 + std::sqrt(std::max(rad, 0.0)));
        p *= s[i];
      }
      return p - J;
    };
    double s[3];
    if (resid(lo, s) < 0.0) return OR_ERR_DOMAIN;
    if (resid(hi, s) > 0.0) return OR_ERR_DOMAIN;
    for (int it = 0; it < 400; ++it) {
      double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (resid(mid, s) >= 0.0) lo = mid; else hi = mid;
    }
    double rl = resid(lo, s);
    double sl[3] = {s[0], s[1], s[2]};
    double rh = resid(hi, s);
    if (std::fabs(rl) <= std::fabs(rh)) { sig[0] = sl[0]; sig[1] = sl[1]; sig[2] = sl[2]; }
    else { sig[0] = s[0]; sig[1] = s[1]; sig[2] = s[2]; }
  } else {
    return OR_ERR_ARG;
  }
  return st;
}

// Rotation-free base (Sec. 4.2-4.3): eigenvectors U of tau give the principal
// directions, the model inverse gives the stretches, S = U diag(sigma) U^T.
int stretch_from_tau(const or_material* m, const double* tau, double* S) {
  double Ts[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ts[i * 3 + j] = 0.5 * (tau[i * 3 + j] + tau[j * 3 + i]);
  double w[3], U[9];
  jacobi_eigen(3, Ts, w, U);
  double sig[3] = {1.0, 1.0, 1.0};
  int st = stretch_from_principal(m, w, sig);
  if (st != OR_OK && st != OR_ERR_DOMAIN) return st;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += U[i * 3 + k] * sig[k] * U[j * 3 + k];
      S[i * 3 + j] = acc;
    }
  return st;
}

double psi_any(const or_material* m, const double* F) {
  switch (m->model) {
    case OR_NEOHOOKEAN: return psi_nh(m, F);
    case OR_FIXED_COROTATED: return psi_fcr(m, F);
    case OR_HENCKY: return psi_hencky(m, F);
    case OR_WATER: return psi_water(m, F);
  }
  return kInf;
}
int piola_any(const or_material* m, const double* F, double* P) {
  switch (m->model) {
    case OR_NEOHOOKEAN: return piola_nh(m, F, P);
    case OR_FIXED_COROTATED: return piola_fcr(m, F, P);
    case OR_HENCKY: return piola_hencky(m, F, P);
    case OR_WATER: return piola_water(m, F, P);
  }
  return OR_ERR_ARG;
}
int dpdf_any(const or_material* m, const double* F, double* A) {
  switch (m->model) {
    case OR_NEOHOOKEAN: return dpdf_nh(m, F, A);
    case OR_FIXED_COROTATED: return dpdf_fcr(m, F, A);
    case OR_HENCKY: return dpdf_hencky(m, F, A);
    case OR_WATER: return dpdf_water(m, F, A);
  }
  return OR_ERR_ARG;
}
// Kirchhoff stress tau = P F^T (Sec. 3.2), evaluated in place per particle.
int tau_any(const or_material* m, const double* F, double* tau) {
  double P[9], Ft[9];
  int st = piola_any(m, F, P);
  if (st != OR_OK) return st;
  m3_transpose(F, Ft);
  m3_mul(P, Ft, tau);
  return OR_OK;
}

// Plastic projection of a particle's elastic F in Hencky strain e = log(sigma).
int plastic_project(const or_material* m, double* F, double* eps_acc) {
  if (m->plastic == OR_PLASTIC_NONE) return OR_OK;
  double U[9], s[3], V[9];
  svd3(F, U, s, V);
  if (!(s[2] > 0.0)) return OR_ERR_DOMAIN;
  double e[3] = {std::log(s[0]), std::log(s[1]), std::log(s[2])};
  double tr = e[0] + e[1] + e[2];
  double dev[3] = {e[0] - tr / 3.0, e[1] - tr / 3.0, e[2] - tr / 3.0};
  double nd = std::sqrt(dev[0] * dev[0] + dev[1] * dev[1] + dev[2] * dev[2]);
  double dgamma = 0.0;
  if (m->plastic == OR_PLASTIC_VON_MISES) {
    // Deviatoric Kirchhoff stress 2 mu |dev e| capped at the yield stress.
    if (2.0 * m->mu * nd > m->yield_stress && nd > 0.0) {
      dgamma = nd - m->yield_stress / (2.0 * m->mu);
      for (int i = 0; i < 3; ++i) e[i] -= dgamma * dev[i] / nd;
    }
  } else if (m->plastic == OR_PLASTIC_DRUCKER_PRAGER) {
    const double sphi = std::sin(m->friction_deg * M_PI / 180.0);
    const double alpha_f = std::sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi);
    if (tr > 0.0) {
      dgamma = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
      e[0] = e[1] = e[2] = 0.0;
    } else {
      double dg = nd + (3.0 * m->lambda + 2.0 * m->mu) / (2.0 * m->mu) * tr * alpha_f;
      if (dg > 0.0 && nd > 0.0) {
        dgamma = dg;
        for (int i = 0; i < 3; ++i) e[i] -= dg * dev[i] / nd;
      }
    }
  }
  if (dgamma > 0.0) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += U[i * 3 + k] * std::exp(e[k]) * V[j * 3 + k];
        F[i * 3 + j] = acc;
      }
    if (eps_acc) *eps_acc += dgamma;
  }
  return OR_OK;
}

// ---------------------------------------------------------------------------
// Grid geometry.
// ---------------------------------------------------------------------------
struct Grid {
  int n;
  double dx;
  int64_t nn() const { return (int64_t)(n + 1) * (n + 1) * (n + 1); }
  int64_t nc() const { return (int64_t)n * n * n; }
  int64_t node(int i, int j, int k) const { return ((int64_t)i * (n + 1) + j) * (n + 1) + k; }
  int64_t cell(int i, int j, int k) const { return ((int64_t)i * n + j) * n + k; }
};
// Q1 centre->node gradient in 3-D: grad w_ic = (x_i - x_c)/(2 dx^2) = (2 delta - 1)/(4 dx)
// per component for corner offset delta in {0,1}^3 (Sec. 3.3).
inline void grad_w(int d, double dx, double* gw) {
  for (int a = 0; a < 3; ++a) {
    int da = (d >> (2 - a)) & 1;
    gw[a] = (2.0 * da - 1.0) / (4.0 * dx);
  }
}
inline void corner(int d, int* o) {
  o[0] = (d >> 2) & 1;
  o[1] = (d >> 1) & 1;
  o[2] = d & 1;
}
// Velocity component a of node nidx is a degree of freedom: the node has
// mass and no boundary condition fixes that component (fixed[] bit a clear).
inline bool dof_free(const double* mi, const uint8_t* fixed, int64_t nidx, int a) {
  return mi[nidx] != 0.0 && !((fixed[nidx] >> a) & 1u);
}

// Particle -> centre stencil (Sec. 3.1): xi = x/dx - 1/2, base b = floor(xi),
// f = xi - b; the 8 centres b + delta get weight prod_a (delta_a ? f_a : 1 - f_a).
struct Stencil {
  int b[3];
  double f[3];
};
inline bool make_stencil(const Grid& g, const double* x, Stencil* s) {
  for (int a = 0; a < 3; ++a) {
    double xi = x[a] / g.dx - 0.5;
    double fb = std::floor(xi);
    s->b[a] = (int)fb;
    s->f[a] = xi - fb;
    if (s->b[a] < 0 || s->b[a] + 1 > g.n - 1) return false;
  }
  return true;
}
inline double stencil_weight(const Stencil& s, int d) {
  int o[3];
  corner(d, o);
  double w = 1.0;
  for (int a = 0; a < 3; ++a) w *= o[a] ? s.f[a] : 1.0 - s.f[a];
  return w;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

double or_psi(const or_material* mat, const double F[9]) { return psi_any(mat, F); }
int or_piola(const or_material* mat, const double F[9], double P[9]) { return piola_any(mat, F, P); }
int or_tau(const or_material* mat, const double F[9], double tau[9]) { return tau_any(mat, F, tau); }
int or_dpdf(const or_material* mat, const double F[9], double A[81]) { return dpdf_any(mat, F, A); }
int or_stretch(const or_material* mat, const double tau[9], double S[9]) {
  return stretch_from_tau(mat, tau, S);
}
int or_svd3(const double F[9], double U[9], double sig[3], double V[9]) {
  svd3(F, U, sig, V);
  return OR_OK;
}
int or_sym_eigen(int32_t n, const double* A, double* w, double* Q) {
  if (n <= 0 || n > 64) return OR_ERR_ARG;
  jacobi_eigen(n, A, w, Q);
  return OR_OK;
}
int or_project_psd(int32_t n, double* A) {
  if (n <= 0 || n > 64) return OR_ERR_ARG;
  project_psd(n, A);
  return OR_OK;
}
int or_cardano_largest(double p, double q, double* m) {
  *m = cardano_largest(p, q);
  return OR_OK;
}
int or_plastic_project(const or_material* mat, double F[9], double* eps_acc) {
  return plastic_project(mat, F, eps_acc);
}

// Alg. 2: particle -> centre unload (Eqs. of Sec. 3.1 and 3.2), normalise,
// then the centre -> node gather of Sec. 3.3 with w_ic = 1/8.
int or_unload(const or_grid* gg, int64_t np, const double* x, const double* v,
              const double* G, const double* F, const double* m, const double* V,
              const int32_t* mat, int32_t nmat, const or_material* mats,
              double* mc, double* vc, double* Gc, double* Vck, double* tauck,
              double* mi, double* vi) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc(), nn = g.nn();
  std::fill(mc, mc + nc, 0.0);
  std::fill(vc, vc + 3 * nc, 0.0);
  std::fill(Gc, Gc + 9 * nc, 0.0);
  std::fill(Vck, Vck + nmat * nc, 0.0);
  std::fill(tauck, tauck + 9 * nmat * nc, 0.0);
  std::fill(mi, mi + nn, 0.0);
  std::fill(vi, vi + 3 * nn, 0.0);
  int status = OR_OK;
  for (int64_t p = 0; p < np; ++p) {
    Stencil s;
    if (!make_stencil(g, x + 3 * p, &s)) return OR_ERR_OUTSIDE;
    int k = mat[p];
    if (k < 0 || k >= nmat) return OR_ERR_ARG;
    double tau[9];
    int st = tau_any(&mats[k], F + 9 * p, tau);
    if (st != OR_OK) status = st;
    const double* Gp = G + 9 * p;
    for (int d = 0; d < 8; ++d) {
      int o[3];
      corner(d, o);
      int ci = s.b[0] + o[0], cj = s.b[1] + o[1], ck = s.b[2] + o[2];
      int64_t c = g.cell(ci, cj, ck);
      double w = stencil_weight(s, d);
      double xc[3] = {(ci + 0.5) * g.dx, (cj + 0.5) * g.dx, (ck + 0.5) * g.dx};
      double dxp[3] = {xc[0] - x[3 * p], xc[1] - x[3 * p + 1], xc[2] - x[3 * p + 2]};
      double wm = w * m[p];
      mc[c] += wm;
      for (int a = 0; a < 3; ++a) {
        double aff = Gp[a * 3 + 0] * dxp[0] + Gp[a * 3 + 1] * dxp[1] + Gp[a * 3 + 2] * dxp[2];
        vc[3 * c + a] += wm * (v[3 * p + a] + aff);
      }
      for (int e = 0; e < 9; ++e) Gc[9 * c + e] += wm * Gp[e];
      double wV = w * V[p];
      Vck[k * nc + c] += wV;
      for (int e = 0; e < 9; ++e) tauck[(k * nc + c) * 9 + e] += wV * tau[e];
    }
  }
  for (int64_t c = 0; c < nc; ++c) {
    if (mc[c] != 0.0) {
      for (int a = 0; a < 3; ++a) vc[3 * c + a] /= mc[c];
      for (int e = 0; e < 9; ++e) Gc[9 * c + e] /= mc[c];
    }
    for (int k = 0; k < nmat; ++k)
      if (Vck[k * nc + c] != 0.0)
        for (int e = 0; e < 9; ++e) tauck[(k * nc + c) * 9 + e] /= Vck[k * nc + c];
  }
  for (int i = 0; i < g.n; ++i)
    for (int j = 0; j < g.n; ++j)
      for (int kk = 0; kk < g.n; ++kk) {
        int64_t c = g.cell(i, j, kk);
        if (mc[c] == 0.0) continue;
        double wm = mc[c] / 8.0;
        for (int d = 0; d < 8; ++d) {
          int o[3];
          corner(d, o);
          int64_t nidx = g.node(i + o[0], j + o[1], kk + o[2]);
          double r[3] = {(o[0] - 0.5) * g.dx, (o[1] - 0.5) * g.dx, (o[2] - 0.5) * g.dx};
          mi[nidx] += wm;
          for (int a = 0; a < 3; ++a) {
            const double* Gcc = Gc + 9 * c;
            double aff = Gcc[a * 3 + 0] * r[0] + Gcc[a * 3 + 1] * r[1] + Gcc[a * 3 + 2] * r[2];
            vi[3 * nidx + a] += wm * (vc[3 * c + a] + aff);
          }
        }
      }
  for (int64_t nidx = 0; nidx < nn; ++nidx)
    if (mi[nidx] != 0.0)
      for (int a = 0; a < 3; ++a) vi[3 * nidx + a] /= mi[nidx];
  return status;
}

// Dirichlet node sets: an active node (m_i > 0) inside a sticky or moving box
// has all three velocity components fixed to the box velocity (0 for sticky
// boxes); a moving box is translated by velocity * time.  Inside a slip plane
// only the component along the plane's normal axis is fixed, to 0.  fixed[]
// holds one bit per component; a component stays fixed once a box fixes it,
// and its value comes from the last box that fixes it.  Node-in-box uses a
// tolerance of 1e-6 dx.
int or_node_bcs(const or_grid* gg, const double* mi, int32_t nbc, const or_bc* bcs,
                double time, uint8_t* fixed, double* vfix) {
  Grid g{gg->n, gg->dx};
  const double eps = 1e-6 * g.dx;
  std::vector<int> slip_axis(nbc, -1);
  for (int b = 0; b < nbc; ++b) {
    if (bcs[b].kind == OR_BC_SLIP_PLANE) {
      int nz = 0;
      for (int a = 0; a < 3; ++a)
        if (bcs[b].velocity[a] != 0.0) { ++nz; slip_axis[b] = a; }
      if (nz != 1) return OR_ERR_ARG;
    } else if (bcs[b].kind != OR_BC_STICKY_BOX && bcs[b].kind != OR_BC_MOVING_BOX) {
      return OR_ERR_ARG;
    }
  }
  for (int i = 0; i <= g.n; ++i)
    for (int j = 0; j <= g.n; ++j)
      for (int k = 0; k <= g.n; ++k) {
        int64_t nidx = g.node(i, j, k);
        fixed[nidx] = 0;
        vfix[3 * nidx] = vfix[3 * nidx + 1] = vfix[3 * nidx + 2] = 0.0;
        if (mi[nidx] == 0.0) continue;
        double xn[3] = {i * g.dx, j * g.dx, k * g.dx};
        for (int b = 0; b < nbc; ++b) {
          double sh[3] = {0, 0, 0};
          if (bcs[b].kind == OR_BC_MOVING_BOX)
            for (int a = 0; a < 3; ++a) sh[a] = bcs[b].velocity[a] * time;
          bool in = true;
          for (int a = 0; a < 3; ++a)
            if (xn[a] < bcs[b].lo[a] + sh[a] - eps || xn[a] > bcs[b].hi[a] + sh[a] + eps) in = false;
          if (!in) continue;
          if (bcs[b].kind == OR_BC_SLIP_PLANE) {
            fixed[nidx] |= (uint8_t)(1u << slip_axis[b]);
            vfix[3 * nidx + slip_axis[b]] = 0.0;
            continue;
          }
          fixed[nidx] = 7;
          for (int a = 0; a < 3; ++a)
            vfix[3 * nidx + a] = bcs[b].kind == OR_BC_MOVING_BOX ? bcs[b].velocity[a] : 0.0;
        }
      }
  return OR_OK;
}

// Alg. 3, first loop: S_{c,k} from tau_{c,k} wherever V_{c,k} != 0.
int or_reconstruct(const or_grid* gg, int32_t nmat, const or_material* mats,
                   const double* Vck, const double* tauck, double* Sck) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc();
  int status = OR_OK;
  for (int k = 0; k < nmat; ++k) {
#pragma omp parallel for schedule(static) reduction(min : status)
    for (int64_t c = 0; c < nc; ++c) {
      double* S = Sck + (k * nc + c) * 9;
      if (Vck[k * nc + c] == 0.0) {
        for (int e = 0; e < 9; ++e) S[e] = (e % 4 == 0) ? 1.0 : 0.0;
        continue;
      }
      int st = stretch_from_tau(&mats[k], tauck + (k * nc + c) * 9, S);
      if (st != OR_OK) status = std::min(status, st);
    }
  }
  return status;
}

}  // extern "C"

namespace {

// G_c(v) = sum_i v_i (x) grad w_ic over the 8 corners (Sec. 3.3).
inline void cell_velocity_gradient(const Grid& g, int i, int j, int k, const double* v, double* Gm) {
  for (int e = 0; e < 9; ++e) Gm[e] = 0.0;
  for (int d = 0; d < 8; ++d) {
    int o[3];
    corner(d, o);
    const double* vn = v + 3 * g.node(i + o[0], j + o[1], k + o[2]);
    double gw[3];
    grad_w(d, g.dx, gw);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Gm[a * 3 + b] += vn[a] * gw[b];
  }
}

}  // namespace

extern "C" {

// Incremental potential of Sec. 4.2 / Alg. 3 with the rotation-free base:
//   Phi(v) = sum_free 1/2 m_i |v_i - vhat_i|^2 + sum_{c,k} V_{c,k} psi_k((I + dt G_c(v)) S_{c,k})
//   grad_i = m_i (v_i - vhat_i) + dt sum_c (sum_k V_{c,k} P_k(F_{c,k}) S_{c,k}^T) grad w_ic
// (the gradient of Phi, i.e. M(v - vhat) - dt f_int).  Fixed components and
// massless nodes get a zero gradient, and the kinetic sum runs over the free
// components.  energy = +inf if any F_{c,k} leaves the model's
// domain (det F <= 0 for Neo-Hookean / Hencky).
int or_energy_grad(const or_grid* gg, int32_t nmat, const or_material* mats, double dt,
                   const double* mi, const double* vhat, const uint8_t* fixed,
                   const double* Vck, const double* Sck, const double* v,
                   double* energy, double* grad) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc(), nn = g.nn();
  std::vector<double> ec(nc, 0.0), Q(9 * nc, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; ++c) {
    bool any = false;
    for (int k = 0; k < nmat; ++k) any = any || (Vck[k * nc + c] != 0.0);
    if (!any) continue;
    int i = (int)(c / ((int64_t)g.n * g.n)), j = (int)((c / g.n) % g.n), kk = (int)(c % g.n);
    double Gm[9];
    cell_velocity_gradient(g, i, j, kk, v, Gm);
    for (int k = 0; k < nmat; ++k) {
      double Vv = Vck[k * nc + c];
      if (Vv == 0.0) continue;
      const double* S = Sck + (k * nc + c) * 9;
      double A[9] = {1.0 + dt * Gm[0], dt * Gm[1], dt * Gm[2], dt * Gm[3], 1.0 + dt * Gm[4],
                     dt * Gm[5], dt * Gm[6], dt * Gm[7], 1.0 + dt * Gm[8]};
      double Fm[9];
      m3_mul(A, S, Fm);
      double e = psi_any(&mats[k], Fm);
      ec[c] += Vv * e;
      if (!std::isfinite(e)) continue;
      double P[9], St[9], PS[9];
      piola_any(&mats[k], Fm, P);
      m3_transpose(S, St);
      m3_mul(P, St, PS);
      for (int q = 0; q < 9; ++q) Q[9 * c + q] += Vv * PS[q];
    }
  }
  double E = 0.0;
  for (int64_t c = 0; c < nc; ++c) E += ec[c];
  for (int64_t nidx = 0; nidx < nn; ++nidx) {
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
      if (!dof_free(mi, fixed, nidx, a)) continue;
      double dv = v[3 * nidx + a] - vhat[3 * nidx + a];
      s += dv * dv;
    }
    E += 0.5 * mi[nidx] * s;
  }
  *energy = E;
  if (grad) {
    for (int64_t nidx = 0; nidx < nn; ++nidx)
      for (int a = 0; a < 3; ++a) grad[3 * nidx + a] = 0.0;
    for (int i = 0; i < g.n; ++i)
      for (int j = 0; j < g.n; ++j)
        for (int kk = 0; kk < g.n; ++kk) {
          int64_t c = g.cell(i, j, kk);
          const double* Qc = Q.data() + 9 * c;
          for (int d = 0; d < 8; ++d) {
            int o[3];
            corner(d, o);
            int64_t nidx = g.node(i + o[0], j + o[1], kk + o[2]);
            double gw[3];
            grad_w(d, g.dx, gw);
            for (int a = 0; a < 3; ++a)
              grad[3 * nidx + a] += dt * (Qc[a * 3 + 0] * gw[0] + Qc[a * 3 + 1] * gw[1] + Qc[a * 3 + 2] * gw[2]);
          }
        }
    for (int64_t nidx = 0; nidx < nn; ++nidx)
      for (int a = 0; a < 3; ++a) {
        if (!dof_free(mi, fixed, nidx, a)) {
          grad[3 * nidx + a] = 0.0;
          continue;
        }
        grad[3 * nidx + a] += mi[nidx] * (v[3 * nidx + a] - vhat[3 * nidx + a]);
      }
  }
  return std::isfinite(E) ? OR_OK : OR_ERR_DOMAIN;
}

// Per-cell tangent in velocity-gradient space:
//   Abar_c = dt^2 sum_k V_{c,k} Shat_k^T [dP_k/dF(F_{c,k})]_+ Shat_k,
// where Shat maps vec(dG) to vec(dG S) (dF = dt dG S) and [.]_+ clamps the
// negative eigenvalues of the 9x9 model tangent (project = 1) or leaves it
// as is (project = 0).  Abar is 81 doubles per cell, row-major over
// (a*3+b, a'*3+b').
int or_tangent(const or_grid* gg, int32_t nmat, const or_material* mats, double dt,
               const double* Vck, const double* Sck, const double* v, int32_t project,
               double* Abar) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc();
  int status = OR_OK;
#pragma omp parallel for schedule(dynamic, 64) reduction(min : status)
  for (int64_t c = 0; c < nc; ++c) {
    double* Ac = Abar + 81 * c;
    for (int e = 0; e < 81; ++e) Ac[e] = 0.0;
    bool any = false;
    for (int k = 0; k < nmat; ++k) any = any || (Vck[k * nc + c] != 0.0);
    if (!any) continue;
    int i = (int)(c / ((int64_t)g.n * g.n)), j = (int)((c / g.n) % g.n), kk = (int)(c % g.n);
    double Gm[9];
    cell_velocity_gradient(g, i, j, kk, v, Gm);
    for (int k = 0; k < nmat; ++k) {
      double Vv = Vck[k * nc + c];
      if (Vv == 0.0) continue;
      const double* S = Sck + (k * nc + c) * 9;
      double Am[9] = {1.0 + dt * Gm[0], dt * Gm[1], dt * Gm[2], dt * Gm[3], 1.0 + dt * Gm[4],
                      dt * Gm[5], dt * Gm[6], dt * Gm[7], 1.0 + dt * Gm[8]};
      double Fm[9];
      m3_mul(Am, S, Fm);
      double T[81];
      int st = dpdf_any(&mats[k], Fm, T);
      if (st != OR_OK) { status = std::min(status, st); continue; }
      if (project) project_psd(9, T);
      double Sh[81] = {0};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          for (int dd = 0; dd < 3; ++dd) Sh[(a * 3 + b) * 9 + (a * 3 + dd)] = S[dd * 3 + b];
      double TS[81];
      for (int r = 0; r < 9; ++r)
        for (int cc = 0; cc < 9; ++cc) {
          double s = 0.0;
          for (int q = 0; q < 9; ++q) s += T[r * 9 + q] * Sh[q * 9 + cc];
          TS[r * 9 + cc] = s;
        }
      for (int r = 0; r < 9; ++r)
        for (int cc = 0; cc < 9; ++cc) {
          double s = 0.0;
          for (int q = 0; q < 9; ++q) s += Sh[q * 9 + r] * TS[q * 9 + cc];
          Ac[r * 9 + cc] += dt * dt * Vv * s;
        }
    }
  }
  return status;
}

// Matrix-free product with the Hessian H = M + sum_c B_c^T Abar_c B_c on the
// free DOFs: dG_c(u) = sum_i u_i (x) grad w_ic, y_c = Abar_c vec(dG_c),
// (Hu)_i = m_i u_i + sum_c Y_c grad w_ic.  u is read as zero on fixed
// components and massless nodes, and Hu is zero there.
int or_hv(const or_grid* gg, const double* mc, const double* mi, const uint8_t* fixed,
          const double* Abar, const double* u, double* Hu) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc(), nn = g.nn();
  std::vector<double> um(3 * nn, 0.0), Y(9 * nc, 0.0);
  for (int64_t nidx = 0; nidx < nn; ++nidx)
    for (int a = 0; a < 3; ++a)
      if (dof_free(mi, fixed, nidx, a)) um[3 * nidx + a] = u[3 * nidx + a];
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; ++c) {
    if (mc[c] == 0.0) continue;
    int i = (int)(c / ((int64_t)g.n * g.n)), j = (int)((c / g.n) % g.n), kk = (int)(c % g.n);
    double dG[9];
    cell_velocity_gradient(g, i, j, kk, um.data(), dG);
    const double* Ac = Abar + 81 * c;
    for (int r = 0; r < 9; ++r) {
      double s = 0.0;
      for (int q = 0; q < 9; ++q) s += Ac[r * 9 + q] * dG[q];
      Y[9 * c + r] = s;
    }
  }
  for (int64_t nidx = 0; nidx < nn; ++nidx)
    for (int a = 0; a < 3; ++a) Hu[3 * nidx + a] = 0.0;
  for (int i = 0; i < g.n; ++i)
    for (int j = 0; j < g.n; ++j)
      for (int kk = 0; kk < g.n; ++kk) {
        int64_t c = g.cell(i, j, kk);
        if (mc[c] == 0.0) continue;
        const double* Yc = Y.data() + 9 * c;
        for (int d = 0; d < 8; ++d) {
          int o[3];
          corner(d, o);
          int64_t nidx = g.node(i + o[0], j + o[1], kk + o[2]);
          double gw[3];
          grad_w(d, g.dx, gw);
          for (int a = 0; a < 3; ++a)
            Hu[3 * nidx + a] += Yc[a * 3 + 0] * gw[0] + Yc[a * 3 + 1] * gw[1] + Yc[a * 3 + 2] * gw[2];
        }
      }
  for (int64_t nidx = 0; nidx < nn; ++nidx)
    for (int a = 0; a < 3; ++a)
      Hu[3 * nidx + a] = dof_free(mi, fixed, nidx, a) ? Hu[3 * nidx + a] + mi[nidx] * um[3 * nidx + a] : 0.0;
  return OR_OK;
}

// Explicit internal force (Sec. 4 opening): f_i = -sum_c sum_k V_{c,k} tau_{c,k} grad w_ic.
int or_explicit_force(const or_grid* gg, int32_t nmat, const double* Vck,
                      const double* tauck, double* f) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc(), nn = g.nn();
  for (int64_t nidx = 0; nidx < 3 * nn; ++nidx) f[nidx] = 0.0;
  for (int i = 0; i < g.n; ++i)
    for (int j = 0; j < g.n; ++j)
      for (int kk = 0; kk < g.n; ++kk) {
        int64_t c = g.cell(i, j, kk);
        for (int k = 0; k < nmat; ++k) {
          double Vv = Vck[k * nc + c];
          if (Vv == 0.0) continue;
          const double* T = tauck + (k * nc + c) * 9;
          for (int d = 0; d < 8; ++d) {
            int o[3];
            corner(d, o);
            int64_t nidx = g.node(i + o[0], j + o[1], kk + o[2]);
            double gw[3];
            grad_w(d, g.dx, gw);
            for (int a = 0; a < 3; ++a)
              f[3 * nidx + a] -= Vv * (T[a * 3 + 0] * gw[0] + T[a * 3 + 1] * gw[1] + T[a * 3 + 2] * gw[2]);
          }
        }
      }
  return OR_OK;
}

int or_plastic_base(const or_grid* gg, int32_t nmat, const or_material* mats, double dt,
                    const double* Vck, const double* S0, const double* v, double* Seff) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc();
  int status = OR_OK;
#pragma omp parallel for schedule(static) reduction(min : status)
  for (int64_t c = 0; c < nc; ++c) {
    int i = (int)(c / ((int64_t)g.n * g.n)), j = (int)((c / g.n) % g.n), kk = (int)(c % g.n);
    bool need = false;
    for (int k = 0; k < nmat; ++k)
      need = need || (Vck[k * nc + c] != 0.0 && mats[k].plastic != OR_PLASTIC_NONE);
    double A[9], Ai[9];
    if (need) {
      double Gm[9];
      cell_velocity_gradient(g, i, j, kk, v, Gm);
      for (int e = 0; e < 9; ++e) A[e] = dt * Gm[e];
      A[0] += 1.0; A[4] += 1.0; A[8] += 1.0;
      if (!m3_inverse(A, Ai)) need = false, status = std::min(status, (int)OR_ERR_DOMAIN);
    }
    for (int k = 0; k < nmat; ++k) {
      const double* S = S0 + (k * nc + c) * 9;
      double* Se = Seff + (k * nc + c) * 9;
      for (int e = 0; e < 9; ++e) Se[e] = S[e];
      if (!need || Vck[k * nc + c] == 0.0 || mats[k].plastic == OR_PLASTIC_NONE) continue;
      double F[9];
      m3_mul(A, S, F);
      double inc = 0.0;
      int st = plastic_project(&mats[k], F, &inc);
      if (st != OR_OK) { status = std::min(status, st); continue; }
      if (inc > 0.0) m3_mul(Ai, F, Se);
    }
  }
  return status;
}

// Vertex block descent (Sec. 5, VBD) on Phi: see or_solver_opts.vbd_sweeps.
static int vbd_solve(const or_grid* gg, int32_t nmat, const or_material* mats, double dt,
                     const double* mi, const double* vhat, const uint8_t* fixed,
                     const double* Vck, const double* Sck, int sweeps, double* v,
                     or_solver_stats* stats) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc(), nn = g.nn();
  std::vector<double> grad(3 * nn), Abar(81 * nc);
  for (int64_t i = 0; i < 3 * nn; ++i) v[i] = vhat[i];
  double E = 0.0;
  int rc = or_energy_grad(gg, nmat, mats, dt, mi, vhat, fixed, Vck, Sck, v, &E, grad.data());
  if (rc != OR_OK) return rc;
  auto gnorm = [&]() {
    double s = 0.0;
    for (int64_t i = 0; i < 3 * nn; ++i) s += grad[i] * grad[i];
    return std::sqrt(s);
  };
  or_solver_stats st{};
  st.g0_norm = gnorm();
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int color = 0; color < 8; ++color) {
      rc = or_energy_grad(gg, nmat, mats, dt, mi, vhat, fixed, Vck, Sck, v, &E, grad.data());
      if (rc != OR_OK) return rc;
      rc = or_tangent(gg, nmat, mats, dt, Vck, Sck, v, 1, Abar.data());
      if (rc != OR_OK) return rc;
      for (int i = 0; i <= g.n; ++i)
        for (int j = 0; j <= g.n; ++j)
          for (int k = 0; k <= g.n; ++k) {
            if ((((i & 1) << 2) | ((j & 1) << 1) | (k & 1)) != color) continue;
            const int64_t nidx = g.node(i, j, k);
            if (mi[nidx] == 0.0 || fixed[nidx] == 7) continue;
            double H[9] = {mi[nidx], 0, 0, 0, mi[nidx], 0, 0, 0, mi[nidx]};
            // the node is corner d = ((i-ci), (j-cj), (k-ck)) of each adjacent cell
            for (int d = 0; d < 8; ++d) {
              int o[3];
              corner(d, o);
              const int ci = i - o[0], cj = j - o[1], ck = k - o[2];
              if (ci < 0 || cj < 0 || ck < 0 || ci >= g.n || cj >= g.n || ck >= g.n) continue;
              const double* Ac = Abar.data() + 81 * g.cell(ci, cj, ck);
              double gw[3];
              grad_w(d, g.dx, gw);
              for (int a = 0; a < 3; ++a)
                for (int a2 = 0; a2 < 3; ++a2) {
                  double s = 0.0;
                  for (int b = 0; b < 3; ++b)
                    for (int b2 = 0; b2 < 3; ++b2) s += Ac[(a * 3 + b) * 9 + (a2 * 3 + b2)] * gw[b] * gw[b2];
                  H[a * 3 + a2] += s;
                }
            }
            // Newton on the free components only (the gradient is 0 on the
            // fixed ones; their row and column become the identity's)
            for (int a = 0; a < 3; ++a)
              if (!dof_free(mi, fixed, nidx, a))
                for (int a2 = 0; a2 < 3; ++a2) H[3 * a + a2] = H[3 * a2 + a] = (a == a2) ? 1.0 : 0.0;
            double Hi[9];
            if (!m3_inverse(H, Hi)) return OR_ERR_NOT_CONVERGED;
            for (int a = 0; a < 3; ++a)
              v[3 * nidx + a] -= Hi[a * 3] * grad[3 * nidx] + Hi[a * 3 + 1] * grad[3 * nidx + 1] +
                                 Hi[a * 3 + 2] * grad[3 * nidx + 2];
          }
    }
  }
  rc = or_energy_grad(gg, nmat, mats, dt, mi, vhat, fixed, Vck, Sck, v, &E, grad.data());
  st.newton_iters = sweeps;
  st.g_norm = gnorm();
  st.energy = E;
  if (stats) *stats = st;
  return rc;
}

// Newton's method on Phi with the projected Hessian, Jacobi- or 3x3
// block-Jacobi-preconditioned CG
// for each linear system and Armijo backtracking (halving, with a rounding
// allowance) and the model's feasibility (Phi = +inf outside the domain).
//   stop Newton when |g_free| <= newton_rtol * |g_free(vhat)|,
//   stop CG when |b - H x| <= pcg_rtol * |b| (both 2-norms over free DOFs).
// Diagonal of H = M + sum_c B_c^T Abar_c B_c on free DOFs (0 elsewhere):
// entry (i, a) = m_i + sum over the cells c around node i of
// sum_{b, b'} Abar_c[(a, b), (a, b')] dw_ic/dx_b dw_ic/dx_b'.
int or_jacobi_diag(const or_grid* gg, const double* mc, const double* mi, const uint8_t* fixed,
                   const double* Abar, double* D) {
  Grid g{gg->n, gg->dx};
  const int64_t nn = g.nn();
  std::fill(D, D + 3 * nn, 0.0);
  for (int i = 0; i < g.n; ++i)
    for (int j = 0; j < g.n; ++j)
      for (int kk = 0; kk < g.n; ++kk) {
        int64_t c = g.cell(i, j, kk);
        if (mc[c] == 0.0) continue;
        const double* Ac = Abar + 81 * c;
        for (int d = 0; d < 8; ++d) {
          int o[3];
          corner(d, o);
          int64_t nidx = g.node(i + o[0], j + o[1], kk + o[2]);
          double gw[3];
          grad_w(d, g.dx, gw);
          for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int b = 0; b < 3; ++b)
              for (int b2 = 0; b2 < 3; ++b2) s += Ac[(a * 3 + b) * 9 + (a * 3 + b2)] * gw[b] * gw[b2];
            D[3 * nidx + a] += s;
          }
        }
      }
  for (int64_t nidx = 0; nidx < nn; ++nidx)
    for (int a = 0; a < 3; ++a) {
      D[3 * nidx + a] = dof_free(mi, fixed, nidx, a) ? D[3 * nidx + a] + mi[nidx] : 0.0;
    }
  return OR_OK;
}

// 3x3 nodal block-Jacobi preconditioner: the inverse of each free node's
// diagonal 3x3 block of H = M + sum_c B_c^T Abar_c B_c (the coupling of the
// node's three velocity components with each other; Jacobi keeps only its
// diagonal),
//   H_ii[a][a'] = m_i delta_aa'
//               + sum_c sum_{b,b'} Abar_c[(a,b),(a',b')] dw_ic/dx_b dw_ic/dx_b',
// and 0 on massless nodes.  On a node with fixed components the block is that
// of its free components (the inverse is 0 in the fixed rows and columns).
// Binv: [nnode][9], row-major.
int or_block_jacobi(const or_grid* gg, const double* mc, const double* mi, const uint8_t* fixed,
                    const double* Abar, double* Binv) {
  Grid g{gg->n, gg->dx};
  const int64_t nn = g.nn();
  std::vector<double> H(9 * nn, 0.0);
  for (int i = 0; i < g.n; ++i)
    for (int j = 0; j < g.n; ++j)
      for (int kk = 0; kk < g.n; ++kk) {
        int64_t c = g.cell(i, j, kk);
        if (mc[c] == 0.0) continue;
        const double* Ac = Abar + 81 * c;
        for (int d = 0; d < 8; ++d) {
          int o[3];
          corner(d, o);
          int64_t nidx = g.node(i + o[0], j + o[1], kk + o[2]);
          double gw[3];
          grad_w(d, g.dx, gw);
          for (int a = 0; a < 3; ++a)
            for (int a2 = 0; a2 < 3; ++a2) {
              double s = 0.0;
              for (int b = 0; b < 3; ++b)
                for (int b2 = 0; b2 < 3; ++b2) s += Ac[(a * 3 + b) * 9 + (a2 * 3 + b2)] * gw[b] * gw[b2];
              H[9 * nidx + 3 * a + a2] += s;
            }
        }
      }
  int status = OR_OK;
  for (int64_t nidx = 0; nidx < nn; ++nidx) {
    double* Bi = Binv + 9 * nidx;
    std::fill(Bi, Bi + 9, 0.0);
    if (mi[nidx] == 0.0 || fixed[nidx] == 7) continue;
    double* Hn = H.data() + 9 * nidx;
    for (int a = 0; a < 3; ++a) Hn[4 * a] += mi[nidx];
    // the block of the free components: a fixed component's row and column
    // become those of the identity, and its row and column of the inverse 0
    for (int a = 0; a < 3; ++a)
      if (!dof_free(mi, fixed, nidx, a))
        for (int a2 = 0; a2 < 3; ++a2) Hn[3 * a + a2] = Hn[3 * a2 + a] = (a == a2) ? 1.0 : 0.0;
    if (!m3_inverse(Hn, Bi)) status = OR_ERR_DOMAIN;
    for (int a = 0; a < 3; ++a)
      if (!dof_free(mi, fixed, nidx, a))
        for (int a2 = 0; a2 < 3; ++a2) Bi[3 * a + a2] = Bi[3 * a2 + a] = 0.0;
  }
  return status;
}

int or_solve(const or_grid* gg, int32_t nmat, const or_material* mats, double dt,
             const double* mc, const double* mi, const double* vhat, const uint8_t* fixed,
             const double* Vck, const double* S0, const or_solver_opts* opts,
             double* v, or_solver_stats* stats) {
  if (opts->vbd_sweeps > 0)
    return vbd_solve(gg, nmat, mats, dt, mi, vhat, fixed, Vck, S0, opts->vbd_sweeps, v, stats);
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc(), nn = g.nn(), nd = 3 * nn;
  std::vector<double> grad(nd), Abar(81 * nc), p(nd), r(nd), z(nd), q(nd), x(nd), D(nd),
      vt(nd), dir(nd), Binv(opts->block_jacobi ? 9 * nn : 0);
  for (int64_t i = 0; i < nd; ++i) v[i] = vhat[i];
  // the base the energy uses: S0, or with fixed-point plasticity the
  // return-mapped base of the current iterate (re-projected after every step)
  std::vector<double> Seff(S0, S0 + 9 * (size_t)nmat * nc);
  const double* Sck = Seff.data();
  auto reproject = [&]() {
    return opts->fixed_point_plasticity
               ? or_plastic_base(gg, nmat, mats, dt, Vck, S0, v, Seff.data())
               : (int)OR_OK;
  };
  or_solver_stats st{};
  double E;
  if (int rp = reproject(); rp != OR_OK) return rp;
  int rc = or_energy_grad(gg, nmat, mats, dt, mi, vhat, fixed, Vck, Sck, v, &E, grad.data());
  if (rc != OR_OK) return rc;
  auto dot = [&](const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for (int64_t i = 0; i < nd; ++i) s += a[i] * b[i];
    return s;
  };
  double g0 = std::sqrt(dot(grad, grad));
  st.g0_norm = g0;
  double escale = 0.0;  // energy rounding scale: sum V (mu + |lambda|)
  for (int k = 0; k < nmat; ++k)
    for (int64_t c = 0; c < nc; ++c)
      escale += Vck[k * nc + c] * (mats[k].mu + std::fabs(mats[k].lambda));
  double gn = g0;
  int result = OR_OK;
  for (int it = 0;; ++it) {
    if (gn == 0.0 || gn <= opts->newton_rtol * g0) break;
    if (it >= opts->max_newton) { result = OR_ERR_NOT_CONVERGED; break; }
    or_tangent(gg, nmat, mats, dt, Vck, Sck, v, 1, Abar.data());
    // preconditioner: the diagonal of H (Jacobi) or its inverted 3x3 node
    // blocks (block-Jacobi); z = P r
    or_jacobi_diag(gg, mc, mi, fixed, Abar.data(), D.data());
    if (opts->block_jacobi) {
      if (int rb = or_block_jacobi(gg, mc, mi, fixed, Abar.data(), Binv.data()); rb != OR_OK) {
        result = rb;
        break;
      }
    }
    auto precondition = [&]() {
      if (opts->block_jacobi) {
        for (int64_t n = 0; n < nn; ++n)
          for (int a = 0; a < 3; ++a)
            z[3 * n + a] = Binv[9 * n + 3 * a] * r[3 * n] + Binv[9 * n + 3 * a + 1] * r[3 * n + 1] +
                           Binv[9 * n + 3 * a + 2] * r[3 * n + 2];
      } else {
        for (int64_t i = 0; i < nd; ++i) z[i] = D[i] > 0.0 ? r[i] / D[i] : 0.0;
      }
    };
    // CG on H x = -g
    for (int64_t i = 0; i < nd; ++i) {
      x[i] = 0.0;
      r[i] = -grad[i];
    }
    precondition();
    for (int64_t i = 0; i < nd; ++i) p[i] = z[i];
    double bn = std::sqrt(dot(r, r));
    double rz = dot(r, z);
    int k = 0;
    for (; k < opts->max_pcg; ++k) {
      or_hv(gg, mc, mi, fixed, Abar.data(), p.data(), q.data());
      double pq = dot(p, q);
      if (!(pq > 0.0)) break;
      double alpha = rz / pq;
      for (int64_t i = 0; i < nd; ++i) {
        x[i] += alpha * p[i];
        r[i] -= alpha * q[i];
      }
      if (std::sqrt(dot(r, r)) <= opts->pcg_rtol * bn) { ++k; break; }
      precondition();
      double rz2 = dot(r, z);
      double beta = rz2 / rz;
      rz = rz2;
      for (int64_t i = 0; i < nd; ++i) p[i] = z[i] + beta * p[i];
    }
    st.pcg_iters_total += k;
    // Backtracking line search on Phi.
    double gtp = dot(grad, x);
    double allowance = 1e-14 * escale + 1e-13 * std::fabs(E);
    double alpha = 1.0, Et = kInf;
    int ls = 0;
    bool ok = false;
    for (; ls <= opts->max_ls; ++ls) {
      for (int64_t i = 0; i < nd; ++i) vt[i] = v[i] + alpha * x[i];
      int rc2 = or_energy_grad(gg, nmat, mats, dt, mi, vhat, fixed, Vck, Sck, vt.data(), &Et, nullptr);
      // Armijo sufficient decrease, with an allowance for the rounding of
      // the energy: each psi is a difference of O(mu + |lambda|) terms, so
      // the allowance is 1e-14 sum_{c,k} V_{c,k} (mu_k + |lambda_k|) plus
      // 1e-13 |Phi| (near the minimiser the predicted decrease falls below
      // the energy's own rounding error).
      if (rc2 == OR_OK && std::isfinite(Et) &&
          Et <= E + opts->armijo_c * alpha * gtp + allowance) { ok = true; break; }
      alpha *= 0.5;
    }
    st.ls_halvings += ls;
    st.newton_iters = it + 1;
    if (!ok) { result = OR_ERR_LINESEARCH; break; }
    for (int64_t i = 0; i < nd; ++i) v[i] = vt[i];
    if (int rp = reproject(); rp != OR_OK) { result = rp; break; }
    or_energy_grad(gg, nmat, mats, dt, mi, vhat, fixed, Vck, Sck, v, &E, grad.data());
    gn = std::sqrt(dot(grad, grad));
  }
  st.g_norm = gn;
  st.energy = E;
  if (stats) *stats = st;
  return result;
}

// Alg. 4, first loop: v_c = sum_i w_ic v_i, G_c = sum_i v_i (x) grad w_ic on
// cells with m_c != 0 (others are left at zero).
int or_node_to_centre(const or_grid* gg, const double* mc, const double* vnode,
                      double* vc, double* Gc) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc();
  for (int64_t c = 0; c < nc; ++c) {
    for (int a = 0; a < 3; ++a) vc[3 * c + a] = 0.0;
    for (int e = 0; e < 9; ++e) Gc[9 * c + e] = 0.0;
    if (mc[c] == 0.0) continue;
    int i = (int)(c / ((int64_t)g.n * g.n)), j = (int)((c / g.n) % g.n), kk = (int)(c % g.n);
    for (int d = 0; d < 8; ++d) {
      int o[3];
      corner(d, o);
      const double* vn = vnode + 3 * g.node(i + o[0], j + o[1], kk + o[2]);
      for (int a = 0; a < 3; ++a) vc[3 * c + a] += vn[a] / 8.0;
    }
    cell_velocity_gradient(g, i, j, kk, vnode, Gc + 9 * c);
  }
  return OR_OK;
}

// Alg. 4: sample v, G at the centres, interpolate to particles with the same
// w_cp as the unload (positions x^n), advect, F <- (I + dt G_p) F, then the
// plastic projection of F (applied after the update, semi-implicitly).
// Alg. 4 for the particles, given the centre fields of the new velocity
// (vc, Gc) and, for the FLIP/PIC transfer (Sec. 3, Degradation to FLIP/PIC),
// the centre field dvc of the node velocity increment (NULL for APIC).
static int load_particles(const Grid& g, double dt, const double* vc, const double* Gc,
                          const double* dvc, double flip, int64_t np, const int32_t* mat,
                          const or_material* mats, double* x, double* v, double* G, double* F,
                          double* eps_acc) {
  int status = OR_OK;
  for (int64_t p = 0; p < np; ++p) {
    Stencil s;
    if (!make_stencil(g, x + 3 * p, &s)) return OR_ERR_OUTSIDE;
    double vp[3] = {0, 0, 0}, Gp[9] = {0}, dvp[3] = {0, 0, 0};
    for (int d = 0; d < 8; ++d) {
      int o[3];
      corner(d, o);
      int64_t c = g.cell(s.b[0] + o[0], s.b[1] + o[1], s.b[2] + o[2]);
      double w = stencil_weight(s, d);
      if (w == 0.0) continue;
      for (int a = 0; a < 3; ++a) vp[a] += w * vc[3 * c + a];
      for (int e = 0; e < 9; ++e) Gp[e] += w * Gc[9 * c + e];
      if (dvc)
        for (int a = 0; a < 3; ++a) dvp[a] += w * dvc[3 * c + a];
    }
    for (int a = 0; a < 3; ++a) {
      // APIC: v_p is the interpolated new velocity.  FLIP/PIC: the PIC
      // velocity vp advects, the particle keeps flip (v_p + dv_p) + (1 - flip) vp
      v[3 * p + a] = dvc ? flip * (v[3 * p + a] + dvp[a]) + (1.0 - flip) * vp[a] : vp[a];
      x[3 * p + a] += dt * vp[a];
    }
    for (int e = 0; e < 9; ++e) G[9 * p + e] = Gp[e];
    double A[9] = {1.0 + dt * Gp[0], dt * Gp[1], dt * Gp[2], dt * Gp[3], 1.0 + dt * Gp[4],
                   dt * Gp[5], dt * Gp[6], dt * Gp[7], 1.0 + dt * Gp[8]};
    if (mats[mat[p]].model == OR_WATER) {
      // Sec. 3, Water: J^{n+1} = (1 + dt tr G_p) J^n, carried as F = J^{1/3} I
      double Jn = (1.0 + dt * (Gp[0] + Gp[4] + Gp[8])) * m3_det(F + 9 * p);
      if (!(Jn > 0.0)) {
        status = OR_ERR_DOMAIN;
        continue;
      }
      double c = std::cbrt(Jn);
      for (int e = 0; e < 9; ++e) F[9 * p + e] = (e % 4 == 0) ? c : 0.0;
      continue;
    }
    m3_mul(A, F + 9 * p, F + 9 * p);
    int st = plastic_project(&mats[mat[p]], F + 9 * p, eps_acc ? eps_acc + p : nullptr);
    if (st != OR_OK) status = st;
  }
  return status;
}

int or_load(const or_grid* gg, double dt, const double* mc, const double* vnode,
            int64_t np, const int32_t* mat, const or_material* mats,
            double* x, double* v, double* G, double* F, double* eps_acc) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc();
  std::vector<double> vc(3 * nc), Gc(9 * nc);
  or_node_to_centre(gg, mc, vnode, vc.data(), Gc.data());
  return load_particles(g, dt, vc.data(), Gc.data(), nullptr, 0.0, np, mat, mats, x, v, G, F,
                        eps_acc);
}

// Load with the FLIP/PIC transfer (Sec. 3, Degradation to FLIP/PIC): the new
// node velocity and the node increment vnode - vnode_old are both sampled at
// centres and interpolated to the particles; flip in [0, 1] is the FLIP share.
int or_load_flip(const or_grid* gg, double dt, const double* mc, const double* vnode,
                 const double* vnode_old, double flip, int64_t np, const int32_t* mat,
                 const or_material* mats, double* x, double* v, double* G, double* F,
                 double* eps_acc) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc(), nn = g.nn();
  std::vector<double> vc(3 * nc), Gc(9 * nc), dvc(3 * nc), dGc(9 * nc), dv(3 * nn);
  or_node_to_centre(gg, mc, vnode, vc.data(), Gc.data());
  for (int64_t i = 0; i < 3 * nn; ++i) dv[i] = vnode[i] - vnode_old[i];
  or_node_to_centre(gg, mc, dv.data(), dvc.data(), dGc.data());
  return load_particles(g, dt, vc.data(), Gc.data(), dvc.data(), flip, np, mat, mats, x, v, G, F,
                        eps_acc);
}

// Alg. 1: Unload -> Integrate (implicit) -> Load.  External gravity enters
// through vhat = v^n + dt g on free nodes; fixed nodes take their prescribed
// velocity.  The particle arrays are updated in place.
int or_step(const or_grid* gg, int32_t nmat, const or_material* mats, double dt,
            const double gravity[3], int32_t nbc, const or_bc* bcs, double time,
            const or_solver_opts* opts, int64_t np, double* x, double* v, double* G,
            double* F, const double* m, const double* V, const int32_t* mat,
            double* eps_acc, or_solver_stats* stats, double* vnode_out) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc(), nn = g.nn();
  std::vector<double> mc(nc), vc(3 * nc), Gc(9 * nc), Vck(nmat * nc), tauck(9 * nmat * nc),
      mi(nn), vi(3 * nn), Sck(9 * nmat * nc), vhat(3 * nn), vfix(3 * nn), vnew(3 * nn);
  std::vector<uint8_t> fixed(nn);
  int rc = or_unload(gg, np, x, v, G, F, m, V, mat, nmat, mats, mc.data(), vc.data(), Gc.data(),
                     Vck.data(), tauck.data(), mi.data(), vi.data());
  if (rc != OR_OK && rc != OR_ERR_DOMAIN) return rc;
  rc = or_node_bcs(gg, mi.data(), nbc, bcs, time, fixed.data(), vfix.data());
  if (rc != OR_OK) return rc;
  for (int64_t nidx = 0; nidx < nn; ++nidx)
    for (int a = 0; a < 3; ++a)
      vhat[3 * nidx + a] = ((fixed[nidx] >> a) & 1u) ? vfix[3 * nidx + a]
                           : (mi[nidx] != 0.0 ? vi[3 * nidx + a] + dt * gravity[a] : 0.0);
  rc = or_reconstruct(gg, nmat, mats, Vck.data(), tauck.data(), Sck.data());
  if (rc != OR_OK && rc != OR_ERR_DOMAIN) return rc;
  rc = or_solve(gg, nmat, mats, dt, mc.data(), mi.data(), vhat.data(), fixed.data(), Vck.data(),
                Sck.data(), opts, vnew.data(), stats);
  if (rc != OR_OK) return rc;
  if (vnode_out) std::memcpy(vnode_out, vnew.data(), sizeof(double) * 3 * nn);
  return or_load(gg, dt, mc.data(), vnew.data(), np, mat, mats, x, v, G, F, eps_acc);
}

// One explicit step: the Integrate algorithm's explicit branch between the
// unload and the load.  vhat_i = v_i^n + dt gravity on free nodes (the
// prescribed velocity on Dirichlet nodes), then v_i^{n+1} = vhat_i + dt f_i / m_i
// with f_i = -sum_c sum_k V_{c,k} tau_{c,k} grad w_ic (Eq. explicitforce).
int or_step_explicit(const or_grid* gg, int32_t nmat, const or_material* mats, double dt,
                     const double gravity[3], int32_t nbc, const or_bc* bcs, double time,
                     int64_t np, double* x, double* v, double* G, double* F, const double* m,
                     const double* V, const int32_t* mat, double* eps_acc, double* vnode_out) {
  Grid g{gg->n, gg->dx};
  const int64_t nc = g.nc(), nn = g.nn();
  std::vector<double> mc(nc), vc(3 * nc), Gc(9 * nc), Vck(nmat * nc), tauck(9 * nmat * nc),
      mi(nn), vi(3 * nn), vfix(3 * nn), f(3 * nn), vnew(3 * nn);
  std::vector<uint8_t> fixed(nn);
  int rc = or_unload(gg, np, x, v, G, F, m, V, mat, nmat, mats, mc.data(), vc.data(), Gc.data(),
                     Vck.data(), tauck.data(), mi.data(), vi.data());
  if (rc != OR_OK && rc != OR_ERR_DOMAIN) return rc;
  rc = or_node_bcs(gg, mi.data(), nbc, bcs, time, fixed.data(), vfix.data());
  if (rc != OR_OK) return rc;
  or_explicit_force(gg, nmat, Vck.data(), tauck.data(), f.data());
  for (int64_t nidx = 0; nidx < nn; ++nidx)
    for (int a = 0; a < 3; ++a) {
      const int64_t i = 3 * nidx + a;
      if ((fixed[nidx] >> a) & 1u)
        vnew[i] = vfix[i];
      else if (mi[nidx] != 0.0)
        vnew[i] = vi[i] + dt * gravity[a] + dt * f[i] / mi[nidx];
      else
        vnew[i] = 0.0;
    }
  if (vnode_out) std::memcpy(vnode_out, vnew.data(), sizeof(double) * 3 * nn);
  return or_load(gg, dt, mc.data(), vnew.data(), np, mat, mats, x, v, G, F, eps_acc);
}

}  // extern "C"
