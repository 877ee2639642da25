// Dominant Z-eigenpair machinery shared by the per-candidate solver and the
// all-voxel rotation map (Theorem "main"; eq. "Zeigen"): the compile-time
// packed multi-indices of S^n(R^4), lambda(q) = C q^n, the matrix A q^{n-2}
// with its gradient and value, and the safeguarded Newton / shifted power
// (SS-HOPM) iteration on S^3.
#pragma once

#include "ttm_device.h"
#include "ttm_internal.h"

namespace ttm {

constexpr int hidx(int i, int j) { return i * 4 - i * (i - 1) / 2 + (j - i); }   // upper triangle, i <= j

// compile-time packed multi-indices, in the order of alpha_of_dev
struct Alpha {
  int a[4];
};
constexpr Alpha alpha_c(int n, int k) {
  int idx = 0;
  for (int a1 = n; a1 >= 0; --a1)
    for (int a2 = n - a1; a2 >= 0; --a2)
      for (int a3 = n - a1 - a2; a3 >= 0; --a3) {
        if (idx == k) return Alpha{{a1, a2, a3, n - a1 - a2 - a3}};
        ++idx;
      }
  return Alpha{{0, 0, 0, 0}};
}
// packed index of the multi-index (a1, a2, a3, n - a1 - a2 - a3)
constexpr int alpha_pos(int n, int a1, int a2, int a3) {
  int idx = 0;
  for (int b1 = n; b1 >= 0; --b1)
    for (int b2 = n - b1; b2 >= 0; --b2)
      for (int b3 = n - b1 - b2; b3 >= 0; --b3) {
        if (b1 == a1 && b2 == a2 && b3 == a3) return idx;
        ++idx;
      }
  return -1;
}
constexpr double fact_c(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}
// multinomial multiplicity n! / (a1! a2! a3! a4!)
constexpr double mult_c(int n, Alpha a) {
  return fact_c(n) / (fact_c(a.a[0]) * fact_c(a.a[1]) * fact_c(a.a[2]) * fact_c(a.a[3]));
}
constexpr int pair_i(int k) { return k < 4 ? 0 : k < 7 ? 1 : k < 9 ? 2 : 3; }
constexpr int pair_j(int k) { return k < 4 ? k : k < 7 ? k - 3 : k < 9 ? k - 5 : 3; }

// lambda(q) = sum_alpha muA_alpha q^alpha with compile-time exponents and the
// powers of q in registers (the seed scan)
template <int N>
__device__ __forceinline__ double eval_lambda(const double* __restrict__ muA, const double* q) {
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  double pw[4][N + 1];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    pw[d][0] = 1.0;
#pragma unroll
    for (int e = 1; e <= N; ++e) pw[d][e] = pw[d][e - 1] * q[d];
  }
  double l = 0.0;
  static_for<0, K>([&](auto kk) {
    constexpr Alpha A = alpha_c(N, decltype(kk)::value);
    l += muA[decltype(kk)::value] * (pw[0][A.a[0]] * pw[1][A.a[1]]) * (pw[2][A.a[2]] * pw[3][A.a[3]]);
  });
  return l;
}

// H = A x^{n-2} (upper triangle), g = A x^{n-1} = H x and lambda = A x^n = x . g
// for the symmetric tensor with packed entries C: (A x^{n-2})_ij is the sum over
// the multi-indices b of degree n - 2 of mult(b) C[b + e_i + e_j] x^b.  The
// weighted monomials mult(b) x^b are formed first; then each entry C[c] is
// read once and added into every H_ij with c - e_i - e_j >= 0.  Every index is
// a compile-time constant, so all lanes run one instruction stream.
template <int N, class CA>
__device__ __forceinline__ void eval_H(const CA& C, const double* x, double& lam, double* g, double* H) {
  constexpr int NM = N - 2;
  constexpr int KB = (NM + 1) * (NM + 2) * (NM + 3) / 6;
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  double pw[4][NM + 1];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    pw[d][0] = 1.0;
#pragma unroll
    for (int e = 1; e <= NM; ++e) pw[d][e] = pw[d][e - 1] * x[d];
  }
  double m[KB];
  static_for<0, KB>([&](auto bb) {
    constexpr Alpha B = alpha_c(NM, decltype(bb)::value);
    constexpr double mb = mult_c(NM, B);
    m[decltype(bb)::value] = mb * (pw[0][B.a[0]] * pw[1][B.a[1]]) * (pw[2][B.a[2]] * pw[3][B.a[3]]);
  });
  double h[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) h[k] = 0.0;
  // the entries are re-read from LDS on every call rather than held in
  // registers across the solver's iterations
  asm volatile("" ::: "memory");
  static_for<0, K>([&](auto cc) {
    constexpr Alpha G = alpha_c(N, decltype(cc)::value);
    const double c = C[decltype(cc)::value];
    static_for<0, 10>([&](auto kk) {
      constexpr int i = pair_i(decltype(kk)::value), j = pair_j(decltype(kk)::value);
      constexpr int b0 = G.a[0] - (i == 0) - (j == 0), b1 = G.a[1] - (i == 1) - (j == 1);
      constexpr int b2 = G.a[2] - (i == 2) - (j == 2), b3 = G.a[3] - (i == 3) - (j == 3);
      if constexpr (b0 >= 0 && b1 >= 0 && b2 >= 0 && b3 >= 0) {
        constexpr int bi = alpha_pos(NM, b0, b1, b2);
        h[decltype(kk)::value] += c * m[bi];
      }
    });
  });
#pragma unroll
  for (int k = 0; k < 10; ++k) H[k] = h[k];
  lam = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double gi = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) gi += h[i <= j ? hidx(i, j) : hidx(j, i)] * x[j];
    g[i] = gi;
    lam += x[i] * gi;
  }
}

__device__ __forceinline__ double fact_d(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}


// lambda(q) = C q^n = sum_alpha mult(alpha) C_alpha q^alpha, every index a
// compile-time constant (C read through the accessor)
template <int N, class CA>
__device__ __forceinline__ double lambda_at(const CA& C, const double* q) {
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  double pw[4][N + 1];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    pw[d][0] = 1.0;
#pragma unroll
    for (int e = 1; e <= N; ++e) pw[d][e] = pw[d][e - 1] * q[d];
  }
  double l = 0.0;
  static_for<0, K>([&](auto kk) {
    constexpr Alpha A = alpha_c(N, decltype(kk)::value);
    constexpr double mu = mult_c(N, A);
    l += (mu * C[decltype(kk)::value]) * ((pw[0][A.a[0]] * pw[1][A.a[1]]) * (pw[2][A.a[2]] * pw[3][A.a[3]]));
  });
  return l;
}

// From the unit start x, maximise lambda(x) = C x^n on S^3: a Newton step in
// the tangent space is taken when it is an ascent direction and a
// backtracking search along it raises lambda, otherwise the shifted power
// step (which never lowers lambda).  On return x is the last iterate (unit),
// lam = lambda(x); the result says whether the gradient test or the
// stationarity test was met within max_iter iterations.
template <int N, class CA>
__device__ bool eig_polish(const CA& C, double* x, double& lam, int max_iter, double tol) {
  constexpr int n = N;
  bool conv = false;
  double gv[4], Hm[10];
  eval_H<N>(C, x, lam, gv, Hm);
  const double nn1 = (double)(n * (n - 1));
  for (int it = 1; it <= max_iter; ++it) {
    double M[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i; j < 4; ++j) {
        M[i][j] = nn1 * Hm[hidx(i, j)];
        M[j][i] = M[i][j];
      }
    double gnorm = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double gr = n * (gv[i] - lam * x[i]);
      gnorm += gr * gr;
    }
    gnorm = sqrt(gnorm);
    const double scale = fmax(1.0, fabs(lam));
    if (gnorm <= 1e-10 * scale) {
      conv = true;
      break;
    }
    // Newton step in the tangent space of S^3 at x, spanned by the unit
    // quaternions x i, x j, x k (orthonormal, orthogonal to x): with the
    // Riemannian Hessian S = n(n-1) B^T H B - n lambda I_3 and gradient
    // gs = n B^T g of lambda(x) = A x^n on the sphere, xi = -S^-1 gs and the
    // direction is B xi.  Where S is not negative definite it is shifted
    // by its Gershgorin bound, which keeps the step an ascent direction.
    const double Bt[3][4] = {{-x[1], x[0], x[3], -x[2]},
                             {-x[2], -x[3], x[0], x[1]},
                             {-x[3], x[2], -x[1], x[0]}};
    double HB[3][4];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) v += M[i][j] * Bt[k][j];
        HB[k][i] = v;
      }
    double S[3][3], gs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int l = k; l < 3; ++l) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) v += Bt[k][i] * HB[l][i];
        S[k][l] = v - (k == l ? n * lam : 0.0);
        S[l][k] = S[k][l];
      }
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) v += Bt[k][i] * gv[i];
      gs[k] = n * v;
    }
    auto det3 = [&]() {
      return S[0][0] * (S[1][1] * S[2][2] - S[1][2] * S[1][2]) - S[0][1] * (S[0][1] * S[2][2] - S[1][2] * S[0][2]) +
             S[0][2] * (S[0][1] * S[1][2] - S[1][1] * S[0][2]);
    };
    double D = det3();
    const bool nd = S[0][0] < 0.0 && S[0][0] * S[1][1] - S[0][1] * S[0][1] > 0.0 && D < 0.0;
    if (!nd) {
      double mu = -INFINITY;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double r = S[k][k];
#pragma unroll
        for (int l = 0; l < 3; ++l)
          if (l != k) r += fabs(S[k][l]);
        mu = fmax(mu, r);
      }
      mu += 1e-6 * scale;
#pragma unroll
      for (int k = 0; k < 3; ++k) S[k][k] -= mu;
      D = det3();
    }
    double dir[4] = {0.0, 0.0, 0.0, 0.0};
    double slope = 0.0;
    const bool newton = D != 0.0 && isfinite(D);
    if (newton) {
      // xi = -S^-1 gs by the adjugate of the symmetric S
      const double a00 = S[1][1] * S[2][2] - S[1][2] * S[1][2], a01 = S[0][2] * S[1][2] - S[0][1] * S[2][2],
                   a02 = S[0][1] * S[1][2] - S[0][2] * S[1][1], a11 = S[0][0] * S[2][2] - S[0][2] * S[0][2],
                   a12 = S[0][1] * S[0][2] - S[0][0] * S[1][2], a22 = S[0][0] * S[1][1] - S[0][1] * S[0][1];
      const double iD = -1.0 / D;
      const double xi[3] = {iD * (a00 * gs[0] + a01 * gs[1] + a02 * gs[2]),
                            iD * (a01 * gs[0] + a11 * gs[1] + a12 * gs[2]),
                            iD * (a02 * gs[0] + a12 * gs[1] + a22 * gs[2])};
#pragma unroll
      for (int i = 0; i < 4; ++i) dir[i] = Bt[0][i] * xi[0] + Bt[1][i] * xi[1] + Bt[2][i] * xi[2];
      slope = xi[0] * gs[0] + xi[1] * gs[1] + xi[2] * gs[2];
    }
    double y[4], lam_new = -INFINITY, gv2[4], Hm2[10];
    bool moved = false;
    if (newton && slope > 0.0) {
      // Newton ascent direction with backtracking: 1, 1/2, 1/4, ...
      double step = 1.0;
      for (int bt = 0; bt < 8; ++bt, step *= 0.5) {
        double ny = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          y[i] = x[i] + step * dir[i];
          ny += y[i] * y[i];
        }
        ny = 1.0 / sqrt(ny);
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] *= ny;
        eval_H<N>(C, y, lam_new, gv2, Hm2);
        if (lam_new >= lam) {
          moved = true;
          break;
        }
      }
    }
    if (!moved) {
      // shifted power step (SS-HOPM): y = A x^{n-1} + alpha x, with alpha
      // keeping (1/n) A x^n + alpha/2 |x|^2 locally convex (Gershgorin
      // bound on the smallest eigenvalue of A x^{n-2}); it never lowers lambda
      double gmin = INFINITY;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double r = Hm[hidx(i, i)];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j != i) r -= fabs(Hm[i < j ? hidx(i, j) : hidx(j, i)]);
        gmin = fmin(gmin, r);
      }
      const double alpha = fmax(0.0, 1e-6 - (n - 1) * gmin);
      double ny = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        y[i] = gv[i] + alpha * x[i];
        ny += y[i] * y[i];
      }
      ny = 1.0 / sqrt(ny);
#pragma unroll
      for (int i = 0; i < 4; ++i) y[i] *= ny;
      eval_H<N>(C, y, lam_new, gv2, Hm2);
    }
    const double dl = fabs(lam_new - lam);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      x[i] = y[i];
      gv[i] = gv2[i];
    }
#pragma unroll
    for (int i = 0; i < 10; ++i) Hm[i] = Hm2[i];
    lam = lam_new;
    if (dl <= tol * fmax(1.0, fabs(lam)) && gnorm <= 1e-7 * scale) {
      conv = true;
      break;
    }
  }
  return conv;
}

}  // namespace ttm
