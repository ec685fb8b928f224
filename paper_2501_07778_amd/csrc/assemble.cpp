// assemble.cpp — Alg. 1 in Z-ordered QTT form: qtt_assemble_stiffness.
//
// The exact (unrounded) tensor trains are written down on the host from
// 1-D factors, and every intermediate is rounded by the library's own GPU
// rounding.  On a uniform square mesh the element integrals of the Q1
// stiffness with exact 2x2 Gauss quadrature, summed over the 16 vertex
// pairs with shift matrices (the nodal and subdomain
// stiffness equations of Sec. 3.5), equal Kronecker products of three 1-D
// matrices on n = 2^d nodes:
//   S1 = int phi_a' phi_b'   ((1/h) tridiag(-1, 2, -1), end diagonals 1/h)
//   M1 = int phi_a  phi_b    ((h/6) tridiag(1, 4, 1), end diagonals 2h/6)
//   G1 = int phi_a' phi_b    (1/2 (J^T - J) - 1/2 e0e0^T + 1/2 e_{n-1}e_{n-1}^T)
// with the Voigt blocks (y-factor (x) x-factor)
//   K_xx = C11 M1(x)S1 + C33 S1(x)M1      K_yy = C22 S1(x)M1 + C33 M1(x)S1
//   K_xy = C12 G1^T(x)G1 + C33 G1(x)G1^T  K_yx = C12 G1(x)G1^T + C33 G1^T(x)G1
// and z-kron interleaves the digits of the two factors (Z-order, Sec. 3.2).
// The shift matrix J (J[a, a+1] = 1) is an exact rank-2 QTT whose bond
// carries the binary carry of a + 1.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace qtt {
namespace {

// Host tensor train; core k element (a, i, j, b) at a + r0 (i + n (j + m b)).
struct HTT {
  int D = 0;
  std::vector<int> n, m, r;  // r has D+1 entries
  std::vector<std::vector<double>> c;
  bool matrix = false;
  double &at(int k, int a, int i, int j, int b) {
    return c[k][a + (size_t)r[k] * (i + (size_t)n[k] * (j + (size_t)m[k] * b))];
  }
  double get(int k, int a, int i, int j, int b) const {
    return c[k][a + (size_t)r[k] * (i + (size_t)n[k] * (j + (size_t)m[k] * b))];
  }
  void alloc(int k) { c[k].assign((size_t)r[k] * n[k] * m[k] * r[k + 1], 0.0); }
  static HTT make(int D, bool mat) {
    HTT t;
    t.D = D;
    t.matrix = mat;
    t.n.assign(D, 2);
    t.m.assign(D, mat ? 2 : 1);
    t.r.assign(D + 1, 1);
    t.c.resize(D);
    return t;
  }
};

// ---------------------------------------------------------------- 1-D
HTT identity1(int d, int size = 2) {
  HTT t = HTT::make(d, true);
  for (int k = 0; k < d; ++k) {
    t.n[k] = t.m[k] = size;
    t.alloc(k);
    for (int i = 0; i < size; ++i) t.at(k, 0, i, i, 0) = 1.0;
  }
  return t;
}

HTT shift1(int d) {
  HTT t = HTT::make(d, true);
  for (int k = 0; k <= d; ++k) t.r[k] = (k == 0 || k == d) ? 1 : 2;
  for (int k = 0; k < d; ++k) {
    t.alloc(k);
    for (int cin = 0; cin < 2; ++cin) {
      if (k == 0 && cin == 0) continue;  // the carry into the first digit is 1
      for (int a = 0; a < 2; ++a) {
        const int s = a + cin, b = s & 1, cout = s >> 1;
        if (k == d - 1 && cout == 1) continue;  // no overflow past the top digit
        const int ia = (k == 0) ? 0 : cin;
        const int ib = (k == d - 1) ? 0 : cout;
        t.at(k, ia, a, b, ib) = 1.0;
      }
    }
  }
  return t;
}

HTT transpose(const HTT &A) {
  HTT t = A;
  for (int k = 0; k < A.D; ++k) {
    std::swap(t.n[k], t.m[k]);
    t.alloc(k);
    for (int a = 0; a < A.r[k]; ++a)
      for (int i = 0; i < A.n[k]; ++i)
        for (int j = 0; j < A.m[k]; ++j)
          for (int b = 0; b < A.r[k + 1]; ++b) t.at(k, a, j, i, b) = A.get(k, a, i, j, b);
  }
  return t;
}

// e_a e_b^T with a, b in {0, 2^d - 1} chosen by the bits (1 = last)
HTT outer1(int d, int row_bit, int col_bit) {
  HTT t = HTT::make(d, true);
  for (int k = 0; k < d; ++k) {
    t.alloc(k);
    t.at(k, 0, row_bit, col_bit, 0) = 1.0;
  }
  return t;
}

HTT unit1(int d, int bit) {
  HTT t = HTT::make(d, false);
  for (int k = 0; k < d; ++k) {
    t.alloc(k);
    t.at(k, 0, bit, 0, 0) = 1.0;
  }
  return t;
}

HTT ones1(int d) {
  HTT t = HTT::make(d, false);
  for (int k = 0; k < d; ++k) {
    t.alloc(k);
    t.at(k, 0, 0, 0, 0) = t.at(k, 0, 1, 0, 0) = 1.0;
  }
  return t;
}

// sin(omega j), j = 0..2^d-1: the pair (cos phi, sin phi) of the partial
// angle is rotated by omega 2^k j_k at digit k; exact rank 2.
HTT sine1(int d, double omega) {
  HTT t = HTT::make(d, false);
  for (int k = 0; k <= d; ++k) t.r[k] = (k == 0 || k == d) ? 1 : 2;
  for (int k = 0; k < d; ++k) {
    t.alloc(k);
    for (int bit = 0; bit < 2; ++bit) {
      const double th = omega * std::ldexp(1.0, k) * bit;
      const double cs = std::cos(th), sn = std::sin(th);
      // state row (cos, sin) times [[cos, sin], [-sin, cos]]
      const double R[2][2] = {{cs, sn}, {-sn, cs}};
      for (int a = 0; a < 2; ++a) {
        if (k == 0 && a == 1) continue;  // initial state (1, 0)
        for (int b = 0; b < 2; ++b) {
          if (k == d - 1 && b == 0) continue;  // read the sine
          const int ia = (k == 0) ? 0 : a;
          const int ib = (k == d - 1) ? 0 : b;
          t.at(k, ia, bit, 0, ib) = R[a][b];
        }
      }
    }
  }
  return t;
}

// ---------------------------------------------------------------- algebra
HTT add(const std::vector<const HTT *> &terms, const std::vector<double> &coef) {
  const HTT &t0 = *terms[0];
  HTT out = t0;
  const int D = t0.D;
  out.r[0] = 1;
  out.r[D] = 1;
  for (int k = 1; k < D; ++k) {
    int s = 0;
    for (auto *t : terms) s += t->r[k];
    out.r[k] = s;
  }
  if (D == 1) {
    out.alloc(0);
    for (size_t u = 0; u < terms.size(); ++u)
      for (size_t e = 0; e < out.c[0].size(); ++e) out.c[0][e] += coef[u] * terms[u]->c[0][e];
    return out;
  }
  for (int k = 0; k < D; ++k) {
    out.alloc(k);
    int oa = 0, ob = 0;
    for (size_t u = 0; u < terms.size(); ++u) {
      const HTT &t = *terms[u];
      const double s = (k == 0) ? coef[u] : 1.0;
      for (int a = 0; a < t.r[k]; ++a)
        for (int i = 0; i < t.n[k]; ++i)
          for (int j = 0; j < t.m[k]; ++j)
            for (int b = 0; b < t.r[k + 1]; ++b)
              out.at(k, (k == 0) ? 0 : oa + a, i, j, (k == D - 1) ? 0 : ob + b) =
                  s * t.get(k, a, i, j, b);
      oa += t.r[k];
      ob += t.r[k + 1];
    }
  }
  return out;
}

// Z-ordered Kronecker product: X acts on the digits i_k, Y on j_k;
// cores alternate X_k (x) I_{bY} and I_{aX} (x) Y_k, pair index a*b0 + b.
HTT zkron(const HTT &Y, const HTT &X) {
  const int d = X.D;
  HTT t = HTT::make(2 * d, X.matrix);
  for (int k = 0; k < d; ++k) {
    const int a0 = X.r[k], a1 = X.r[k + 1], b0 = Y.r[k], b1 = Y.r[k + 1];
    // X core
    int kc = 2 * k;
    t.n[kc] = X.n[k];
    t.m[kc] = X.m[k];
    t.r[kc] = a0 * b0;
    t.r[kc + 1] = a1 * b0;
    t.alloc(kc);
    for (int a = 0; a < a0; ++a)
      for (int b = 0; b < b0; ++b)
        for (int i = 0; i < X.n[k]; ++i)
          for (int j = 0; j < X.m[k]; ++j)
            for (int c = 0; c < a1; ++c) t.at(kc, a * b0 + b, i, j, c * b0 + b) = X.get(k, a, i, j, c);
    // Y core
    kc = 2 * k + 1;
    t.n[kc] = Y.n[k];
    t.m[kc] = Y.m[k];
    t.r[kc + 1] = a1 * b1;
    t.alloc(kc);
    for (int a = 0; a < a1; ++a)
      for (int b = 0; b < b0; ++b)
        for (int i = 0; i < Y.n[k]; ++i)
          for (int j = 0; j < Y.m[k]; ++j)
            for (int e = 0; e < b1; ++e) t.at(kc, a * b0 + b, i, j, a * b1 + e) = Y.get(k, b, i, j, e);
  }
  return t;
}

// small rank-1 cores in front: result digits = [pre..., t...]
HTT prefix(const std::vector<std::vector<double>> &pre, const std::vector<int> &pn,
           const std::vector<int> &pm, const HTT &t) {
  HTT out;
  out.D = (int)pre.size() + t.D;
  out.matrix = t.matrix;
  for (size_t u = 0; u < pre.size(); ++u) {
    out.n.push_back(pn[u]);
    out.m.push_back(pm[u]);
    out.r.push_back(1);
    out.c.push_back(pre[u]);
  }
  for (int k = 0; k < t.D; ++k) {
    out.n.push_back(t.n[k]);
    out.m.push_back(t.m[k]);
    out.r.push_back(t.r[k]);
    out.c.push_back(t.c[k]);
  }
  out.r.push_back(1);
  return out;
}

// C = A B core by core, pair index a*rB + b
HTT matmat(const HTT &A, const HTT &B) {
  HTT t = HTT::make(A.D, true);
  for (int k = 0; k <= A.D; ++k) t.r[k] = A.r[k] * B.r[k];
  for (int k = 0; k < A.D; ++k) {
    t.n[k] = A.n[k];
    t.m[k] = B.m[k];
    t.alloc(k);
    for (int a = 0; a < A.r[k]; ++a)
      for (int c = 0; c < A.r[k + 1]; ++c)
        for (int i = 0; i < A.n[k]; ++i)
          for (int l = 0; l < A.m[k]; ++l) {
            const double av = A.get(k, a, i, l, c);
            if (av == 0.0) continue;
            for (int b = 0; b < B.r[k]; ++b)
              for (int e = 0; e < B.r[k + 1]; ++e)
                for (int j = 0; j < B.m[k]; ++j)
                  t.at(k, a * B.r[k] + b, i, j, c * B.r[k + 1] + e) += av * B.get(k, b, l, j, e);
          }
  }
  return t;
}

HTT matvec_h(const HTT &A, const HTT &x) {
  HTT t = HTT::make(A.D, false);
  for (int k = 0; k <= A.D; ++k) t.r[k] = A.r[k] * x.r[k];
  for (int k = 0; k < A.D; ++k) {
    t.n[k] = A.n[k];
    t.alloc(k);
    for (int a = 0; a < A.r[k]; ++a)
      for (int c = 0; c < A.r[k + 1]; ++c)
        for (int i = 0; i < A.n[k]; ++i)
          for (int j = 0; j < A.m[k]; ++j) {
            const double av = A.get(k, a, i, j, c);
            if (av == 0.0) continue;
            for (int b = 0; b < x.r[k]; ++b)
              for (int e = 0; e < x.r[k + 1]; ++e)
                t.at(k, a * x.r[k] + b, i, 0, c * x.r[k + 1] + e) += av * x.get(k, b, j, 0, e);
          }
  }
  return t;
}

HTT hadamard(const HTT &x, const HTT &y) {
  HTT t = HTT::make(x.D, false);
  for (int k = 0; k <= x.D; ++k) t.r[k] = x.r[k] * y.r[k];
  for (int k = 0; k < x.D; ++k) {
    t.n[k] = x.n[k];
    t.alloc(k);
    for (int a = 0; a < x.r[k]; ++a)
      for (int b = 0; b < y.r[k]; ++b)
        for (int i = 0; i < x.n[k]; ++i)
          for (int c = 0; c < x.r[k + 1]; ++c)
            for (int e = 0; e < y.r[k + 1]; ++e)
              t.at(k, a * y.r[k] + b, i, 0, c * y.r[k + 1] + e) = x.get(k, a, i, 0, c) * y.get(k, b, i, 0, e);
  }
  return t;
}

HTT diag_matrix(const HTT &x) {
  HTT t = HTT::make(x.D, true);
  t.r = x.r;
  for (int k = 0; k < x.D; ++k) {
    t.n[k] = t.m[k] = x.n[k];
    t.alloc(k);
    for (int a = 0; a < x.r[k]; ++a)
      for (int i = 0; i < x.n[k]; ++i)
        for (int b = 0; b < x.r[k + 1]; ++b) t.at(k, a, i, i, b) = x.get(k, a, i, 0, b);
  }
  return t;
}

HTT diag_of(const HTT &A) {
  HTT t = HTT::make(A.D, false);
  t.r = A.r;
  for (int k = 0; k < A.D; ++k) {
    t.n[k] = A.n[k];
    t.alloc(k);
    for (int a = 0; a < A.r[k]; ++a)
      for (int i = 0; i < A.n[k]; ++i)
        for (int b = 0; b < A.r[k + 1]; ++b) t.at(k, a, i, 0, b) = A.get(k, a, i, i, b);
  }
  return t;
}

double trace(const HTT &A) {
  std::vector<double> v(1, 1.0);
  for (int k = 0; k < A.D; ++k) {
    std::vector<double> w(A.r[k + 1], 0.0);
    for (int a = 0; a < A.r[k]; ++a)
      for (int b = 0; b < A.r[k + 1]; ++b) {
        double s = 0.0;
        for (int i = 0; i < A.n[k]; ++i) s += A.get(k, a, i, i, b);
        w[b] += v[a] * s;
      }
    v.swap(w);
  }
  return v[0];
}

HTT ones_like(const HTT &x) {
  HTT t = HTT::make(x.D, false);
  for (int k = 0; k < x.D; ++k) {
    t.n[k] = x.n[k];
    t.alloc(k);
    for (int i = 0; i < x.n[k]; ++i) t.at(k, 0, i, 0, 0) = 1.0;
  }
  return t;
}

HTT identity_like(const HTT &A) {
  HTT t = HTT::make(A.D, true);
  for (int k = 0; k < A.D; ++k) {
    t.n[k] = t.m[k] = A.n[k];
    t.alloc(k);
    for (int i = 0; i < A.n[k]; ++i) t.at(k, 0, i, i, 0) = 1.0;
  }
  return t;
}

// ---------------------------------------------------------------- GPU round
struct Rounder {
  Arena base;
  hipStream_t s;
  double eps;
  int max_rank_seen = 0;
  qtt_status st = QTT_OK;

  // round t in place with the library's GPU rounding
  bool operator()(HTT &t) {
    if (st != QTT_OK) return false;
    Arena ar = base;
    TTDesc d;
    std::vector<int> caps(t.r.begin(), t.r.end());
    for (int k = 0; k <= t.D; ++k) max_rank_seen = std::max(max_rank_seen, t.r[k]);
    if (!arena_tt(ar, d, t.D, t.n.data(), t.m.data(), caps)) {
      st = fail(QTT_E_CAPACITY, "assembly workspace too small (intermediate rank " +
                                    std::to_string(max_rank_seen) + ")");
      return false;
    }
    RoundWs w;
    if (!round_ws_take(ar, d.v, w)) {
      st = fail(QTT_E_CAPACITY, "assembly workspace too small for rounding (rank " +
                                    std::to_string(max_rank_seen) + ")");
      return false;
    }
    auto chk = [&](hipError_t e, const char *what) {
      if (e != hipSuccess && st == QTT_OK)
        st = fail(QTT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
      return e == hipSuccess;
    };
    for (int k = 0; k < t.D; ++k)
      if (!chk(hipMemcpyAsync(d.v.data + d.v.off[k], t.c[k].data(), sizeof(double) * t.c[k].size(),
                              hipMemcpyHostToDevice, s), "upload"))
        return false;
    if (!chk(upload_ranks(d.v, t.r.data(), s), "ranks")) return false;
    if (!chk(round_tt(d.v, eps, 0, w, s), "round")) return false;
    std::vector<int> r(t.D + 1);
    if (!chk(hipMemcpyAsync(r.data(), d.v.rk, sizeof(int) * (t.D + 1), hipMemcpyDeviceToHost, s), "ranks"))
      return false;
    if (!chk(hipStreamSynchronize(s), "sync")) return false;
    t.r = r;
    for (int k = 0; k < t.D; ++k) {
      t.alloc(k);
      if (!chk(hipMemcpyAsync(t.c[k].data(), d.v.data + d.v.off[k], sizeof(double) * t.c[k].size(),
                              hipMemcpyDeviceToHost, s), "download"))
        return false;
    }
    return chk(hipStreamSynchronize(s), "sync");
  }
};

struct Geometry {
  int d, q;
  const qtt_problem *p;
};

std::vector<double> sel_matrix(int n, int a, int b) {
  std::vector<double> e((size_t)n * n, 0.0);
  e[a + (size_t)n * b] = 1.0;
  return e;
}
std::vector<double> unit_vec(int n, int a) {
  std::vector<double> e(n, 0.0);
  e[a] = 1.0;
  return e;
}
std::vector<double> eye(int n) {
  std::vector<double> e((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) e[i + (size_t)n * i] = 1.0;
  return e;
}

// [component | subdomain (q > 1) | nodes]
HTT with_prefix_matrix(const Geometry &g, std::vector<double> comp, std::vector<double> sub,
                       const HTT &nodes) {
  if (g.q > 1) return prefix({comp, sub}, {2, g.q}, {2, g.q}, nodes);
  return prefix({comp}, {2}, {2}, nodes);
}
HTT with_prefix_vector(const Geometry &g, std::vector<double> comp, std::vector<double> sub,
                       const HTT &nodes) {
  if (g.q > 1) return prefix({comp, sub}, {2, g.q}, {1, 1}, nodes);
  return prefix({comp}, {2}, {1}, nodes);
}

void voigt(const qtt_problem *p, double &c11, double &c12, double &c22, double &c33) {
  if (p->plane_strain) {
    const double lam = p->E * p->nu / ((1.0 + p->nu) * (1.0 - 2.0 * p->nu));
    const double mu = p->E / (2.0 * (1.0 + p->nu));
    c11 = c22 = lam + 2.0 * mu;
    c12 = lam;
    c33 = mu;
  } else {
    c11 = c22 = p->E / (1.0 - p->nu * p->nu);
    c12 = p->nu * c11;
    c33 = p->E / (2.0 * (1.0 + p->nu));
  }
}

void one_d(int d, double h, Rounder &rd, HTT &S1, HTT &M1, HTT &G1) {
  HTT I = identity1(d), J = shift1(d), Jt = transpose(J);
  HTT E0 = outer1(d, 0, 0), En = outer1(d, 1, 1);
  S1 = add({&I, &J, &Jt, &E0, &En}, {2.0 / h, -1.0 / h, -1.0 / h, -1.0 / h, -1.0 / h});
  M1 = add({&I, &J, &Jt, &E0, &En}, {4.0 * h / 6, h / 6, h / 6, -2.0 * h / 6, -2.0 * h / 6});
  G1 = add({&J, &Jt, &E0, &En}, {-0.5, 0.5, -0.5, 0.5});
  rd(S1);
  rd(M1);
  rd(G1);
}

// Edge vectors a, b of subdomain m: the map (s, t) -> x0 + s a + t b of the
// parameter square (a square of side L: a = (L, 0), b = (0, L)).
void edge_vectors(const qtt_square &q, double a[2], double b[2]) {
  const bool given = q.edges[0] != 0.0 || q.edges[1] != 0.0 || q.edges[2] != 0.0 ||
                     q.edges[3] != 0.0;
  a[0] = given ? q.edges[0] : q.side;
  a[1] = given ? q.edges[1] : 0.0;
  b[0] = given ? q.edges[2] : 0.0;
  b[1] = given ? q.edges[3] : q.side;
}

// K_bd = sum_{c,c'} E_cc' (x) I_q (x) K_cc'.  With the affine map A = [a b]
// of the parameter square every element has the Jacobian A / (n - 1), and
// the gradient is grad_x = A^-T grad_(s,t) (Sec. 3.4, exact here: the
// Jacobian is constant).  So K_cc' = |det A| sum_{alpha,beta in {s,t}}
// W_cc'[alpha][beta] S_alpha,beta with W_cc'[al][be] = sum_{p,q}
// C(c,p,c',q) G[p][al] G[q][be], G = A^-T, C the elasticity tensor (test
// component c and derivative p, trial c' and q), and the parameter-domain
// Kronecker factors (1-D matrices at h = 1, their h cancels in 2-D; t
// factor (x) s factor): S_ss = M1 (x) S1, S_tt = S1 (x) M1, S_st (test
// derivative in s, trial in t) = G1^T (x) G1, S_ts = G1 (x) G1^T.  For the
// square (G = I / L) this reduces to K_xx = C11 M1(x)S1 + C33 S1(x)M1 and
// K_xy = C12 G1^T(x)G1 + C33 G1(x)G1^T.
HTT block_stiffness(const Geometry &g, Rounder &rd) {
  double c11, c12, c22, c33;
  voigt(g.p, c11, c12, c22, c33);
  // C(c, p, c', q), indices 0 = x, 1 = y
  double Ct[2][2][2][2] = {};
  Ct[0][0][0][0] = c11;
  Ct[1][1][1][1] = c22;
  Ct[0][0][1][1] = Ct[1][1][0][0] = c12;
  Ct[0][1][0][1] = Ct[0][1][1][0] = Ct[1][0][0][1] = Ct[1][0][1][0] = c33;
  double a[2], b[2];
  edge_vectors(g.p->sub[0], a, b);
  const double det = a[0] * b[1] - a[1] * b[0];
  // G = A^-T with A = [a b] (columns): A^-1 = [[b1, -b0], [-a1, a0]] / det
  const double G[2][2] = {{b[1] / det, -a[1] / det}, {-b[0] / det, a[0] / det}};
  HTT S1, M1, G1;
  one_d(g.d, 1.0, rd, S1, M1, G1);
  HTT G1t = transpose(G1);
  HTT Sst[2][2] = {{zkron(M1, S1), zkron(G1t, G1)}, {zkron(G1, G1t), zkron(S1, M1)}};
  HTT Kc[2][2];
  for (int c = 0; c < 2; ++c)
    for (int cp = 0; cp < 2; ++cp) {
      std::vector<const HTT *> terms;
      std::vector<double> coef;
      for (int al = 0; al < 2; ++al)
        for (int be = 0; be < 2; ++be) {
          double w = 0.0;
          for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) w += Ct[c][p][cp][q] * G[p][al] * G[q][be];
          w *= std::fabs(det);
          if (w == 0.0) continue;
          terms.push_back(&Sst[al][be]);
          coef.push_back(w);
        }
      Kc[c][cp] = add(terms, coef);
      rd(Kc[c][cp]);
    }
  HTT &Kxx = Kc[0][0], &Kxy = Kc[0][1], &Kyx = Kc[1][0], &Kyy = Kc[1][1];
  HTT t00 = with_prefix_matrix(g, sel_matrix(2, 0, 0), eye(g.q), Kxx);
  HTT t01 = with_prefix_matrix(g, sel_matrix(2, 0, 1), eye(g.q), Kxy);
  HTT t10 = with_prefix_matrix(g, sel_matrix(2, 1, 0), eye(g.q), Kyx);
  HTT t11 = with_prefix_matrix(g, sel_matrix(2, 1, 1), eye(g.q), Kyy);
  HTT K = add({&t00, &t01, &t10, &t11}, {1, 1, 1, 1});
  rd(K);
  return K;
}

// nodes of one side as a Z-ordered indicator
HTT side_delta(int d, int side) {
  HTT one = ones1(d);
  if (side == 0) return zkron(one, unit1(d, 0));
  if (side == 1) return zkron(one, unit1(d, 1));
  if (side == 2) return zkron(unit1(d, 0), one);
  return zkron(unit1(d, 1), one);
}

HTT mask_vector(const Geometry &g, Rounder &rd) {
  std::vector<HTT> terms;
  for (int m = 0; m < g.q; ++m) {
    for (int c = 0; c < 2; ++c) {
      HTT node;
      {
        HTT o1 = ones1(g.d);
        node = zkron(o1, o1);
      }
      for (int s = 0; s < 4; ++s) {
        if (!g.p->sub[m].fixed[s][c]) continue;
        HTT one = ones_like(node);
        HTT dl = side_delta(g.d, s);
        HTT f = add({&one, &dl}, {1.0, -1.0});
        node = hadamard(node, f);
        rd(node);
      }
      terms.push_back(with_prefix_vector(g, unit_vec(2, c), unit_vec(g.q, m), node));
    }
  }
  std::vector<const HTT *> ptr;
  std::vector<double> co;
  for (auto &t : terms) {
    ptr.push_back(&t);
    co.push_back(1.0);
  }
  HTT mk = add(ptr, co);
  rd(mk);
  return mk;
}

HTT load_vector(const Geometry &g, Rounder &rd, bool &any) {
  const int d = g.d, n = 1 << d;
  std::vector<HTT> terms;
  for (int m = 0; m < g.q; ++m) {
    // parameter-domain 1-D mass (h = 1/(n-1)); the area element is |det A|
    // and an edge's length element |a| (south, north) or |b| (west, east)
    double a[2], b[2];
    edge_vectors(g.p->sub[m], a, b);
    const double det = std::fabs(a[0] * b[1] - a[1] * b[0]);
    const double la = std::hypot(a[0], a[1]), lb = std::hypot(b[0], b[1]);
    HTT S1, M1, G1;
    one_d(d, 1.0 / (n - 1), rd, S1, M1, G1);
    for (int c = 0; c < 2; ++c) {
      if (g.p->body[c] == 0.0) continue;
      HTT mv = matvec_h(M1, ones1(d));
      rd(mv);
      HTT node = zkron(mv, mv);
      HTT t = with_prefix_vector(g, unit_vec(2, c), unit_vec(g.q, m), node);
      for (auto &v : t.c[0]) v *= g.p->body[c] * det;
      terms.push_back(t);
    }
    for (int u = 0; u < g.p->ntrac; ++u) {
      const qtt_traction &tr = g.p->trac[u];
      if (tr.sub != m) continue;
      std::vector<HTT> sines;
      std::vector<double> co;
      if (tr.constant != 0.0) {
        sines.push_back(ones1(d));
        co.push_back(tr.constant);
      }
      for (int k = 1; k <= tr.nmodes; ++k) {
        if (tr.amp[k - 1] == 0.0) continue;
        sines.push_back(sine1(d, k * M_PI / (n - 1)));
        co.push_back(tr.amp[k - 1]);
      }
      if (sines.empty()) continue;
      std::vector<const HTT *> ptr;
      for (auto &s : sines) ptr.push_back(&s);
      HTT tbar = add(ptr, co);
      rd(tbar);
      HTT edge = matvec_h(M1, tbar);
      rd(edge);
      for (auto &v : edge.c[0]) v *= (tr.side <= 1) ? lb : la;
      HTT node = (tr.side <= 1) ? zkron(edge, unit1(d, tr.side)) : zkron(unit1(d, tr.side - 2), edge);
      terms.push_back(with_prefix_vector(g, unit_vec(2, tr.comp), unit_vec(g.q, m), node));
    }
  }
  any = !terms.empty();
  if (!any) {
    HTT z = with_prefix_vector(g, unit_vec(2, 0), unit_vec(g.q, 0), zkron(ones1(d), ones1(d)));
    for (auto &v : z.c[0]) v = 0.0;
    return z;
  }
  std::vector<const HTT *> ptr;
  std::vector<double> co;
  for (auto &t : terms) {
    ptr.push_back(&t);
    co.push_back(1.0);
  }
  HTT f = add(ptr, co);
  rd(f);
  return f;
}

// Pi^(mp): rows on subdomain m, columns on p, 1 where nodes coincide.
bool connectivity(const Geometry &g, int m, int p, HTT &out) {
  const qtt_square &a = g.p->sub[m], &b = g.p->sub[p];
  const double s = a.side;
  const long dx = std::lround((b.x0 - a.x0) / s), dy = std::lround((b.y0 - a.y0) / s);
  if (std::fabs(b.side - a.side) > 1e-12 * s) return false;
  if (std::labs(dx) > 1 || std::labs(dy) > 1 || (dx == 0 && dy == 0)) return false;
  // check the offsets are exact multiples of the side
  if (std::fabs(b.x0 - a.x0 - dx * s) > 1e-9 * s || std::fabs(b.y0 - a.y0 - dy * s) > 1e-9 * s)
    return false;
  const int d = g.d;
  HTT X = (dx == 0) ? identity1(d) : outer1(d, dx == 1 ? 1 : 0, dx == 1 ? 0 : 1);
  HTT Y = (dy == 0) ? identity1(d) : outer1(d, dy == 1 ? 1 : 0, dy == 1 ? 0 : 1);
  out = with_prefix_matrix(g, eye(2), sel_matrix(g.q, m, p), zkron(Y, X));
  return true;
}

bool coupled(const Geometry &g, Rounder &rd, HTT &K, HTT &f) {
  const int q = g.q;
  std::vector<HTT> P;
  std::vector<std::pair<int, int>> idx;
  for (int m = 0; m < q; ++m)
    for (int p = 0; p < q; ++p) {
      if (m == p) continue;
      HTT t;
      if (connectivity(g, m, p, t)) {
        P.push_back(t);
        idx.push_back({m, p});
      }
    }
  auto find = [&](int m, int p) -> int {
    for (size_t u = 0; u < idx.size(); ++u)
      if (idx[u].first == m && idx[u].second == p) return (int)u;
    return -1;
  };
  std::vector<HTT> lap;
  std::vector<double> lco;
  std::vector<HTT> degt;
  for (size_t u = 0; u < idx.size(); ++u) {
    const int m = idx[u].first, p = idx[u].second;
    const int v = find(p, m);
    HTT PQ = matmat(P[u], P[v]);
    degt.push_back(PQ);
    if (m < p) {
      lap.push_back(PQ);
      lap.push_back(matmat(P[v], P[u]));
      lap.push_back(P[u]);
      lap.push_back(P[v]);
      lco.insert(lco.end(), {1.0, 1.0, -1.0, -1.0});
    }
  }
  std::vector<const HTT *> ptr;
  for (auto &t : lap) ptr.push_back(&t);
  HTT L = add(ptr, lco);
  rd(L);
  double c11, c12, c22, c33;
  voigt(g.p, c11, c12, c22, c33);
  Geometry g1 = g;
  g1.q = 1;
  HTT Ksq = block_stiffness(g1, rd);
  const double gamma =
      g.p->gamma > 0.0 ? g.p->gamma : trace(Ksq) / (2.0 * std::ldexp(1.0, 2 * g.d));
  HTT I = identity_like(K);
  if (g.p->coupling == QTT_COUPLING_PAPER) {
    std::vector<const HTT *> pp;
    std::vector<double> pc;
    for (auto &t : P) {
      pp.push_back(&t);
      pc.push_back(1.0);
    }
    pp.push_back(&I);
    pc.push_back(1.0);
    HTT IP = add(pp, pc);
    rd(IP);
    HTT IPK = matmat(IP, K);
    rd(IPK);
    HTT Kc = add({&IPK, &L}, {1.0, gamma});
    rd(Kc);
    HTT fc = matvec_h(IP, f);
    rd(fc);
    K = Kc;
    f = fc;
    return rd.st == QTT_OK;
  }
  // symmetric: T = I - diag(w) L, w = 1/(deg+1) on deg in {0,1,2,3}
  std::vector<const HTT *> dp;
  std::vector<double> dc;
  for (auto &t : degt) {
    dp.push_back(&t);
    dc.push_back(1.0);
  }
  HTT Dm = add(dp, dc);
  rd(Dm);
  HTT deg = diag_of(Dm);
  rd(deg);
  HTT d2 = hadamard(deg, deg);
  rd(d2);
  HTT d3 = hadamard(d2, deg);
  rd(d3);
  // cubic through (0,1), (1,1/2), (2,1/3), (3,1/4)
  const double c0 = 1.0, c1 = -3.0 / 4.0, c2 = 7.0 / 24.0, c3 = -1.0 / 24.0;
  HTT one = ones_like(deg);
  HTT w = add({&one, &deg, &d2, &d3}, {c0, c1, c2, c3});
  rd(w);
  HTT WL = matmat(diag_matrix(w), L);
  rd(WL);
  HTT Tm = add({&I, &WL}, {1.0, -1.0});
  rd(Tm);
  HTT TK = matmat(Tm, K);
  rd(TK);
  HTT TKT = matmat(TK, Tm);
  rd(TKT);
  HTT Kc = add({&TKT, &L}, {1.0, gamma});
  rd(Kc);
  HTT fc = matvec_h(Tm, f);
  rd(fc);
  K = Kc;
  f = fc;
  return rd.st == QTT_OK;
}

int64_t packed_size(const HTT &t) {
  int64_t e = 0;
  for (int k = 0; k < t.D; ++k) e += (int64_t)t.c[k].size();
  return e;
}

qtt_status check_problem(const qtt_problem *p) {
  if (!p) return fail(QTT_E_INVAL, "problem is NULL");
  if (p->level < 1 || p->level > 19) return fail(QTT_E_INVAL, "level must be in 1..19");
  if (p->q < 1 || p->q > 32) return fail(QTT_E_INVAL, "q must be in 1..32");
  if (1 + (p->q > 1) + 2 * p->level > QTT_MAX_CORES) return fail(QTT_E_INVAL, "too many cores");
  if (!p->sub) return fail(QTT_E_INVAL, "sub is NULL");
  if (!(p->E > 0.0) || !(p->nu > -1.0 && p->nu < 0.5)) return fail(QTT_E_INVAL, "bad material");
  for (int m = 0; m < p->q; ++m)
    if (!(p->sub[m].side > 0.0)) return fail(QTT_E_INVAL, "subdomain side must be > 0");
  for (int m = 1; m < p->q; ++m)
    if (std::fabs(p->sub[m].side - p->sub[0].side) > 1e-12 * p->sub[0].side)
      return fail(QTT_E_UNSUPPORTED, "subdomains must share one side length");
  for (int m = 0; m < p->q; ++m) {
    const double *e = p->sub[m].edges;
    if (e[0] == 0.0 && e[1] == 0.0 && e[2] == 0.0 && e[3] == 0.0) continue;
    if (p->q > 1)
      return fail(QTT_E_UNSUPPORTED, "parallelogram subdomains: one subdomain only (q = 1)");
    const double det = e[0] * e[3] - e[1] * e[2];
    if (!(std::fabs(det) > 1e-12 * (std::fabs(e[0] * e[3]) + std::fabs(e[1] * e[2]))))
      return fail(QTT_E_INVAL, "degenerate parallelogram (edge vectors parallel)");
  }
  if (p->ntrac < 0 || (p->ntrac > 0 && !p->trac)) return fail(QTT_E_INVAL, "bad tractions");
  for (int u = 0; u < p->ntrac; ++u) {
    const qtt_traction &t = p->trac[u];
    if (t.sub < 0 || t.sub >= p->q || t.side < 0 || t.side > 3 || t.comp < 0 || t.comp > 1 ||
        t.nmodes < 0 || (t.nmodes > 0 && !t.amp))
      return fail(QTT_E_INVAL, "bad traction entry");
  }
  if (p->coupling != QTT_COUPLING_PAPER && p->coupling != QTT_COUPLING_SYMMETRIC)
    return fail(QTT_E_INVAL, "coupling must be QTT_COUPLING_PAPER or QTT_COUPLING_SYMMETRIC");
  if (!(p->gamma == p->gamma)) return fail(QTT_E_INVAL, "gamma is NaN");
  return QTT_OK;
}


// ---------------------------------------------------------------- BPX
// Linear function f(s) = c0 + sum_k ck 2^k s_k of the low l digits as a
// rank-2 QTT "column" (row mode 2, column mode 1): the bond carries
// (1, partial sum).
HTT linear_low(int l, double c0, double slope) {
  HTT t = HTT::make(l, true);
  for (int k = 0; k < l; ++k) t.m[k] = 1;
  for (int k = 0; k <= l; ++k) t.r[k] = (k == 0 || k == l) ? 1 : 2;
  for (int k = 0; k < l; ++k) {
    t.alloc(k);
    const double ck = slope * std::ldexp(1.0, k);
    for (int i = 0; i < 2; ++i) {
      // 2x2 block [[1, ck i], [0, 1]] between the states (1, S)
      double G[2][2] = {{1.0, ck * i}, {0.0, 1.0}};
      if (k == 0) {
        // start from the row (1, c0)
        const double a0 = 1.0, a1 = c0;
        const double v0 = a0 * G[0][0] + a1 * G[1][0];
        const double v1 = a0 * G[0][1] + a1 * G[1][1];
        if (l == 1) {
          t.at(k, 0, i, 0, 0) = v1;
        } else {
          t.at(k, 0, i, 0, 0) = v0;
          t.at(k, 0, i, 0, 1) = v1;
        }
      } else if (k == l - 1) {
        // end by reading the sum: column (0, 1)
        t.at(k, 0, i, 0, 0) = G[0][1];
        t.at(k, 1, i, 0, 0) = G[1][1];
      } else {
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) t.at(k, a, i, 0, b) = G[a][b];
      }
    }
  }
  return t;
}

HTT concat(const HTT &lo, const HTT &hi) {
  HTT t = lo;
  t.D = lo.D + hi.D;
  t.n.insert(t.n.end(), hi.n.begin(), hi.n.end());
  t.m.insert(t.m.end(), hi.m.begin(), hi.m.end());
  t.r.pop_back();
  t.r.insert(t.r.end(), hi.r.begin(), hi.r.end());
  t.c.insert(t.c.end(), hi.c.begin(), hi.c.end());
  return t;
}

// B_l = P_l diag(m) P_l^T on 2^d points: P_l interpolates linearly between
// the coarse nodes i = 2^l j and is constant past the last one; a clamp at
// the low end drops coarse node 0 (m = 1 - e_0), a clamp at the high end
// mirrors the construction (every digit flipped).
HTT bpx_level_1d(int d, int l, bool clamp_lo, bool clamp_hi, Rounder &rd) {
  HTT P;
  const bool clamp = clamp_lo || clamp_hi;
  if (l == 0) {
    P = identity1(d);
  } else if (l == d) {
    if (clamp) return HTT();  // only the constant: removed by the clamp
    P = HTT::make(d, true);
    for (int k = 0; k < d; ++k) {
      P.m[k] = 1;
      P.alloc(k);
      P.at(k, 0, 0, 0, 0) = P.at(k, 0, 1, 0, 0) = 1.0;
    }
  } else {
    const double H = std::ldexp(1.0, l);
    HTT a = linear_low(l, 1.0, -1.0 / H);
    HTT b = linear_low(l, 0.0, 1.0 / H);
    HTT I = identity1(d - l);
    HTT J = shift1(d - l), El = outer1(d - l, 1, 1);
    HTT S = add({&J, &El}, {1.0, 1.0});
    HTT t1 = concat(a, I), t2 = concat(b, S);
    P = add({&t1, &t2}, {1.0, 1.0});
  }
  HTT Pt = transpose(P);
  HTT B;
  if (clamp && l < d) {
    // drop coarse node 0: P diag(1 - e_0) P^T
    HTT mk = HTT::make(d, true);
    for (int k = 0; k < d; ++k) {
      const bool low = k < l;
      mk.n[k] = mk.m[k] = low ? 1 : 2;
      mk.alloc(k);
      if (low) mk.at(k, 0, 0, 0, 0) = 1.0;
      else mk.at(k, 0, 0, 0, 0) = mk.at(k, 0, 1, 1, 0) = 1.0;
    }
    HTT e0 = HTT::make(d, true);
    for (int k = 0; k < d; ++k) {
      const bool low = k < l;
      e0.n[k] = e0.m[k] = low ? 1 : 2;
      e0.alloc(k);
      e0.at(k, 0, 0, 0, 0) = 1.0;
    }
    HTT m = add({&mk, &e0}, {1.0, -1.0});
    if (l == 0) {
      // level 0: P = I, the mask acts on the fine nodes directly
      m = add({&mk, &e0}, {1.0, -1.0});
    }
    HTT Pm = matmat(P, m);
    B = matmat(Pm, Pt);
  } else {
    B = matmat(P, Pt);
  }
  rd(B);
  if (clamp_hi) {
    for (int k = 0; k < B.D; ++k) {
      std::vector<double> c = B.c[k];
      for (int a = 0; a < B.r[k]; ++a)
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            for (int e = 0; e < B.r[k + 1]; ++e)
              B.at(k, a, i, j, e) = c[a + (size_t)B.r[k] * ((1 - i) + 2 * ((1 - j) + 2 * (size_t)e))];
    }
  }
  return B;
}

// node part of C for one component: sum_l B_l^y (z) B_l^x
HTT bpx_nodes(int d, const uint8_t fixed[4][2], int c, Rounder &rd, bool &ok) {
  const bool w = fixed[0][c], e = fixed[1][c], s = fixed[2][c], n = fixed[3][c];
  ok = !(w && e) && !(s && n);
  HTT acc;
  bool have = false;
  for (int l = 0; l <= d && ok; ++l) {
    HTT bx = bpx_level_1d(d, l, w, e, rd);
    HTT by = bpx_level_1d(d, l, s, n, rd);
    if (bx.D == 0 || by.D == 0) continue;
    HTT z = zkron(by, bx);
    if (!have) {
      acc = z;
      have = true;
    } else {
      acc = add({&acc, &z}, {1.0, 1.0});
    }
    rd(acc);
  }
  return acc;
}

// bound on the rank of any intermediate before its rounding: products of
// the copy-averaging operator with the block stiffness reach ~930 for three
// subdomains; a single square stays below 256
int assembly_rank_bound(const qtt_problem *p) { return p->q > 1 ? 1024 : 256; }

}  // namespace
}  // namespace qtt

using namespace qtt;

extern "C" qtt_status qtt_assemble_workspace(const qtt_problem *p, size_t *bytes,
                                             int64_t *K_capacity, int64_t *f_capacity) {
  qtt_status st = check_problem(p);
  if (st != QTT_OK) return st;
  if (!bytes) return fail(QTT_E_INVAL, "bytes is NULL");
  const int D = 1 + (p->q > 1) + 2 * p->level;
  std::vector<int32_t> n(D, 2), m(D, 2);
  if (p->q > 1) n[1] = m[1] = p->q;
  // unrounded intermediates may exceed the mode-product bounds, so every
  // interior bond gets the full rank bound
  std::vector<int> caps(D + 1, assembly_rank_bound(p));
  caps.front() = caps.back() = 1;
  Arena ar;
  ar.dry = true;
  TTDesc t;
  arena_tt(ar, t, D, n.data(), m.data(), caps);
  RoundWs w;
  round_ws_take(ar, t.v, w);
  *bytes = ar.used + 4096;
  // final operators: rank <= 96 for K, <= 64 for f (checked on output)
  std::vector<int> kc = bounded_caps(D, n.data(), m.data(), 96);
  std::vector<int> fcp = bounded_caps(D, n.data(), nullptr, 64);
  int64_t ke = 0, fe = 0;
  for (int k = 0; k < D; ++k) {
    ke += (int64_t)kc[k] * n[k] * m[k] * kc[k + 1];
    fe += (int64_t)fcp[k] * n[k] * fcp[k + 1];
  }
  if (K_capacity) *K_capacity = ke;
  if (f_capacity) *f_capacity = fe;
  return QTT_OK;
}

extern "C" qtt_status qtt_assemble_stiffness(const qtt_problem *p, double eps, qtt_tt *K,
                                             qtt_tt *f, void *ws, size_t ws_bytes,
                                             void *stream) {
  qtt::clear_stale_error();
  qtt_status st = check_problem(p);
  if (st != QTT_OK) return st;
  if (!K || !f || !K->data || !f->data || !K->ranks || !f->ranks)
    return fail(QTT_E_INVAL, "K or f has a NULL field");
  if (!(eps >= 0.0)) return fail(QTT_E_INVAL, "eps must be >= 0");
  const int D = 1 + (p->q > 1) + 2 * p->level;
  if (K->ncores != D || f->ncores != D) return fail(QTT_E_SHAPE, "K and f need ncores = 1 + (q>1) + 2 level");
  if (!ws) return fail(QTT_E_CAPACITY, "workspace is NULL");
  Geometry g{p->level, p->q, p};
  Rounder rd;
  rd.base.base = (char *)ws;
  rd.base.size = ws_bytes;
  rd.s = (hipStream_t)stream;
  rd.eps = eps;
  HTT Kb = block_stiffness(g, rd);
  bool any = false;
  HTT fb = load_vector(g, rd, any);
  if (rd.st != QTT_OK) return rd.st;
  if (p->q > 1 && !coupled(g, rd, Kb, fb)) return rd.st;
  const double N = 2.0 * p->q * std::ldexp(1.0, 2 * p->level);
  const double gD = trace(Kb) / N;
  HTT mk = mask_vector(g, rd);
  HTT Pm = diag_matrix(mk);
  HTT one = ones_like(mk);
  HTT cm = add({&one, &mk}, {1.0, -1.0});
  rd(cm);
  HTT Pc = diag_matrix(cm);
  HTT PK = matmat(Pm, Kb);
  rd(PK);
  HTT PKP = matmat(PK, Pm);
  rd(PKP);
  HTT Kbc = add({&PKP, &Pc}, {1.0, gD});
  rd(Kbc);
  HTT fbc = hadamard(mk, fb);
  rd(fbc);
  if (rd.st != QTT_OK) return rd.st;
  // write out
  auto put = [&](const HTT &t, qtt_tt *o, const char *name) -> qtt_status {
    for (int k = 0; k < D; ++k) {
      if (o->nrow[k] != t.n[k]) return fail(QTT_E_SHAPE, std::string(name) + ": nrow mismatch");
      if (t.matrix && (!o->ncol || o->ncol[k] != t.m[k]))
        return fail(QTT_E_SHAPE, std::string(name) + ": ncol mismatch");
    }
    if (packed_size(t) > o->capacity)
      return fail(QTT_E_CAPACITY, std::string(name) + ": capacity " + std::to_string(o->capacity) +
                                      " < " + std::to_string(packed_size(t)));
    int64_t off = 0;
    for (int k = 0; k < D; ++k) {
      QTT_HIP(hipMemcpyAsync(o->data + off, t.c[k].data(), sizeof(double) * t.c[k].size(),
                             hipMemcpyHostToDevice, rd.s));
      off += (int64_t)t.c[k].size();
    }
    for (int k = 0; k <= D; ++k) o->ranks[k] = t.r[k];
    QTT_HIP(publish_ranks(o, rd.s));
    return QTT_OK;
  };
  if ((st = put(Kbc, K, "K")) != QTT_OK) return st;
  if ((st = put(fbc, f, "f")) != QTT_OK) return st;
  QTT_HIP(hipStreamSynchronize(rd.s));
  return QTT_OK;
}

extern "C" qtt_status qtt_assemble_bpx(const qtt_problem *p, double eps, qtt_tt *C, void *ws,
                                       size_t ws_bytes, void *stream) {
  qtt::clear_stale_error();
  qtt_status st = check_problem(p);
  if (st != QTT_OK) return st;
  if (p->q != 1) return fail(QTT_E_UNSUPPORTED, "the BPX preconditioner is built for q = 1");
  if (p->sub[0].edges[0] != 0.0 || p->sub[0].edges[1] != 0.0 || p->sub[0].edges[2] != 0.0 ||
      p->sub[0].edges[3] != 0.0)
    return fail(QTT_E_UNSUPPORTED, "the BPX preconditioner is built for a square subdomain");
  if (!C || !C->data || !C->ranks || !C->ncol) return fail(QTT_E_INVAL, "C has a NULL field");
  const int D = 1 + 2 * p->level;
  if (C->ncores != D) return fail(QTT_E_SHAPE, "C needs ncores = 1 + 2 level");
  if (!ws) return fail(QTT_E_CAPACITY, "workspace is NULL");
  Geometry g{p->level, 1, p};
  Rounder rd;
  rd.base.base = (char *)ws;
  rd.base.size = ws_bytes;
  rd.s = (hipStream_t)stream;
  rd.eps = eps;
  // gamma_D = trace(K)/N as in the assembly
  HTT Kb = block_stiffness(g, rd);
  if (rd.st != QTT_OK) return rd.st;
  const double N = 2.0 * std::ldexp(1.0, 2 * p->level);
  const double gD = trace(Kb) / N;
  std::vector<HTT> comp;
  for (int c = 0; c < 2; ++c) {
    bool ok = true;
    HTT node = bpx_nodes(p->level, p->sub[0].fixed, c, rd, ok);
    if (!ok) return fail(QTT_E_UNSUPPORTED, "BPX needs at most one clamped end per direction");
    if (rd.st != QTT_OK) return rd.st;
    comp.push_back(with_prefix_matrix(g, sel_matrix(2, c, c), eye(1), node));
  }
  HTT Cm = add({&comp[0], &comp[1]}, {1.0, 1.0});
  rd(Cm);
  HTT mk = mask_vector(g, rd);
  HTT Pm = diag_matrix(mk);
  HTT one = ones_like(mk);
  HTT cm = add({&one, &mk}, {1.0, -1.0});
  rd(cm);
  HTT Pc = diag_matrix(cm);
  HTT PC = matmat(Pm, Cm);
  rd(PC);
  HTT PCP = matmat(PC, Pm);
  rd(PCP);
  HTT Cbc = add({&PCP, &Pc}, {1.0, 1.0 / gD});
  rd(Cbc);
  if (rd.st != QTT_OK) return rd.st;
  for (int k = 0; k < D; ++k)
    if (C->nrow[k] != Cbc.n[k] || C->ncol[k] != Cbc.m[k]) return fail(QTT_E_SHAPE, "C modes");
  if (packed_size(Cbc) > C->capacity)
    return fail(QTT_E_CAPACITY, "C: capacity " + std::to_string(C->capacity) + " < " +
                                    std::to_string(packed_size(Cbc)));
  int64_t off = 0;
  for (int k = 0; k < D; ++k) {
    QTT_HIP(hipMemcpyAsync(C->data + off, Cbc.c[k].data(), sizeof(double) * Cbc.c[k].size(),
                           hipMemcpyHostToDevice, rd.s));
    off += (int64_t)Cbc.c[k].size();
  }
  for (int k = 0; k <= D; ++k) C->ranks[k] = Cbc.r[k];
  QTT_HIP(publish_ranks(C, rd.s));
  QTT_HIP(hipStreamSynchronize(rd.s));
  return QTT_OK;
}
