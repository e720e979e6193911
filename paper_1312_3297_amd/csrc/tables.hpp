// Compile-time lattice and moment-basis tables for the HIP collide-stream kernels.
//
// Everything here is exact rational arithmetic evaluated by the compiler, so a
// kernel instantiated for one (lattice, basis) pair sees only literal constants
// and the unrolled per-node algebra folds every zero away.
//
// Notation (section 1 of the paper, with the velocity scale set to 1; the
// library rescales velocities by 1/lambda, which is exact for the built-in
// bases because each basis polynomial is homogeneous in (X, lambda)):
//   c_j        integer lattice directions, w_j the equilibrium weights
//   P_k        the user-facing moment basis (rates s_k act on it)
//   W_l        the "working" basis the kernel shifts in: same span as P,
//              P = R W with a constant, block-diagonal R
//   M_W(0)     W_l(c_j);   M_W(u~) = T_W(u~) M_W(0)             eq. (MatMu)
//   D_a        derivation matrix: d/dX_a W_k = sum_l D_a[k][l] W_l
//   T_W(u~)    = prod_a exp(-u~_a D_a)  (the shift matrix, eq. (matTu); this
//              product form is exact when span(W) is closed under
//              differentiation, which is checked below and is what makes
//              u~ -> T(u~) a group morphism, Prop. th:csd2q9)
#pragma once

#include <cstdint>

namespace lbmrv {

// ---------------------------------------------------------------- rationals
constexpr int64_t iabs(int64_t a) { return a < 0 ? -a : a; }
constexpr int64_t igcd(int64_t a, int64_t b) {
  a = iabs(a);
  b = iabs(b);
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

struct Rat {
  int64_t n = 0, d = 1;
  constexpr Rat() = default;
  constexpr Rat(int64_t num, int64_t den = 1) : n(num), d(den) {
    if (d < 0) { n = -n; d = -d; }
    int64_t g = igcd(n, d);
    if (g > 1) { n /= g; d /= g; }
    if (n == 0) d = 1;
  }
  constexpr bool zero() const { return n == 0; }
  constexpr double val() const { return double(n) / double(d); }
};
constexpr Rat operator+(Rat a, Rat b) {
  int64_t g = igcd(a.d, b.d);
  return Rat(a.n * (b.d / g) + b.n * (a.d / g), a.d / g * b.d);
}
constexpr Rat operator-(Rat a) { return Rat(-a.n, a.d); }
constexpr Rat operator-(Rat a, Rat b) { return a + (-b); }
constexpr Rat operator*(Rat a, Rat b) {
  int64_t g1 = igcd(a.n, b.d), g2 = igcd(b.n, a.d);
  if (g1 == 0) g1 = 1;
  if (g2 == 0) g2 = 1;
  return Rat((a.n / g1) * (b.n / g2), (a.d / g2) * (b.d / g1));
}
constexpr Rat operator/(Rat a, Rat b) { return a * Rat(b.d, b.n); }
constexpr bool operator==(Rat a, Rat b) { return a.n == b.n && a.d == b.d; }
constexpr bool operator!=(Rat a, Rat b) { return !(a == b); }

// ---------------------------------------------------------------- polynomials
// Sparse polynomials in X, Y, Z: at most kMaxTerms monomials X^a Y^b Z^c,
// kept merged (no repeated exponents, no zero coefficients).
constexpr int kDeg = 4;
constexpr int kP = kDeg + 1;
constexpr int kMaxTerms = 16;

struct PTerm {
  int a = 0, b = 0, e = 0;
  Rat c;
};
struct Poly {
  int n = 0;
  PTerm t[kMaxTerms] = {};
  bool overflow = false;
  constexpr Poly() = default;
  constexpr void add(int a, int b, int e, Rat c) {
    if (c.zero()) return;
    for (int i = 0; i < n; ++i)
      if (t[i].a == a && t[i].b == b && t[i].e == e) {
        t[i].c = t[i].c + c;
        if (t[i].c.zero()) {
          for (int k = i; k + 1 < n; ++k) t[k] = t[k + 1];
          --n;
        }
        return;
      }
    if (n == kMaxTerms) { overflow = true; return; }
    t[n].a = a; t[n].b = b; t[n].e = e; t[n].c = c;
    ++n;
  }
};
struct Term {
  int a, b, e;
  int64_t num, den;
};

template <int N>
constexpr Poly poly(const Term (&ts)[N]) {
  Poly p;
  for (int i = 0; i < N; ++i) p.add(ts[i].a, ts[i].b, ts[i].e, Rat(ts[i].num, ts[i].den));
  return p;
}
constexpr Poly mono(int a, int b, int e) {
  Poly p;
  p.add(a, b, e, Rat(1));
  return p;
}
constexpr Poly padd(const Poly& x, const Poly& y, Rat ky) {
  Poly p = x;
  for (int i = 0; i < y.n; ++i) p.add(y.t[i].a, y.t[i].b, y.t[i].e, ky * y.t[i].c);
  p.overflow = p.overflow || x.overflow || y.overflow;
  return p;
}
constexpr bool peq(const Poly& x, const Poly& y) {
  if (x.overflow || y.overflow || x.n != y.n) return false;
  for (int i = 0; i < x.n; ++i) {
    bool found = false;
    for (int k = 0; k < y.n; ++k)
      if (y.t[k].a == x.t[i].a && y.t[k].b == x.t[i].b && y.t[k].e == x.t[i].e) found = (y.t[k].c == x.t[i].c);
    if (!found) return false;
  }
  return true;
}
constexpr Poly pderiv(const Poly& x, int axis) {
  Poly p;
  for (int i = 0; i < x.n; ++i) {
    int ex[3] = {x.t[i].a, x.t[i].b, x.t[i].e};
    if (ex[axis] == 0) continue;
    int k = ex[axis];
    ex[axis] -= 1;
    p.add(ex[0], ex[1], ex[2], Rat(k) * x.t[i].c);
  }
  return p;
}
constexpr Rat peval(const Poly& x, int X, int Y, int Z) {
  Rat s;
  for (int i = 0; i < x.n; ++i) {
    int64_t m = 1;
    for (int k = 0; k < x.t[i].a; ++k) m *= X;
    for (int k = 0; k < x.t[i].b; ++k) m *= Y;
    for (int k = 0; k < x.t[i].e; ++k) m *= Z;
    s = s + x.t[i].c * Rat(m);
  }
  return s;
}
// Homogeneous degree of a polynomial (-1 if not homogeneous or zero).
constexpr int phomdeg(const Poly& x) {
  int deg = -1;
  for (int i = 0; i < x.n; ++i) {
    int d = x.t[i].a + x.t[i].b + x.t[i].e;
    if (deg < 0) deg = d;
    else if (deg != d) return -1;
  }
  return deg;
}

// ---------------------------------------------------------------- matrices
template <int Q>
struct Mat {
  Rat m[Q][Q] = {};
};
template <int Q>
constexpr Mat<Q> mmul(const Mat<Q>& A, const Mat<Q>& B) {
  Mat<Q> C;
  for (int i = 0; i < Q; ++i)
    for (int k = 0; k < Q; ++k) {
      if (A.m[i][k].zero()) continue;
      for (int j = 0; j < Q; ++j)
        if (!B.m[k][j].zero()) C.m[i][j] = C.m[i][j] + A.m[i][k] * B.m[k][j];
    }
  return C;
}
template <int Q>
constexpr Mat<Q> mscale(const Mat<Q>& A, Rat s) {
  Mat<Q> C;
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) C.m[i][j] = A.m[i][j] * s;
  return C;
}
template <int Q>
constexpr Mat<Q> mtrans(const Mat<Q>& A) {
  Mat<Q> C;
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) C.m[i][j] = A.m[j][i];
  return C;
}
template <int Q>
constexpr bool mzero(const Mat<Q>& A) {
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j)
      if (!A.m[i][j].zero()) return false;
  return true;
}
template <int Q>
constexpr bool midentity(const Mat<Q>& A) {
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j)
      if (A.m[i][j] != Rat(i == j ? 1 : 0)) return false;
  return true;
}
// Gauss-Jordan inverse; ok = false if singular.
template <int Q>
struct InvResult {
  Mat<Q> inv;
  bool ok;
};
template <int Q>
constexpr InvResult<Q> minv(const Mat<Q>& A) {
  Mat<Q> a = A, b;
  for (int i = 0; i < Q; ++i) b.m[i][i] = Rat(1);
  for (int col = 0; col < Q; ++col) {
    int piv = -1;
    for (int r = col; r < Q; ++r)
      if (!a.m[r][col].zero()) { piv = r; break; }
    if (piv < 0) return {b, false};
    for (int j = 0; j < Q; ++j) {
      Rat t = a.m[col][j]; a.m[col][j] = a.m[piv][j]; a.m[piv][j] = t;
      t = b.m[col][j]; b.m[col][j] = b.m[piv][j]; b.m[piv][j] = t;
    }
    Rat p = a.m[col][col];
    for (int j = 0; j < Q; ++j) {
      a.m[col][j] = a.m[col][j] / p;
      b.m[col][j] = b.m[col][j] / p;
    }
    for (int r = 0; r < Q; ++r) {
      if (r == col || a.m[r][col].zero()) continue;
      Rat f = a.m[r][col];
      for (int j = 0; j < Q; ++j) {
        if (!a.m[col][j].zero()) a.m[r][j] = a.m[r][j] - f * a.m[col][j];
        if (!b.m[col][j].zero()) b.m[r][j] = b.m[r][j] - f * b.m[col][j];
      }
    }
  }
  return {b, true};
}

// Sparse row of a matrix: the nonzero columns c >= minc of row k.
template <int Q>
struct SpRow {
  int n = 0;
  int col[Q] = {};
  Rat val[Q] = {};
};
template <int Q>
constexpr SpRow<Q> sprow(const Mat<Q>& M, int k, int minc) {
  SpRow<Q> r;
  for (int c = minc; c < Q; ++c)
    if (!M.m[k][c].zero()) {
      r.col[r.n] = c;
      r.val[r.n] = M.m[k][c];
      ++r.n;
    }
  return r;
}

// ---------------------------------------------------------------- lattices
// Directions are an interface convention (documented in include/lbmrv.h).
struct Dir {
  int x, y, z;
};

struct D2Q9Lat {
  static constexpr int D = 2, Q = 9;
  static constexpr Dir c[Q] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                               {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
  static constexpr Rat w(int j) {
    int s = c[j].x * c[j].x + c[j].y * c[j].y;
    return s == 0 ? Rat(4, 9) : s == 1 ? Rat(1, 9) : Rat(1, 36);
  }
};

struct D3Q19Lat {
  static constexpr int D = 3, Q = 19;
  static constexpr Dir c[Q] = {
      {0, 0, 0},   {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0}, {0, 0, 1},   {0, 0, -1},
      {1, 1, 0},   {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
      {-1, 0, 1},  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  static constexpr Rat w(int j) {
    int s = c[j].x * c[j].x + c[j].y * c[j].y + c[j].z * c[j].z;
    return s == 0 ? Rat(1, 3) : s == 1 ? Rat(1, 18) : Rat(1, 36);
  }
};

struct D3Q27Lat {
  static constexpr int D = 3, Q = 27;
  static constexpr Dir c[Q] = {
      {0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
      {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},
      {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},  {1, 1, 1},   {-1, -1, -1},
      {1, 1, -1},  {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};
  static constexpr Rat w(int j) {
    int s = c[j].x * c[j].x + c[j].y * c[j].y + c[j].z * c[j].z;
    return s == 0 ? Rat(8, 27) : s == 1 ? Rat(2, 27) : s == 2 ? Rat(1, 54) : Rat(1, 216);
  }
};

// Index of the opposite direction -c_j.
template <class L>
constexpr int opposite(int j) {
  for (int k = 0; k < L::Q; ++k)
    if (L::c[k].x == -L::c[j].x && L::c[k].y == -L::c[j].y && L::c[k].z == -L::c[j].z) return k;
  return -1;
}

// ---------------------------------------------------------------- bases
// Each basis provides P (user-facing, rates act on it) and W (working basis).

// eq. (mom), lambda = 1:
//   1, X, Y, 3|X|^2 - 4, X^2 - Y^2, XY, X(3|X|^2 - 5), Y(3|X|^2 - 5),
//   9/2 |X|^4 - 21/2 |X|^2 + 4
struct BasisD2Q9Paper {
  using Lat = D2Q9Lat;
  static constexpr int Q = 9;
  static constexpr Poly P(int k) {
    switch (k) {
      case 0: return mono(0, 0, 0);
      case 1: return mono(1, 0, 0);
      case 2: return mono(0, 1, 0);
      case 3: { constexpr Term t[] = {{2, 0, 0, 3, 1}, {0, 2, 0, 3, 1}, {0, 0, 0, -4, 1}}; return poly(t); }
      case 4: { constexpr Term t[] = {{2, 0, 0, 1, 1}, {0, 2, 0, -1, 1}}; return poly(t); }
      case 5: return mono(1, 1, 0);
      case 6: { constexpr Term t[] = {{3, 0, 0, 3, 1}, {1, 2, 0, 3, 1}, {1, 0, 0, -5, 1}}; return poly(t); }
      case 7: { constexpr Term t[] = {{2, 1, 0, 3, 1}, {0, 3, 0, 3, 1}, {0, 1, 0, -5, 1}}; return poly(t); }
      default: {
        constexpr Term t[] = {{4, 0, 0, 9, 2}, {2, 2, 0, 9, 1}, {0, 4, 0, 9, 2},
                              {2, 0, 0, -21, 2}, {0, 2, 0, -21, 2}, {0, 0, 0, 4, 1}};
        return poly(t);
      }
    }
  }
  static constexpr Poly W(int k) { return P(k); }
  // lambda-homogeneity degree of P_k: P_k(la X) = la^e P_k^{(la=1)}(X) with the
  // paper's normalisation (only q_x, q_y carry lambda)
  static constexpr int lam_deg(int k) { return (k == 1 || k == 2) ? 1 : 0; }
};

// eq. (polgeier): 1, X, Y, X^2+Y^2, X^2-Y^2, XY, XY^2, X^2Y, X^2Y^2
struct BasisD2Q9Geier {
  using Lat = D2Q9Lat;
  static constexpr int Q = 9;
  static constexpr Poly P(int k) {
    switch (k) {
      case 3: { constexpr Term t[] = {{2, 0, 0, 1, 1}, {0, 2, 0, 1, 1}}; return poly(t); }
      case 4: { constexpr Term t[] = {{2, 0, 0, 1, 1}, {0, 2, 0, -1, 1}}; return poly(t); }
      default: return W(k);
    }
  }
  static constexpr Poly W(int k) {
    constexpr int e[9][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {0, 2}, {1, 1}, {1, 2}, {2, 1}, {2, 2}};
    return mono(e[k][0], e[k][1], 0);
  }
  static constexpr int lam_deg(int k) { return phomdeg(P(k)); }
};

// Graded monomial bases for D3Q19 / D3Q27 with the degree-2 block recombined
// into trace, two normal-stress differences and three off-diagonal stresses.
constexpr Poly deg2_user(int k) {  // k = 0..5 within the degree-2 block
  switch (k) {
    case 0: { constexpr Term t[] = {{2, 0, 0, 1, 1}, {0, 2, 0, 1, 1}, {0, 0, 2, 1, 1}}; return poly(t); }
    case 1: { constexpr Term t[] = {{2, 0, 0, 2, 1}, {0, 2, 0, -1, 1}, {0, 0, 2, -1, 1}}; return poly(t); }
    case 2: { constexpr Term t[] = {{0, 2, 0, 1, 1}, {0, 0, 2, -1, 1}}; return poly(t); }
    case 3: return mono(1, 1, 0);
    case 4: return mono(0, 1, 1);
    default: return mono(1, 0, 1);
  }
}
constexpr int kExp19[19][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2},
                               {1, 1, 0}, {0, 1, 1}, {1, 0, 1}, {1, 2, 0}, {1, 0, 2}, {2, 1, 0}, {0, 1, 2},
                               {2, 0, 1}, {0, 2, 1}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};
constexpr int kExp27[27][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2},
                               {1, 1, 0}, {0, 1, 1}, {1, 0, 1}, {1, 2, 0}, {1, 0, 2}, {2, 1, 0}, {0, 1, 2},
                               {2, 0, 1}, {0, 2, 1}, {1, 1, 1}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {2, 1, 1},
                               {1, 2, 1}, {1, 1, 2}, {2, 2, 1}, {2, 1, 2}, {1, 2, 2}, {2, 2, 2}};

struct BasisD3Q19 {
  using Lat = D3Q19Lat;
  static constexpr int Q = 19;
  static constexpr Poly W(int k) { return mono(kExp19[k][0], kExp19[k][1], kExp19[k][2]); }
  static constexpr Poly P(int k) { return (k >= 4 && k < 10) ? deg2_user(k - 4) : W(k); }
  static constexpr int lam_deg(int k) { return phomdeg(P(k)); }
};

struct BasisD3Q27 {
  using Lat = D3Q27Lat;
  static constexpr int Q = 27;
  static constexpr Poly W(int k) { return mono(kExp27[k][0], kExp27[k][1], kExp27[k][2]); }
  static constexpr Poly P(int k) { return (k >= 4 && k < 10) ? deg2_user(k - 4) : W(k); }
  static constexpr int lam_deg(int k) { return phomdeg(P(k)); }
};

// ---------------------------------------------------------------- derived tables
template <int Q>
struct Derived {
  Mat<Q> MW, MWinv;     // W_l(c_j) and its inverse
  Mat<Q> MP;            // P_k(c_j) (fixed-frame user moments)
  Mat<Q> R, Rinv;       // P = R W
  Mat<Q> E[3][kP];      // E[a][n] = D_a^n / n!, n = 1..kDeg
  int nmax[3];          // largest n with E[a][n] != 0
  Rat a[Q];             // m^eq_W(rho, u) = rho (a + b.u + u.C.u)
  Rat b[Q][3];
  Rat C[Q][3][3];
  Rat w[Q];
  Rat restP[Q];         // M_P(0) w: user moments of the rest state per unit density
  int lam_deg[Q];
  // sparse rows used by the kernels (columns restricted as noted)
  SpRow<Q> sMW[Q];        // M_W(0) rows, all columns
  SpRow<Q> sMP[Q];        // M_P(0) rows, all columns
  SpRow<Q> sMWinv[Q];     // M_W(0)^{-1} rows, non-conserved columns
  SpRow<Q> sR[Q];         // R rows, non-conserved columns
  SpRow<Q> sRinv[Q];      // R^{-1} rows, non-conserved columns
  SpRow<Q> sE[3][kP][Q];  // D_a^n / n! rows, non-conserved columns
  // transposed rows for the adjoint
  SpRow<Q> tMWinv[Q];     // row k: (j, M_W^{-1}[j][k]), all j
  SpRow<Q> tMW[Q];        // row j: (k, M_W[k][j]), non-conserved k
  SpRow<Q> tR[Q];         // row l: (k, R[k][l]), non-conserved k
  SpRow<Q> tRinv[Q];      // row l: (k, R^{-1}[k][l]), non-conserved k
  SpRow<Q> tE[3][kP][Q];  // row l: (k, (D_a^n / n!)[k][l]), non-conserved k
  bool ok_rank, ok_closed, ok_R, ok_conserved, ok_lower, ok_hom;
};

template <class B>
constexpr Derived<B::Q> derive() {
  using L = typename B::Lat;
  constexpr int Q = B::Q;
  Derived<Q> t{};
  for (int k = 0; k < Q; ++k)
    for (int j = 0; j < Q; ++j) {
      t.MW.m[k][j] = peval(B::W(k), L::c[j].x, L::c[j].y, L::c[j].z);
      t.MP.m[k][j] = peval(B::P(k), L::c[j].x, L::c[j].y, L::c[j].z);
    }
  auto inv = minv(t.MW);
  t.ok_rank = inv.ok;
  t.MWinv = inv.inv;
  // Express a polynomial in W through its lattice values, then verify the
  // identity as polynomials (so nothing relies on lattice aliasing).
  auto express = [&](const Poly& p, Rat* coef) -> bool {
    Rat vals[Q];
    for (int j = 0; j < Q; ++j) vals[j] = peval(p, L::c[j].x, L::c[j].y, L::c[j].z);
    for (int l = 0; l < Q; ++l) {
      Rat s;
      for (int j = 0; j < Q; ++j) s = s + vals[j] * t.MWinv.m[j][l];
      coef[l] = s;
    }
    Poly back;
    for (int l = 0; l < Q; ++l)
      if (!coef[l].zero()) back = padd(back, B::W(l), coef[l]);
    return peq(back, p);
  };
  t.ok_closed = true;
  Mat<Q> D[3];
  for (int ax = 0; ax < 3; ++ax)
    for (int k = 0; k < Q; ++k) t.ok_closed = express(pderiv(B::W(k), ax), D[ax].m[k]) && t.ok_closed;
  t.ok_R = true;
  for (int k = 0; k < Q; ++k) t.ok_R = express(B::P(k), t.R.m[k]) && t.ok_R;
  auto rinv = minv(t.R);
  t.ok_R = t.ok_R && rinv.ok;
  t.Rinv = rinv.inv;
  // conserved block: W_0 = 1, W_1..W_D = X_1..X_D, and R is the identity there
  t.ok_conserved = true;
  for (int k = 0; k <= L::D; ++k) {
    Poly expect = mono(k == 1, k == 2, k == 3);
    t.ok_conserved = t.ok_conserved && peq(B::W(k), expect);
    for (int l = 0; l < Q; ++l)
      t.ok_conserved = t.ok_conserved && t.R.m[k][l] == Rat(k == l ? 1 : 0) && t.R.m[l][k] == Rat(k == l ? 1 : 0);
  }
  // exponential series of the derivations
  t.ok_lower = true;
  for (int ax = 0; ax < 3; ++ax) {
    Mat<Q> Pn = D[ax];
    t.nmax[ax] = 0;
    Rat fact(1);
    for (int n = 1; n <= kDeg; ++n) {
      fact = fact * Rat(n);
      t.E[ax][n] = mscale(Pn, Rat(1) / fact);
      if (!mzero(Pn)) t.nmax[ax] = n;
      Pn = mmul(Pn, D[ax]);
    }
    t.ok_lower = t.ok_lower && mzero(Pn);  // nilpotent within kDeg steps
    for (int k = 0; k < Q; ++k)            // strictly lower triangular
      for (int l = k; l < Q; ++l) t.ok_lower = t.ok_lower && D[ax].m[k][l].zero();
  }
  // equilibrium moments in W coordinates (second-order polynomial equilibrium;
  // the paper leaves f^eq open):
  // f^eq_j = w_j rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 |u|^2)
  for (int j = 0; j < Q; ++j) t.w[j] = L::w(j);
  for (int k = 0; k < Q; ++k) {
    Rat a;
    Rat b[3] = {};
    Rat C[3][3] = {};
    for (int j = 0; j < Q; ++j) {
      Rat mw = t.MW.m[k][j] * t.w[j];
      int cj[3] = {L::c[j].x, L::c[j].y, L::c[j].z};
      a = a + mw;
      for (int al = 0; al < 3; ++al) {
        b[al] = b[al] + Rat(3) * mw * Rat(cj[al]);
        for (int be = 0; be < 3; ++be) C[al][be] = C[al][be] + Rat(9, 2) * mw * Rat(cj[al] * cj[be]);
      }
    }
    t.a[k] = a;
    for (int al = 0; al < 3; ++al) {
      t.b[k][al] = b[al];
      for (int be = 0; be < 3; ++be) t.C[k][al][be] = C[al][be] - (al == be ? Rat(3, 2) * a : Rat(0));
    }
  }
  for (int k = 0; k < Q; ++k) {
    Rat r;
    for (int j = 0; j < Q; ++j) r = r + t.MP.m[k][j] * t.w[j];
    t.restP[k] = r;
  }
  const int nc = L::D + 1;
  for (int k = 0; k < Q; ++k) {
    t.sMW[k] = sprow(t.MW, k, 0);
    t.sMP[k] = sprow(t.MP, k, 0);
    t.sMWinv[k] = sprow(t.MWinv, k, nc);
    t.sR[k] = sprow(t.R, k, nc);
    t.sRinv[k] = sprow(t.Rinv, k, nc);
    for (int ax = 0; ax < 3; ++ax)
      for (int n = 1; n < kP; ++n) t.sE[ax][n][k] = sprow(t.E[ax][n], k, nc);
  }
  {
    const Mat<Q> MWinvT = mtrans(t.MWinv), MWT = mtrans(t.MW), RT = mtrans(t.R), RinvT = mtrans(t.Rinv);
    for (int k = 0; k < Q; ++k) {
      t.tMWinv[k] = sprow(MWinvT, k, 0);
      t.tMW[k] = sprow(MWT, k, nc);
      t.tR[k] = sprow(RT, k, nc);
      t.tRinv[k] = sprow(RinvT, k, nc);
    }
    for (int ax = 0; ax < 3; ++ax)
      for (int n = 1; n < kP; ++n) {
        const Mat<Q> ET = mtrans(t.E[ax][n]);
        for (int k = 0; k < Q; ++k) t.tE[ax][n][k] = sprow(ET, k, nc);
      }
  }
  t.ok_hom = true;
  for (int k = 0; k < Q; ++k) {
    t.lam_deg[k] = B::lam_deg(k);
    t.ok_hom = t.ok_hom && t.lam_deg[k] >= 0;
  }
  return t;
}

template <class B>
struct Tab {
  static constexpr Derived<B::Q> t = derive<B>();
  static_assert(t.ok_rank, "M(0) of the working basis must be invertible on the lattice");
  static_assert(t.ok_closed, "span of the basis must be closed under differentiation");
  static_assert(t.ok_R, "user basis must span the same space as the working basis");
  static_assert(t.ok_conserved, "basis must start with 1, X_1..X_d");
  static_assert(t.ok_lower, "derivations must be nilpotent and strictly lower triangular");
  static_assert(t.ok_hom, "basis elements must be lambda-homogeneous");
};

}  // namespace lbmrv
