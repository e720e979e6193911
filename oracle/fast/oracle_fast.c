/*
 * Oracle B: the relative-velocity step in plain C, FP64, OpenMP over nodes.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests and by the CPU-baseline leg of the
 * benchmark; never by the HIP library.  Shares no code or tables with it: the
 * lattice, weights and basis polynomials are passed in by oracle/fast.py from
 * oracle/lattices.py.
 *
 * It follows the definition of section 1.2 of the paper node by node, exactly
 * as Oracle A does:
 *   rho = sum f, q = sum v f, u = q / rho                          eq. (rhoq)
 *   u~ = 0 | alpha u | given field                                  section 1.2
 *   f^eq_j = w_j rho (1 + v.u/cs2 + (v.u)^2/(2 cs2^2) - |u|^2/(2 cs2))
 *   M(u~)_kj = P_k(v_j - u~) from the polynomial terms              eq. (MatMu)
 *   m = M f, m^eq = M f^eq, m*_k = m_k + s_k (m^eq_k - m_k)         eq. (relaxationu)
 *   f* = M(u~)^{-1} m*  by Gaussian elimination, partial pivoting
 *   f_j(x + c_j) = f*_j(x), periodic                                 eq. (transport)
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define QMAX 27

typedef struct {
  int d, q;
  const int *c;            /* [q][3] integer directions, v_j = la * c_j */
  const double *w;         /* [q] weights */
  int nterms;
  const int *term_poly;    /* [nterms] basis index of each monomial term */
  const int *term_exp;     /* [nterms][3] exponents of X, Y, Z */
  const double *term_coef; /* [nterms] coefficients (lambda already applied) */
  double la;
} ob_lattice;

static double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

/* Solve A x = b (A n x n row-major, destroyed); x returned in b.  0 = ok. */
static int gauss_solve(int n, double *A, double *b) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    double best = fabs(A[col * n + col]);
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[r * n + col]) > best) { best = fabs(A[r * n + col]); piv = r; }
    if (best == 0.0) return -1;
    if (piv != col) {
      for (int j = 0; j < n; ++j) { double t = A[col * n + j]; A[col * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
      double t = b[col]; b[col] = b[piv]; b[piv] = t;
    }
    for (int r = col + 1; r < n; ++r) {
      double f = A[r * n + col] / A[col * n + col];
      if (f == 0.0) continue;
      for (int j = col; j < n; ++j) A[r * n + j] -= f * A[col * n + j];
      b[r] -= f * b[col];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int j = r + 1; j < n; ++j) s -= A[r * n + j] * b[j];
    b[r] = s / A[r * n + r];
  }
  return 0;
}

/* Relaxation at every node: fstar[q][N] from f[q][N].  mode 0/1/2 = zero/fluid/field. */
int ob_collide(const ob_lattice *L, const double *s, int mode, double alpha, const double *field, int64_t N,
               const double *f, double *fstar, int nthreads) {
  const int q = L->q, d = L->d;
  const double la = L->la, cs2 = la * la / 3.0;
  int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(| : bad)
  for (int64_t n = 0; n < N; ++n) {
    double fn[QMAX], feq[QMAX], M[QMAX * QMAX], m[QMAX], meq[QMAX];
    double rho = 0.0, qm[3] = {0, 0, 0}, u[3] = {0, 0, 0}, ut[3] = {0, 0, 0};
    for (int j = 0; j < q; ++j) {
      fn[j] = f[(int64_t)j * N + n];
      rho += fn[j];
      for (int a = 0; a < d; ++a) qm[a] += la * L->c[3 * j + a] * fn[j];
    }
    for (int a = 0; a < d; ++a) u[a] = qm[a] / rho;
    for (int a = 0; a < d; ++a)
      ut[a] = mode == 0 ? 0.0 : mode == 1 ? alpha * u[a] : field[(int64_t)a * N + n];
    double uu = 0.0;
    for (int a = 0; a < d; ++a) uu += u[a] * u[a];
    for (int j = 0; j < q; ++j) {
      double vu = 0.0;
      for (int a = 0; a < d; ++a) vu += la * L->c[3 * j + a] * u[a];
      feq[j] = L->w[j] * rho * (1.0 + vu / cs2 + vu * vu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
    /* M(u~)_kj = P_k(v_j - u~) */
    for (int i = 0; i < q * q; ++i) M[i] = 0.0;
    for (int j = 0; j < q; ++j) {
      double X[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) X[a] = la * L->c[3 * j + a] - ut[a];
      for (int t = 0; t < L->nterms; ++t) {
        const int *e = L->term_exp + 3 * t;
        M[L->term_poly[t] * q + j] += L->term_coef[t] * ipow(X[0], e[0]) * ipow(X[1], e[1]) * ipow(X[2], e[2]);
      }
    }
    for (int k = 0; k < q; ++k) {
      double a = 0.0, b = 0.0;
      for (int j = 0; j < q; ++j) { a += M[k * q + j] * fn[j]; b += M[k * q + j] * feq[j]; }
      m[k] = a;
      meq[k] = b;
    }
    for (int k = 0; k < q; ++k) m[k] = m[k] + s[k] * (meq[k] - m[k]); /* m* */
    if (gauss_solve(q, M, m)) bad = 1;
    for (int j = 0; j < q; ++j) fstar[(int64_t)j * N + n] = m[j];
  }
  return bad ? -1 : 0;
}

/* Transport: out_j(x) = in_j(x - c_j), periodic; dims = (nx, ny, nz). */
void ob_stream(const ob_lattice *L, const int64_t *dims, const double *in, double *out, int nthreads) {
  const int64_t nx = dims[0], ny = dims[1], nz = dims[2], N = nx * ny * nz;
  for (int j = 0; j < L->q; ++j) {
    const int cx = L->c[3 * j], cy = L->c[3 * j + 1], cz = L->c[3 * j + 2];
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t zy = 0; zy < nz * ny; ++zy) {
      const int64_t z = zy / ny, y = zy % ny;
      const int64_t zs = ((z - cz) % nz + nz) % nz, ys = ((y - cy) % ny + ny) % ny;
      const double *src = in + (int64_t)j * N + (zs * ny + ys) * nx;
      double *dst = out + (int64_t)j * N + (z * ny + y) * nx;
      for (int64_t x = 0; x < nx; ++x) dst[x] = src[((x - cx) % nx + nx) % nx];
    }
  }
}

/* nsteps full steps; f [q][N] in/out, scratch [q][N]. */
int ob_run(const ob_lattice *L, const double *s, int mode, double alpha, const double *field, const int64_t *dims,
           int64_t nsteps, double *f, double *scratch, int nthreads) {
  const int64_t N = dims[0] * dims[1] * dims[2];
  for (int64_t t = 0; t < nsteps; ++t) {
    if (ob_collide(L, s, mode, alpha, field, N, f, scratch, nthreads)) return -1;
    ob_stream(L, dims, scratch, f, nthreads);
  }
  return 0;
}
