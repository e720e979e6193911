/*
 * Oracle B, triangular-solve form: the relative-velocity step in plain C,
 * FP64, for long runs on large grids (the stored full-size references).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests and by the scripts that write
 * stored reference values; never by the HIP library.  Shares no code or tables
 * with it: the lattice, weights, basis polynomials and M(0)^{-1} are passed in
 * by oracle/fast.py, which builds them from oracle/lattices.py.
 *
 * Same definition as Oracle A and Oracle B (section 1.2 of the paper), node by
 * node:
 *   rho = sum f, q = sum v f, u = q / rho                          eq. (rhoq)
 *   u~ = 0 | alpha u | given field                                  section 1.2
 *   f^eq_j = w_j rho (1 + v.u/cs2 + (v.u)^2/(2 cs2^2) - |u|^2/(2 cs2))
 *   M(u~)_kj = P_k(v_j - u~) from the polynomial terms              eq. (MatMu)
 *   m = M f, m^eq = M f^eq, m*_k = m_k + s_k (m^eq_k - m_k)         eq. (relaxationu)
 *   f* = M(u~)^{-1} m*                                              section 1.2
 *   f_j(x + c_j) = f*_j(x), periodic                                 eq. (transport)
 * The only difference from Oracle B is how M(u~) x = m* is solved.  Section
 * 1.3 factors the shifted moment matrix as M(u~) = T(u~) M(0) (eq. (matTu)),
 * with T(u~) = M(u~) M(0)^{-1} unit lower triangular when the basis is ordered
 * by degree and its span is closed under differentiation (Prop. th:csd2q9 and
 * the discussion after it).  So here, per node,
 *   T(u~)_kl = sum_i M(u~)_ki M(0)^{-1}_il        (l < k: the strict lower part)
 *   y_k = m*_k - sum_{l<k} T(u~)_kl y_l           (forward substitution)
 *   f*  = M(0)^{-1} y.
 * The caller checks beforehand that T(u~) is unit lower triangular for its
 * basis (oracle/fast.py).  There is no pivoting and no branch on data, so the
 * nodes are processed in batches of NB with the node index innermost, and
 * every loop over the batch is a plain vector loop.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define QMAX 27
#define EMAX 8 /* largest exponent of a basis monomial */
#define NB 32  /* nodes per batch (measured: 32 runs 3.5x faster than 8 or 16 on AVX2) */

typedef struct {
  int d, q;
  const int *c;            /* [q][3] integer directions, v_j = la * c_j */
  const double *w;         /* [q] weights */
  int nterms;
  const int *term_poly;    /* [nterms] basis index of each monomial term */
  const int *term_exp;     /* [nterms][3] exponents of X, Y, Z */
  const double *term_coef; /* [nterms] coefficients (lambda already applied) */
  double la;
} ot_lattice;

/* One batch of nb <= NB consecutive nodes starting at n0; lanes past nb repeat
 * the last node and are not stored. */
static void collide_batch(const ot_lattice *L, const double *M0inv, const double *s, int mode, double alpha,
                          const double *field, int64_t N, const double *f, double *fstar, int64_t n0, int nb) {
  const int q = L->q, d = L->d;
  const double la = L->la, cs2 = la * la / 3.0;
  double fn[QMAX][NB], feq[QMAX][NB], M[QMAX][QMAX][NB], m[QMAX][NB], y[QMAX][NB];
  double rho[NB], u[3][NB], ut[3][NB], uu[NB];
  int64_t idx[NB];
  for (int b = 0; b < NB; ++b) idx[b] = n0 + (b < nb ? b : nb - 1);

  for (int j = 0; j < q; ++j)
    for (int b = 0; b < NB; ++b) fn[j][b] = f[(int64_t)j * N + idx[b]];
  /* conserved moments and u */
  for (int b = 0; b < NB; ++b) rho[b] = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < NB; ++b) u[a][b] = 0.0;
  for (int j = 0; j < q; ++j) {
    for (int b = 0; b < NB; ++b) rho[b] += fn[j][b];
    for (int a = 0; a < d; ++a) {
      const double v = la * L->c[3 * j + a];
      for (int b = 0; b < NB; ++b) u[a][b] += v * fn[j][b];
    }
  }
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < NB; ++b) u[a][b] = u[a][b] / rho[b];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < NB; ++b)
      ut[a][b] = a >= d ? 0.0 : mode == 0 ? 0.0 : mode == 1 ? alpha * u[a][b] : field[(int64_t)a * N + idx[b]];
  /* equilibrium */
  for (int b = 0; b < NB; ++b) {
    double s2 = 0.0;
    for (int a = 0; a < d; ++a) s2 += u[a][b] * u[a][b];
    uu[b] = s2;
  }
  for (int j = 0; j < q; ++j)
    for (int b = 0; b < NB; ++b) {
      double vu = 0.0;
      for (int a = 0; a < d; ++a) vu += la * L->c[3 * j + a] * u[a][b];
      feq[j][b] = L->w[j] * rho[b] * (1.0 + vu / cs2 + vu * vu / (2.0 * cs2 * cs2) - uu[b] / (2.0 * cs2));
    }
  /* M(u~)_kj = P_k(v_j - u~) */
  memset(M, 0, sizeof(M));
  for (int j = 0; j < q; ++j) {
    double pw[3][EMAX + 1][NB];
    for (int a = 0; a < 3; ++a) {
      const double v = a < d ? la * L->c[3 * j + a] : 0.0;
      for (int b = 0; b < NB; ++b) {
        const double X = v - ut[a][b];
        pw[a][0][b] = 1.0;
        for (int e = 1; e <= EMAX; ++e) pw[a][e][b] = pw[a][e - 1][b] * X;
      }
    }
    for (int t = 0; t < L->nterms; ++t) {
      const int *e = L->term_exp + 3 * t;
      const int k = L->term_poly[t];
      const double co = L->term_coef[t];
      for (int b = 0; b < NB; ++b) M[k][j][b] += co * pw[0][e[0]][b] * pw[1][e[1]][b] * pw[2][e[2]][b];
    }
  }
  /* m* = m + s (m^eq - m), m = M f, m^eq = M f^eq (each sum in increasing j;
     the loops run j outside so that the q sums advance side by side) */
  double e[QMAX][NB];
  for (int k = 0; k < q; ++k)
    for (int b = 0; b < NB; ++b) m[k][b] = e[k][b] = 0.0;
  for (int j = 0; j < q; ++j)
    for (int k = 0; k < q; ++k)
      for (int b = 0; b < NB; ++b) {
        m[k][b] += M[k][j][b] * fn[j][b];
        e[k][b] += M[k][j][b] * feq[j][b];
      }
  for (int k = 0; k < q; ++k)
    for (int b = 0; b < NB; ++b) m[k][b] = m[k][b] + s[k] * (e[k][b] - m[k][b]);
  /* T(u~) y = m*, row by row: T(u~)_kl = sum_i M(u~)_ki M(0)^{-1}_il for l < k
     (sums in increasing i), then y_k = m*_k - sum_{l<k} T(u~)_kl y_l */
  for (int k = 0; k < q; ++k) {
    double T[QMAX][NB], acc[NB];
    for (int l = 0; l < k; ++l)
      for (int b = 0; b < NB; ++b) T[l][b] = 0.0;
    for (int i = 0; i < q; ++i)
      for (int l = 0; l < k; ++l) {
        const double mi = M0inv[i * q + l];
        for (int b = 0; b < NB; ++b) T[l][b] += M[k][i][b] * mi;
      }
    for (int b = 0; b < NB; ++b) acc[b] = m[k][b];
    for (int l = 0; l < k; ++l)
      for (int b = 0; b < NB; ++b) acc[b] -= T[l][b] * y[l][b];
    for (int b = 0; b < NB; ++b) y[k][b] = acc[b];
  }
  /* f* = M(0)^{-1} y (sums in increasing k) */
  double fs[QMAX][NB];
  for (int j = 0; j < q; ++j)
    for (int b = 0; b < NB; ++b) fs[j][b] = 0.0;
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < q; ++j) {
      const double mi = M0inv[j * q + k];
      for (int b = 0; b < NB; ++b) fs[j][b] += mi * y[k][b];
    }
  for (int j = 0; j < q; ++j)
    for (int b = 0; b < nb; ++b) fstar[(int64_t)j * N + n0 + b] = fs[j][b];
}

/* Relaxation at every node: fstar[q][N] from f[q][N].  mode 0/1/2 = zero/fluid/field. */
void ot_collide(const ot_lattice *L, const double *M0inv, const double *s, int mode, double alpha,
                const double *field, int64_t N, const double *f, double *fstar, int nthreads) {
  const int64_t nbatch = (N + NB - 1) / NB;
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t i = 0; i < nbatch; ++i) {
    const int64_t n0 = i * NB;
    const int nb = (int)(N - n0 < NB ? N - n0 : NB);
    collide_batch(L, M0inv, s, mode, alpha, field, N, f, fstar, n0, nb);
  }
}

/* Transport: out_j(x) = in_j(x - c_j), periodic; dims = (nx, ny, nz). */
void ot_stream(const ot_lattice *L, const int64_t *dims, const double *in, double *out, int nthreads) {
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
void ot_run(const ot_lattice *L, const double *M0inv, const double *s, int mode, double alpha, const double *field,
            const int64_t *dims, int64_t nsteps, double *f, double *scratch, int nthreads) {
  const int64_t N = dims[0] * dims[1] * dims[2];
  for (int64_t t = 0; t < nsteps; ++t) {
    ot_collide(L, M0inv, s, mode, alpha, field, N, f, scratch, nthreads);
    ot_stream(L, dims, scratch, f, nthreads);
  }
}
