// C-ABI layer of liblbmrv: argument validation, context, call sequencing.
//
// Host code only, apart from the final deterministic reduction kernel of
// lbmrv_conservation.  Validation happens before any HIP call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <array>
#include <mutex>
#include <new>
#include <vector>

#include "lbmrv.h"
#include "launch.hpp"

namespace lbmrv {

// Totals of the kRedBlocks rows of five partial sums, in a fixed order:
// out[0] = sum + add0, out[1 + a] = scale * sum (a < d, else 0), out[4] = the
// count of non-finite values.
__global__ __launch_bounds__(kRedThreads) void k_conserve_final(const double* partial, double* out, double add0,
                                                                double scale, int d) {
  __shared__ double red[5][kRedThreads];
  double acc[5] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < kRedBlocks; b += kRedThreads)
    for (int i = 0; i < 5; ++i) acc[i] += partial[(uint64_t)b * 5 + i];
  for (int i = 0; i < 5; ++i) red[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int i = 0; i < 5; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0][0] + add0;
  if (threadIdx.x >= 1 && threadIdx.x <= 3) out[threadIdx.x] = (int)threadIdx.x <= d ? scale * red[threadIdx.x][0] : 0.0;
  if (threadIdx.x == 4) out[4] = red[4][0];
}

__global__ __launch_bounds__(256) void k_fill_zero(double* p, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// grad_s[k] = sum over blocks of partial[b][k]; zero for the conserved moments
// k <= d.  One workgroup of 32 x 32 threads: thread (k, r) adds the rows
// b = r (mod 32) in increasing b into four interleaved sums, which then meet
// in a fixed tree, so the result does not depend on scheduling.
constexpr int kRedCols = 32, kRedRows = 32;
__global__ __launch_bounds__(kRedCols* kRedRows) void k_reduce_columns(const double* partial, uint64_t nblocks,
                                                                        int q, int d, double* out) {
  __shared__ double red[kRedRows][kRedCols];
  const int k = threadIdx.x, r = threadIdx.y;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (k < q && k > d) {
    uint64_t b = r;
    for (; b + 3 * kRedRows < nblocks; b += 4 * kRedRows)
      for (int m = 0; m < 4; ++m) s[m] += partial[(b + m * kRedRows) * q + k];
    for (int m = 0; b < nblocks; b += kRedRows, ++m) s[m] += partial[b * q + k];
  }
  red[r][k] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  for (int half = kRedRows / 2; half > 0; half >>= 1) {
    if (r < half) red[r][k] += red[r + half][k];
    __syncthreads();
  }
  if (r == 0 && k < q) out[k] = red[0][k];
}

namespace {

using StepFn = hipError_t (*)(const StepLaunch&);
using AdjFn = hipError_t (*)(const AdjLaunch&);
using FinFn = hipError_t (*)(void*, uint32_t, uint32_t, uint32_t, uint64_t, const FinArgs&, hipStream_t);
using MomFn = hipError_t (*)(const MomLaunch&);
using ConsFn = hipError_t (*)(const void*, uint64_t, double*, hipStream_t);
using InitFn = hipError_t (*)(const InitLaunch&);
using ConvFn = hipError_t (*)(const void*, void*, double, uint64_t, int, hipStream_t);
using DevNormFn = hipError_t (*)(const void*, uint64_t, const DevRef&, double*, hipStream_t);
using DevScaleFn = hipError_t (*)(void*, uint64_t, const DevRef&, double, hipStream_t);

struct Entry {
  StepFn step[3];
  MomFn mom[3];
  ConsFn cons[3];
  InitFn init[3];
  ConvFn conv[3];
  AdjFn adj[3];
  AdjFn adj2[3];
  FinFn fin[3];
  DevNormFn dnorm[3];
  DevScaleFn dscale[3];
};

#define LBMRV_ENTRY(NAME)                                                                 \
  Entry {                                                                                 \
    {launch_step_##NAME##_f64, launch_step_##NAME##_f32, launch_step_##NAME##_f16},       \
        {launch_moments_##NAME##_f64, launch_moments_##NAME##_f32, launch_moments_##NAME##_f16}, \
        {launch_conserve_##NAME##_f64, launch_conserve_##NAME##_f32, launch_conserve_##NAME##_f16}, \
        {launch_init_##NAME##_f64, launch_init_##NAME##_f32, launch_init_##NAME##_f16},   \
        {launch_convert_##NAME##_f64, launch_convert_##NAME##_f32, launch_convert_##NAME##_f16}, \
        {launch_adjoint_##NAME##_f64, launch_adjoint_##NAME##_f32, launch_adjoint_##NAME##_f16}, \
        {launch_adjoint2_##NAME##_f64, launch_adjoint2_##NAME##_f32, launch_adjoint2_##NAME##_f16}, \
        {launch_aa_finish_##NAME##_f64, launch_aa_finish_##NAME##_f32, launch_aa_finish_##NAME##_f16}, \
        {launch_devnorm_##NAME##_f64, launch_devnorm_##NAME##_f32, launch_devnorm_##NAME##_f16}, \
        {launch_devscale_##NAME##_f64, launch_devscale_##NAME##_f32, launch_devscale_##NAME##_f16} \
  }

const Entry kEntries[4] = {LBMRV_ENTRY(d2q9_paper), LBMRV_ENTRY(d2q9_geier), LBMRV_ENTRY(d3q19),
                           LBMRV_ENTRY(d3q27)};

}  // namespace
}  // namespace lbmrv

using namespace lbmrv;

struct lbmrv_ctx {
  int lattice, basis, storage;
  int d, q;
  int entry;      // index into kEntries
  int sk;         // StorageKind
  int streaming;  // LBMRV_STREAM_*
  int block;
  double lambda;
  double s[27];
  uint32_t nx, ny, nz;
  uint64_t N;
  double rho0;    // 0 unless a deviation storage
  double* partial = nullptr;  // kRedBlocks * 5 partial sums + 5 results (device)
  int partial_dev = -1;
  uint32_t wall_mask = 0;     // half-way bounce-back faces (bit 2a + side)
  double wall_u[6][3] = {};   // wall velocities (physical units)
  double rho_w = 1.0;
  int equilibrium = LBMRV_EQ_POLYNOMIAL;
  int block_order = LBMRV_ORDER_AUTO;
  // run-time basis P = R W (W the built-in working basis of `entry`)
  // adjoint: a second stream (default priority) on which segments are
  // recomputed ahead of the reverse sweep on the caller's stream, and the
  // events that order the two; created at the first lbmrv_adjoint call that
  // needs them, on that call's device
  hipStream_t astream = nullptr;
  hipEvent_t aev[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int astream_dev = -1;
  int custom = 0;
  std::vector<double> R;              // q x q
  std::vector<double> Rnn, Rnninv;    // non-conserved block and its inverse
  void* dtab = nullptr;               // device: [A | R | Rnn | Rnninv] in the arithmetic type
  int dtab_dev = -1;
};

namespace {

constexpr uint64_t kMaxNodes = (1ull << 32) - 256;

int lattice_q(int lattice) { return lattice == LBMRV_D2Q9 ? 9 : lattice == LBMRV_D3Q19 ? 19 : 27; }
int lattice_d(int lattice) { return lattice == LBMRV_D2Q9 ? 2 : 3; }
size_t elem_bytes(int storage) { return storage == LBMRV_F64 ? 8 : storage == LBMRV_F16DEV ? 2 : 4; }

int check_rates(int q, int d, const double* s) {
  if (!s) return LBMRV_ERR_INVALID_ARG;
  for (int k = 0; k < q; ++k) {
    if (!std::isfinite(s[k])) return LBMRV_ERR_INVALID_ARG;
    if (k <= d && s[k] != 0.0) return LBMRV_ERR_INVALID_ARG;  // conserved moments: s_k = 0
    if (s[k] < 0.0 || s[k] > 2.0) return LBMRV_ERR_INVALID_ARG;
  }
  return LBMRV_OK;
}

int check_ptr(const void* p, size_t align) {
  if (!p) return LBMRV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(p) % align) return LBMRV_ERR_ALIGNMENT;
  return LBMRV_OK;
}

int check_mode(const lbmrv_ctx* c, int ut_mode, double ut_alpha, const float* ut_field) {
  if (ut_mode != LBMRV_UT_ZERO && ut_mode != LBMRV_UT_FLUID && ut_mode != LBMRV_UT_FIELD)
    return LBMRV_ERR_INVALID_ARG;
  if (!std::isfinite(ut_alpha)) return LBMRV_ERR_INVALID_ARG;
  if (ut_mode == LBMRV_UT_FIELD) return check_ptr(ut_field, 4);
  (void)c;
  return LBMRV_OK;
}

// Contiguous tile ranges per XCD while the population array (q N elements)
// fits in the 256 MiB last-level cache (measured faster there, slower beyond).
uint32_t xcd_order(const lbmrv_ctx* c) {
  const bool small = (uint64_t)elem_bytes(c->storage) * c->q * c->N <= (256ull << 20);
  return c->block_order == LBMRV_ORDER_XCD || (c->block_order == LBMRV_ORDER_AUTO && small) ? 1u : 0u;
}

StepLaunch base_launch(const lbmrv_ctx* c, hipStream_t st) {
  StepLaunch L{};
  L.sk = c->sk;
  L.nx = c->nx;
  L.ny = c->ny;
  L.nz = c->nz;
  L.N = c->N;
  L.rho0 = c->rho0;
  L.alpha = 0;
  L.inv_lambda = 1.0 / c->lambda;
  for (int k = 0; k < 27; ++k) L.s[k] = k < c->q ? c->s[k] : 0.0;
  L.wall_mask = c->wall_mask;
  L.eq_maxwell = c->equilibrium == LBMRV_EQ_MAXWELLIAN ? 1u : 0u;
  for (int f = 0; f < 6; ++f)
    for (int ax = 0; ax < 3; ++ax) L.wall_coef[f][ax] = 6.0 * c->rho_w * c->wall_u[f][ax] / c->lambda;
  L.relax = c->custom ? c->dtab : nullptr;
  L.xcd_remap = xcd_order(c);
  L.stream = st;
  L.block = c->block;
  return L;
}

hipError_t run_kind(const lbmrv_ctx* c, int kind, const void* fin, void* fout, int mode, double alpha,
                    const float* ut, hipStream_t st) {
  StepLaunch L = base_launch(c, st);
  L.kind = kind;
  L.mode = mode;
  L.alpha = alpha;
  L.fin = fin;
  L.fout = fout;
  L.ut = ut;
  return kEntries[c->entry].step[c->sk](L);
}

// Launch count kernels alternating (kind_a: p -> q) and (kind_b: q -> p),
// starting with the first; p == q for the in-place form.
hipError_t run_alternating(lbmrv_ctx* c, int kind_a, int kind_b, void* p, void* q, int64_t count, int mode,
                           double alpha, const float* field, hipStream_t st) {
  for (int64_t i = 0; i < count; ++i) {
    const bool even = i % 2 == 0;
    hipError_t e = run_kind(c, even ? kind_a : kind_b, even ? p : q, even ? q : p, mode, alpha, field, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- run-time bases
// Polynomials as dense coefficient vectors over a list of monomials.
using Mono = std::array<int, 3>;

int mono_index(std::vector<Mono>& keys, int a, int b, int e) {
  for (size_t i = 0; i < keys.size(); ++i)
    if (keys[i][0] == a && keys[i][1] == b && keys[i][2] == e) return (int)i;
  keys.push_back({a, b, e});
  return (int)keys.size() - 1;
}

// Terms (monomial index, coefficient) of the built-in working basis W_l.
template <class B>
std::vector<std::vector<std::pair<int, double>>> working_terms(std::vector<Mono>& keys) {
  std::vector<std::vector<std::pair<int, double>>> w(B::Q);
  for (int l = 0; l < B::Q; ++l) {
    const Poly p = B::W(l);
    for (int i = 0; i < p.n; ++i) w[l].push_back({mono_index(keys, p.t[i].a, p.t[i].b, p.t[i].e), p.t[i].c.val()});
  }
  return w;
}

// Gauss-Jordan inverse with partial pivoting of an n x n row-major matrix;
// false if a pivot vanishes.
bool invert(std::vector<double> a, int n, std::vector<double>& inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + col]) > std::fabs(a[(size_t)piv * n + col])) piv = r;
    if (a[(size_t)piv * n + col] == 0.0) return false;
    for (int j = 0; j < n; ++j) {
      std::swap(a[(size_t)col * n + j], a[(size_t)piv * n + j]);
      std::swap(inv[(size_t)col * n + j], inv[(size_t)piv * n + j]);
    }
    const double p = a[(size_t)col * n + col];
    for (int j = 0; j < n; ++j) {
      a[(size_t)col * n + j] /= p;
      inv[(size_t)col * n + j] /= p;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = a[(size_t)r * n + col];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)r * n + j] -= f * a[(size_t)col * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)col * n + j];
      }
    }
  }
  return true;
}

double norm_inf(const std::vector<double>& a, int n) {
  double m = 0.0;
  for (int i = 0; i < n; ++i) {
    double r = 0.0;
    for (int j = 0; j < n; ++j) r += std::fabs(a[(size_t)i * n + j]);
    m = r > m ? r : m;
  }
  return m;
}

// Express the user polynomials in the working basis W of one built-in entry:
// P_k = sum_l R[k][l] W_l, by least squares over the monomial coefficients
// (modified Gram-Schmidt on the columns W_l, applied twice).  Returns false
// if some P_k is not in span(W) to 1e-12 relative.
template <class B>
bool express_in(const lbmrv_poly_basis* pb, std::vector<double>& R) {
  constexpr int Q = B::Q;
  std::vector<Mono> keys;
  auto wt = working_terms<B>(keys);
  std::vector<std::vector<std::pair<int, double>>> pt(Q);
  for (int t = 0; t < pb->nterms; ++t)
    pt[pb->poly_of_term[t]].push_back(
        {mono_index(keys, pb->exps[3 * t], pb->exps[3 * t + 1], pb->exps[3 * t + 2]), pb->coef[t]});
  const int nm = (int)keys.size();
  std::vector<double> Wc((size_t)Q * nm, 0.0), Pc((size_t)Q * nm, 0.0);  // column l: coefficients of W_l
  for (int l = 0; l < Q; ++l)
    for (auto& [i, c] : wt[l]) Wc[(size_t)l * nm + i] += c;
  for (int k = 0; k < Q; ++k)
    for (auto& [i, c] : pt[k]) Pc[(size_t)k * nm + i] += c;
  // W = Qm Rr (columns), Qm orthonormal
  std::vector<double> Qm = Wc, Rr((size_t)Q * Q, 0.0);
  for (int l = 0; l < Q; ++l) {
    double* ql = &Qm[(size_t)l * nm];
    for (int pass = 0; pass < 2; ++pass)
      for (int m = 0; m < l; ++m) {
        const double* qm = &Qm[(size_t)m * nm];
        double dot = 0.0;
        for (int i = 0; i < nm; ++i) dot += qm[i] * ql[i];
        for (int i = 0; i < nm; ++i) ql[i] -= dot * qm[i];
        Rr[(size_t)m * Q + l] += dot;
      }
    double nrm = 0.0;
    for (int i = 0; i < nm; ++i) nrm += ql[i] * ql[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return false;
    for (int i = 0; i < nm; ++i) ql[i] /= nrm;
    Rr[(size_t)l * Q + l] = nrm;
  }
  R.assign((size_t)Q * Q, 0.0);
  for (int k = 0; k < Q; ++k) {
    const double* pk = &Pc[(size_t)k * nm];
    double y[Q], x[Q];
    for (int l = 0; l < Q; ++l) {
      double dot = 0.0;
      for (int i = 0; i < nm; ++i) dot += Qm[(size_t)l * nm + i] * pk[i];
      y[l] = dot;
    }
    for (int l = Q - 1; l >= 0; --l) {  // Rr x = y (upper triangular)
      double v = y[l];
      for (int m = l + 1; m < Q; ++m) v -= Rr[(size_t)l * Q + m] * x[m];
      x[l] = v / Rr[(size_t)l * Q + l];
    }
    double res = 0.0, ref = 0.0;
    for (int i = 0; i < nm; ++i) {
      double v = pk[i];
      for (int l = 0; l < Q; ++l) v -= x[l] * Wc[(size_t)l * nm + i];
      res += v * v;
      ref += pk[i] * pk[i];
    }
    if (!(std::sqrt(res) <= 1e-12 * std::sqrt(ref))) return false;
    for (int l = 0; l < Q; ++l) R[(size_t)k * Q + l] = x[l];
  }
  return true;
}

// Validate a run-time basis and find the built-in entry whose working basis
// spans it; fills R, the non-conserved block of R and its inverse.
int analyse_basis(int lattice, const lbmrv_poly_basis* pb, int& entry, std::vector<double>& R,
                  std::vector<double>& Rnn, std::vector<double>& Rnninv) {
  const int q = lattice_q(lattice), d = lattice_d(lattice), nc = q - d - 1;
  if (!pb || pb->nterms < 1 || pb->nterms > 4096 || !pb->poly_of_term || !pb->exps || !pb->coef)
    return LBMRV_ERR_INVALID_ARG;
  std::vector<int> seen(q, 0);
  for (int t = 0; t < pb->nterms; ++t) {
    const int k = pb->poly_of_term[t];
    if (k < 0 || k >= q || !std::isfinite(pb->coef[t])) return LBMRV_ERR_INVALID_ARG;
    for (int a = 0; a < 3; ++a)
      if (pb->exps[3 * t + a] < 0 || pb->exps[3 * t + a] > 8) return LBMRV_ERR_INVALID_ARG;
    if (d == 2 && pb->exps[3 * t + 2] != 0 && pb->coef[t] != 0.0) return LBMRV_ERR_INVALID_ARG;
    seen[k] = 1;
  }
  for (int k = 0; k < q; ++k)
    if (!seen[k]) return LBMRV_ERR_INVALID_ARG;
  // the conserved polynomials, exactly: P_0 = 1, P_{1+a} = xi_a
  for (int k = 0; k <= d; ++k) {
    double sum[4] = {0, 0, 0, 0};  // coefficients of 1, xi_x, xi_y, xi_z
    double other = 0.0;
    for (int t = 0; t < pb->nterms; ++t) {
      if (pb->poly_of_term[t] != k) continue;
      const int* e = &pb->exps[3 * t];
      const int deg = e[0] + e[1] + e[2];
      if (deg == 0) sum[0] += pb->coef[t];
      else if (deg == 1) sum[1 + (e[0] ? 0 : e[1] ? 1 : 2)] += pb->coef[t];
      else other = std::fabs(pb->coef[t]) > other ? std::fabs(pb->coef[t]) : other;
    }
    for (int i = 0; i < 4; ++i)
      if (sum[i] != (i == k ? 1.0 : 0.0)) return LBMRV_ERR_INVALID_ARG;
    if (other != 0.0) return LBMRV_ERR_INVALID_ARG;
  }
  bool ok = false;
  if (lattice == LBMRV_D2Q9) {
    if ((ok = express_in<BasisD2Q9Paper>(pb, R))) entry = 0;
    else if ((ok = express_in<BasisD2Q9Geier>(pb, R))) entry = 1;
  } else if (lattice == LBMRV_D3Q19) {
    if ((ok = express_in<BasisD3Q19>(pb, R))) entry = 2;
  } else {
    if ((ok = express_in<BasisD3Q27>(pb, R))) entry = 3;
  }
  if (!ok) return LBMRV_ERR_INVALID_ARG;
  for (int k = 0; k <= d; ++k)
    for (int l = 0; l < q; ++l) R[(size_t)k * q + l] = k == l ? 1.0 : 0.0;
  Rnn.assign((size_t)nc * nc, 0.0);
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) Rnn[(size_t)i * nc + j] = R[(size_t)(d + 1 + i) * q + d + 1 + j];
  if (!invert(Rnn, nc, Rnninv)) return LBMRV_ERR_INVALID_ARG;
  const double cond = norm_inf(Rnn, nc) * norm_inf(Rnninv, nc);
  if (!(cond < 1e10)) return LBMRV_ERR_INVALID_ARG;
  return LBMRV_OK;
}

// Fill the device table of a run-time basis: A = Rnn^{-1} S Rnn, R, Rnn,
// Rnn^{-1}, in the arithmetic type of the storage.  Blocking; waits for the
// device first so that no kernel still reads the previous table.
int upload_basis(lbmrv_ctx* c) {
  const int q = c->q, d = c->d, nc = q - d - 1;
  std::vector<double> tab;
  tab.reserve((size_t)3 * nc * nc + (size_t)q * q);
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) {
      double a = 0.0;
      for (int k = 0; k < nc; ++k) a += c->Rnninv[(size_t)i * nc + k] * c->s[d + 1 + k] * c->Rnn[(size_t)k * nc + j];
      tab.push_back(a);
    }
  tab.insert(tab.end(), c->R.begin(), c->R.end());
  tab.insert(tab.end(), c->Rnn.begin(), c->Rnn.end());
  tab.insert(tab.end(), c->Rnninv.begin(), c->Rnninv.end());
  const bool f64 = c->storage == LBMRV_F64;
  const size_t bytes = tab.size() * (f64 ? 8 : 4);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBMRV_ERR_HIP;
  if (c->dtab && dev != c->dtab_dev) return LBMRV_ERR_INVALID_ARG;
  if (!c->dtab) {
    if (hipMalloc(&c->dtab, bytes) != hipSuccess) {
      c->dtab = nullptr;
      return LBMRV_ERR_HIP;
    }
    c->dtab_dev = dev;
  }
  if (hipDeviceSynchronize() != hipSuccess) return LBMRV_ERR_HIP;
  hipError_t e;
  if (f64) {
    e = hipMemcpy(c->dtab, tab.data(), bytes, hipMemcpyHostToDevice);
  } else {
    std::vector<float> t32(tab.begin(), tab.end());
    e = hipMemcpy(c->dtab, t32.data(), bytes, hipMemcpyHostToDevice);
  }
  return e == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
}

// Byte offsets of the tables inside dtab.
size_t tab_offset(const lbmrv_ctx* c, int which) {  // 0 A, 1 R, 2 Rnn, 3 Rnninv
  const size_t nc = (size_t)(c->q - c->d - 1), q = (size_t)c->q, eb = c->storage == LBMRV_F64 ? 8 : 4;
  const size_t off[4] = {0, nc * nc, nc * nc + q * q, 2 * nc * nc + q * q};
  return off[which] * eb;
}

const void* tab_ptr(const lbmrv_ctx* c, int which) {
  return c->custom ? static_cast<const char*>(c->dtab) + tab_offset(c, which) : nullptr;
}

// A context with a run-time basis must be used on the device its table lives on.
int check_device(const lbmrv_ctx* c) {
  if (!c->custom) return LBMRV_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBMRV_ERR_HIP;
  return dev == c->dtab_dev ? LBMRV_OK : LBMRV_ERR_INVALID_ARG;
}

}  // namespace

extern "C" {

int lbmrv_create(lbmrv_ctx** out, int lattice, int basis, double lambda, const double* s, const int64_t* dims,
                 int storage, double rho0) {
  if (!out) return LBMRV_ERR_INVALID_ARG;
  *out = nullptr;
  if (lattice != LBMRV_D2Q9 && lattice != LBMRV_D3Q19 && lattice != LBMRV_D3Q27) return LBMRV_ERR_INVALID_ARG;
  if (basis != LBMRV_BASIS_DEFAULT && basis != LBMRV_BASIS_GEIER) return LBMRV_ERR_INVALID_ARG;
  if (basis == LBMRV_BASIS_GEIER && lattice != LBMRV_D2Q9) return LBMRV_ERR_INVALID_ARG;
  if (!(std::isfinite(lambda) && lambda > 0.0)) return LBMRV_ERR_INVALID_ARG;
  if (storage < LBMRV_F64 || storage > LBMRV_F16DEV) return LBMRV_ERR_INVALID_ARG;
  if (!std::isfinite(rho0)) return LBMRV_ERR_INVALID_ARG;
  const int q = lattice_q(lattice), d = lattice_d(lattice);
  int rc = check_rates(q, d, s);
  if (rc) return rc;
  if (!dims) return LBMRV_ERR_INVALID_ARG;
  uint64_t e[3] = {1, 1, 1};
  for (int a = 0; a < d; ++a) {
    if (dims[a] < 1 || dims[a] > 65535 * 4096LL) return LBMRV_ERR_INVALID_ARG;
    e[a] = (uint64_t)dims[a];
  }
  if (e[1] > 65535 || e[2] > 65535) return LBMRV_ERR_INVALID_ARG;  // grid y/z limits
  const uint64_t N = e[0] * e[1] * e[2];
  // node indices are 32-bit (element offsets j * N + n are formed in 64 bits);
  // the bound also keeps one-dimensional launches of 256-thread blocks below
  // 2^32 work-items
  if (N > kMaxNodes) return LBMRV_ERR_INVALID_ARG;
  lbmrv_ctx* c = new (std::nothrow) lbmrv_ctx();
  if (!c) return LBMRV_ERR_INVALID_ARG;
  c->lattice = lattice;
  c->basis = basis;
  c->storage = storage;
  c->q = q;
  c->d = d;
  c->entry = lattice == LBMRV_D2Q9 ? (basis == LBMRV_BASIS_GEIER ? 1 : 0) : lattice == LBMRV_D3Q19 ? 2 : 3;
  c->sk = storage == LBMRV_F64 ? SK_F64 : storage == LBMRV_F16DEV ? SK_F16 : SK_F32;
  c->streaming = LBMRV_STREAM_PULL;
  c->block = 256;
  c->lambda = lambda;
  for (int k = 0; k < 27; ++k) c->s[k] = k < q ? s[k] : 0.0;
  c->nx = (uint32_t)e[0];
  c->ny = (uint32_t)e[1];
  c->nz = (uint32_t)e[2];
  c->N = N;
  c->rho0 = (storage == LBMRV_F32DEV || storage == LBMRV_F16DEV) ? rho0 : 0.0;
  *out = c;
  return LBMRV_OK;
}

int lbmrv_create_custom(lbmrv_ctx** out, int lattice, const lbmrv_poly_basis* basis, double lambda, const double* s,
                        const int64_t* dims, int storage, double rho0) {
  if (!out) return LBMRV_ERR_INVALID_ARG;
  *out = nullptr;
  if (lattice != LBMRV_D2Q9 && lattice != LBMRV_D3Q19 && lattice != LBMRV_D3Q27) return LBMRV_ERR_INVALID_ARG;
  int entry = -1;
  std::vector<double> R, Rnn, Rnninv;
  int rc = analyse_basis(lattice, basis, entry, R, Rnn, Rnninv);
  if (rc) return rc;
  lbmrv_ctx* c = nullptr;
  if ((rc = lbmrv_create(&c, lattice, entry == 1 ? LBMRV_BASIS_GEIER : LBMRV_BASIS_DEFAULT, lambda, s, dims, storage,
                         rho0)))
    return rc;
  c->basis = LBMRV_BASIS_CUSTOM;
  c->custom = 1;
  c->R = std::move(R);
  c->Rnn = std::move(Rnn);
  c->Rnninv = std::move(Rnninv);
  if ((rc = upload_basis(c))) {
    lbmrv_destroy(c);
    return rc;
  }
  *out = c;
  return LBMRV_OK;
}

int lbmrv_set_rates(lbmrv_ctx* c, const double* s) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  int rc = check_rates(c->q, c->d, s);
  if (rc) return rc;
  if ((rc = check_device(c))) return rc;
  double old[27];
  for (int k = 0; k < 27; ++k) old[k] = c->s[k];
  for (int k = 0; k < c->q; ++k) c->s[k] = s[k];
  if (c->custom && (rc = upload_basis(c))) {
    for (int k = 0; k < 27; ++k) c->s[k] = old[k];  // the context keeps its previous rates
    return rc;
  }
  return LBMRV_OK;
}

int lbmrv_set_streaming(lbmrv_ctx* c, int kind) {
  if (!c || (kind != LBMRV_STREAM_PULL && kind != LBMRV_STREAM_PUSH && kind != LBMRV_STREAM_AA))
    return LBMRV_ERR_INVALID_ARG;
  c->streaming = kind;
  return LBMRV_OK;
}

int lbmrv_set_equilibrium(lbmrv_ctx* c, int kind) {
  if (!c || (kind != LBMRV_EQ_POLYNOMIAL && kind != LBMRV_EQ_MAXWELLIAN)) return LBMRV_ERR_INVALID_ARG;
  c->equilibrium = kind;
  return LBMRV_OK;
}

int lbmrv_set_block_order(lbmrv_ctx* c, int order) {
  if (!c || (order != LBMRV_ORDER_AUTO && order != LBMRV_ORDER_NATURAL && order != LBMRV_ORDER_XCD))
    return LBMRV_ERR_INVALID_ARG;
  c->block_order = order;
  return LBMRV_OK;
}

int lbmrv_set_walls(lbmrv_ctx* c, uint32_t wall_mask, const double* wall_u, double rho_w) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  if (wall_mask >> (2 * c->d)) return LBMRV_ERR_INVALID_ARG;  // faces of existing axes only
  if (!std::isfinite(rho_w)) return LBMRV_ERR_INVALID_ARG;
  double u[6][3] = {};
  if (wall_u)
    for (int f = 0; f < 6; ++f)
      for (int ax = 0; ax < 3; ++ax) {
        if (!std::isfinite(wall_u[3 * f + ax])) return LBMRV_ERR_INVALID_ARG;
        u[f][ax] = (f < 2 * c->d && ax < c->d) ? wall_u[3 * f + ax] : 0.0;
      }
  c->wall_mask = wall_mask;
  for (int f = 0; f < 6; ++f)
    for (int ax = 0; ax < 3; ++ax) c->wall_u[f][ax] = u[f][ax];
  c->rho_w = rho_w;
  return LBMRV_OK;
}

int lbmrv_info(const lbmrv_ctx* c, int64_t* q, int64_t* d, int64_t* nodes, int64_t* bytes_per_pop) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  if (q) *q = c->q;
  if (d) *d = c->d;
  if (nodes) *nodes = (int64_t)c->N;
  if (bytes_per_pop) *bytes_per_pop = (int64_t)elem_bytes(c->storage);
  return LBMRV_OK;
}

int lbmrv_step(lbmrv_ctx* c, void* f_in, void* f_out, int ut_mode, double ut_alpha, const float* ut_field,
               int64_t nsteps, void* hip_stream) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  const size_t eb = elem_bytes(c->storage);
  int rc;
  if ((rc = check_ptr(f_in, eb)) || (rc = check_ptr(f_out, eb))) return rc;
  if (nsteps < 0) return LBMRV_ERR_INVALID_ARG;
  if (f_in == f_out && c->streaming != LBMRV_STREAM_AA) return LBMRV_ERR_INVALID_ARG;
  if ((rc = check_mode(c, ut_mode, ut_alpha, ut_field))) return rc;
  // walls: pull form, or the in-place form with walls on both faces of an axis
  // (a one-sided wall would let two nodes share one slot in place)
  if (c->wall_mask && c->streaming == LBMRV_STREAM_PUSH) return LBMRV_ERR_UNSUPPORTED;
  if (c->wall_mask && c->streaming == LBMRV_STREAM_AA)
    for (int a = 0; a < c->d; ++a)
      if (((c->wall_mask >> (2 * a)) & 1u) != ((c->wall_mask >> (2 * a + 1)) & 1u)) return LBMRV_ERR_UNSUPPORTED;
  if (c->custom && c->streaming == LBMRV_STREAM_AA) return LBMRV_ERR_UNSUPPORTED;
  if ((rc = check_device(c))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (c->streaming == LBMRV_STREAM_AA) {
    // One array, in place: even steps collide at the node and store each
    // population in its opposite slot, odd steps gather from the opposite slots
    // upstream and scatter downstream; after an odd count one swap pass
    // restores the natural layout.
    if (f_in != f_out &&
        hipMemcpyAsync(f_out, f_in, eb * c->q * c->N, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return LBMRV_ERR_HIP;
    hipError_t e = run_alternating(c, K_AA_EVEN, c->wall_mask ? K_AA_ODD_WALLS : K_AA_ODD, f_out, f_out, nsteps,
                                   ut_mode, ut_alpha, ut_field, st);
    if (e != hipSuccess) return LBMRV_ERR_HIP;
    if (nsteps % 2 == 1) {
      FinArgs w{};
      w.wall_mask = c->wall_mask;
      for (int f = 0; f < 6; ++f)
        for (int ax = 0; ax < 3; ++ax) w.wall_coef[f][ax] = 6.0 * c->rho_w * c->wall_u[f][ax] / c->lambda;
      e = kEntries[c->entry].fin[c->sk](f_out, c->nx, c->ny, c->nz, c->N, w, st);
    }
    return e == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
  }
  if (nsteps == 0) {
    return hipMemcpyAsync(f_out, f_in, eb * c->q * c->N, hipMemcpyDeviceToDevice, st) == hipSuccess
               ? LBMRV_OK
               : LBMRV_ERR_HIP;
  }
  hipError_t e = hipSuccess;
  if (c->streaming == LBMRV_STREAM_PUSH) {
    // Pre-collision state throughout: one fused collide-and-scatter pass per
    // step.  Out-of-place passes alternate between the two buffers, so an odd
    // number of them must run to end in f_out.  For even nsteps the first step
    // is split into an out-of-place collision (f_in -> f_out) and a transport
    // (f_out -> f_in), which adds one pass.
    void* cur = f_in;
    int64_t i0 = 0;
    if (nsteps % 2 == 0) {
      e = run_kind(c, K_COLLIDE, f_in, f_out, ut_mode, ut_alpha, ut_field, st);
      if (e == hipSuccess) e = run_kind(c, K_STREAM, f_out, f_in, LBMRV_UT_ZERO, 0.0, nullptr, st);
      if (e != hipSuccess) return LBMRV_ERR_HIP;
      i0 = 1;
    }
    e = run_alternating(c, K_PUSH, K_PUSH, cur, cur == f_in ? f_out : f_in, nsteps - i0, ut_mode, ut_alpha,
                        ut_field, st);
    return e == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
  }
  // Pull: collide once at the start, then nsteps - 1 fused transport+collide
  // passes, then one transport.  The out-of-place passes alternate buffers and
  // the last one writes f_out; the first collision is in place when nsteps is
  // odd and f_in -> f_out when it is even.
  void* cur;
  if (nsteps % 2 == 1) {
    e = run_kind(c, K_COLLIDE, f_in, f_in, ut_mode, ut_alpha, ut_field, st);
    cur = f_in;
  } else {
    e = run_kind(c, K_COLLIDE, f_in, f_out, ut_mode, ut_alpha, ut_field, st);
    cur = f_out;
  }
  if (e != hipSuccess) return LBMRV_ERR_HIP;
  void* other = (cur == f_in) ? f_out : f_in;
  e = run_alternating(c, K_PULL, K_PULL, cur, other, nsteps - 1, ut_mode, ut_alpha, ut_field, st);
  if (e != hipSuccess) return LBMRV_ERR_HIP;
  if ((nsteps - 1) % 2 == 1) cur = other;
  void* nxt = (cur == f_in) ? f_out : f_in;
  e = run_kind(c, K_STREAM, cur, nxt, LBMRV_UT_ZERO, 0.0, nullptr, st);
  return e == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
}

int lbmrv_collide(lbmrv_ctx* c, const void* f_in, void* f_out, int ut_mode, double ut_alpha, const float* ut_field,
                  void* hip_stream) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  const size_t eb = elem_bytes(c->storage);
  int rc;
  if ((rc = check_ptr(f_in, eb)) || (rc = check_ptr(f_out, eb))) return rc;
  if ((rc = check_mode(c, ut_mode, ut_alpha, ut_field))) return rc;
  if ((rc = check_device(c))) return rc;
  hipError_t e = run_kind(c, K_COLLIDE, f_in, f_out, ut_mode, ut_alpha, ut_field, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
}

int lbmrv_transport(lbmrv_ctx* c, const void* f_in, void* f_out, void* hip_stream) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  const size_t eb = elem_bytes(c->storage);
  int rc;
  if ((rc = check_ptr(f_in, eb)) || (rc = check_ptr(f_out, eb))) return rc;
  if (f_in == f_out) return LBMRV_ERR_INVALID_ARG;
  hipError_t e = run_kind(c, K_STREAM, f_in, f_out, LBMRV_UT_ZERO, 0.0, nullptr, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
}

int lbmrv_moments(lbmrv_ctx* c, const void* f, void* rho, void* u, void* m0, void* hip_stream) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  const size_t eb = elem_bytes(c->storage);
  const size_t ob = c->storage == LBMRV_F64 ? 8 : 4;
  int rc;
  if ((rc = check_ptr(f, eb)) || (rc = check_ptr(rho, ob)) || (rc = check_ptr(u, ob))) return rc;
  if (m0 && (rc = check_ptr(m0, ob))) return rc;
  if ((rc = check_device(c))) return rc;
  MomLaunch L{};
  L.sk = c->sk;
  L.f = f;
  L.rho = rho;
  L.u = u;
  L.m0 = m0;
  L.N = c->N;
  L.rho0 = c->rho0;
  L.lambda = c->lambda;
  L.rmat = tab_ptr(c, 1);
  L.stream = static_cast<hipStream_t>(hip_stream);
  return kEntries[c->entry].mom[c->sk](L) == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
}

// Runs a partial-sum kernel over the context's reduction buffer (allocated on
// the first call, on the current device), sums its kRedBlocks rows in a fixed
// order (the total of slot 0 plus add0, slots 1..d times scale) and copies the
// five totals to the host; blocking on `st`.
extern "C++" template <class Partial>
static int reduce5(lbmrv_ctx* c, Partial partial, double add0, double scale, hipStream_t st, double (&h)[5]) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LBMRV_ERR_HIP;
  if (c->partial && c->partial_dev != dev) return LBMRV_ERR_INVALID_ARG;  // context bound to its first device
  if (!c->partial) {
    if (hipMalloc(&c->partial, sizeof(double) * (kRedBlocks * 5 + 8)) != hipSuccess) {
      c->partial = nullptr;
      return LBMRV_ERR_HIP;
    }
    c->partial_dev = dev;
  }
  if (partial(c->partial) != hipSuccess) return LBMRV_ERR_HIP;
  double* res = c->partial + kRedBlocks * 5;
  hipLaunchKernelGGL(k_conserve_final, dim3(1), dim3(kRedThreads), 0, st, c->partial, res, add0, scale, c->d);
  if (hipGetLastError() != hipSuccess) return LBMRV_ERR_HIP;
  if (hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return LBMRV_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return LBMRV_ERR_HIP;
  return LBMRV_OK;
}

// Sums of the stored values; a deviation storage adds back rho0 * N (the
// weights sum to 1 and sum w_j c_j = 0), and the momentum is in units of v_j.
static double conserve_add0(const lbmrv_ctx* c) { return c->rho0 * (double)c->N; }

int lbmrv_conservation(lbmrv_ctx* c, const void* f, double out[4], void* hip_stream) {
  if (!c || !out) return LBMRV_ERR_INVALID_ARG;
  int rc;
  if ((rc = check_ptr(f, elem_bytes(c->storage)))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double h[5];
  if ((rc = reduce5(c, [&](double* p) { return kEntries[c->entry].cons[c->sk](f, c->N, p, st); }, conserve_add0(c),
                    c->lambda, st, h)))
    return rc;
  for (int i = 0; i < 4; ++i) out[i] = h[i];
  return h[4] > 0 ? LBMRV_ERR_NONFINITE : LBMRV_OK;
}

// Scratch of lbmrv_conservation_noalloc: the kRedBlocks rows of five partial
// sums.  One copy per GPU (each device holds its own instance of this
// variable), resident until the process ends.  In host code `scratch` only
// names the variable: its device address on the current GPU comes from
// hipGetSymbolAddress, taken once per device and kept in scratch_addr.
static __device__ __align__(256) double scratch[kRedBlocks * 5];
constexpr int kMaxDevices = 64;
static double* scratch_addr[kMaxDevices];
static std::mutex scratch_mutex;

static int scratch_for_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBMRV_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return LBMRV_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LBMRV_ERR_HIP;
    scratch_addr[dev] = static_cast<double*>(p);
  }
  *out = scratch_addr[dev];
  return LBMRV_OK;
}

int lbmrv_conservation_noalloc(lbmrv_ctx* c, const void* f, double* out_dev, void* hip_stream) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  int rc;
  if ((rc = check_ptr(f, elem_bytes(c->storage))) || (rc = check_ptr(out_dev, 8))) return rc;
  double* part = nullptr;
  if ((rc = scratch_for_current_device(&part))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // the partial kernel writes every row of the scratch before the final
  // kernel reads it, so nothing needs clearing between calls
  if (kEntries[c->entry].cons[c->sk](f, c->N, part, st) != hipSuccess) return LBMRV_ERR_HIP;
  hipLaunchKernelGGL(k_conserve_final, dim3(1), dim3(kRedThreads), 0, st, part, out_dev, conserve_add0(c), c->lambda,
                     c->d);
  return hipGetLastError() == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
}

// The reference populations in the stored representation; INVALID_ARG if
// one is not finite.
static int dev_ref(const lbmrv_ctx* c, const double* f_ref, DevRef& r) {
  if (!f_ref) return LBMRV_ERR_INVALID_ARG;
  double w[27] = {};
  int32_t cd[81];
  lbmrv_lattice_tables(c->lattice, cd, w);
  for (int j = 0; j < 27; ++j) {
    if (j < c->q && !std::isfinite(f_ref[j])) return LBMRV_ERR_INVALID_ARG;
    r.r[j] = j < c->q ? f_ref[j] - w[j] * c->rho0 : 0.0;
  }
  return LBMRV_OK;
}

int lbmrv_deviation_norm(lbmrv_ctx* c, const void* f, const double* f_ref, double* out, void* hip_stream) {
  if (!c || !out) return LBMRV_ERR_INVALID_ARG;
  int rc;
  DevRef r{};
  if ((rc = check_ptr(f, elem_bytes(c->storage))) || (rc = dev_ref(c, f_ref, r))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double h[5];
  if ((rc = reduce5(c, [&](double* p) { return kEntries[c->entry].dnorm[c->sk](f, c->N, r, p, st); }, 0.0, 1.0,
                    st, h)))
    return rc;
  out[0] = h[0];
  return h[4] > 0 ? LBMRV_ERR_NONFINITE : LBMRV_OK;
}

int lbmrv_deviation_scale(lbmrv_ctx* c, void* f, const double* f_ref, double factor, void* hip_stream) {
  if (!c || !std::isfinite(factor)) return LBMRV_ERR_INVALID_ARG;
  int rc;
  DevRef r{};
  if ((rc = check_ptr(f, elem_bytes(c->storage))) || (rc = dev_ref(c, f_ref, r))) return rc;
  return kEntries[c->entry].dscale[c->sk](f, c->N, r, factor, static_cast<hipStream_t>(hip_stream)) == hipSuccess
             ? LBMRV_OK
             : LBMRV_ERR_HIP;
}

int lbmrv_init_equilibrium(lbmrv_ctx* c, const double* rho, const double* u, const double* noise, double noise_amp,
                           void* f_out, void* hip_stream) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  int rc;
  if ((rc = check_ptr(rho, 8)) || (rc = check_ptr(u, 8)) || (rc = check_ptr(f_out, elem_bytes(c->storage)))) return rc;
  if (noise && (rc = check_ptr(noise, 8))) return rc;
  if (!std::isfinite(noise_amp)) return LBMRV_ERR_INVALID_ARG;
  InitLaunch L{};
  L.rho = rho;
  L.u = u;
  L.noise = noise;
  L.amp = noise_amp;
  L.rho0 = c->rho0;
  L.lambda = c->lambda;
  L.N = c->N;
  L.fout = f_out;
  L.stream = static_cast<hipStream_t>(hip_stream);
  return kEntries[c->entry].init[c->sk](L) == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
}

static int convert(lbmrv_ctx* c, const void* in, void* out, int to_storage, void* hip_stream) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  const size_t eb = elem_bytes(c->storage);
  int rc;
  if ((rc = check_ptr(in, to_storage ? 8 : eb)) || (rc = check_ptr(out, to_storage ? eb : 8))) return rc;
  return kEntries[c->entry].conv[c->sk](in, out, c->rho0, c->N, to_storage, static_cast<hipStream_t>(hip_stream)) ==
                 hipSuccess
             ? LBMRV_OK
             : LBMRV_ERR_HIP;
}

int lbmrv_import(lbmrv_ctx* c, const double* f, void* out, void* hip_stream) { return convert(c, f, out, 1, hip_stream); }
int lbmrv_export(lbmrv_ctx* c, const void* in, double* f, void* hip_stream) { return convert(c, in, f, 0, hip_stream); }

int lbmrv_lattice_tables(int lattice, int32_t* cdirs, double* w) {
  if (lattice != LBMRV_D2Q9 && lattice != LBMRV_D3Q19 && lattice != LBMRV_D3Q27) return LBMRV_ERR_INVALID_ARG;
  if (!cdirs || !w) return LBMRV_ERR_INVALID_ARG;
  auto fill = [&](auto lat) {
    using L = decltype(lat);
    for (int j = 0; j < L::Q; ++j) {
      cdirs[3 * j] = L::c[j].x;
      cdirs[3 * j + 1] = L::c[j].y;
      cdirs[3 * j + 2] = L::c[j].z;
      w[j] = L::w(j).val();
    }
  };
  if (lattice == LBMRV_D2Q9) fill(D2Q9Lat{});
  else if (lattice == LBMRV_D3Q19) fill(D3Q19Lat{});
  else fill(D3Q27Lat{});
  return LBMRV_OK;
}

}  // extern "C"

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Grids up to this many nodes reverse two steps per launch (k_adjoint2) where
// the lattice has that kernel: small grids are bound by each launch's latency
// and fixed cost.  Measured (D2Q9 FP32, u~ a field, K = 100), two steps per
// launch against one: 512^2 -16 %, 724^2 -9 %, 1024^2 -5 %, 1448^2 -1.3 %,
// 2048^2 +4.6 % (there HBM bounds both, and the single-step kernel runs more
// wavefronts per SIMD).
constexpr uint64_t kAdj2MaxNodes = 1ull << 21;

struct AdjPlan {
  int64_t nseg, nsnap, nsegslots, nsets;
  size_t state_bytes, lam_bytes, partial_bytes, total;
  uint64_t nblocks;
};

// Workspace: nsnap snapshots (states K, 2K, ...), nsets sets of nsegslots
// segment states (segment sg uses set sg mod nsets; with three sets a segment
// can be recomputed two segments ahead of the reverse sweep), two ping-pong
// states for the forward sweep, one state for f_N when the caller passes none,
// two adjoint states and the rows of dJ/ds partial sums.
AdjPlan adj_plan(const lbmrv_ctx* c, int64_t nsteps, int64_t K) {
  AdjPlan p{};
  p.nseg = (nsteps + K - 1) / K;
  p.nsnap = p.nseg - 1;
  p.nsegslots = (nsteps < K ? nsteps : K) - 1;
  p.nsets = p.nseg < 3 ? p.nseg : 3;
  p.state_bytes = align256(elem_bytes(c->storage) * c->q * c->N);
  p.lam_bytes = align256((c->storage == LBMRV_F64 ? 8 : 4) * (size_t)c->q * c->N);
  const uint64_t gx = (c->nx + c->block - 1) / c->block;
  p.nblocks = gx * c->ny * c->nz;
  if (has_adjoint2(c->d, c->sk)) {  // rows of the two-step kernel's tiles
    const uint64_t n2 = (uint64_t)((c->nx + kA2X - 1) / kA2X) * ((c->ny + kA2Y - 1) / kA2Y);
    if (n2 > p.nblocks) p.nblocks = n2;
  }
  p.partial_bytes = align256(sizeof(double) * p.nblocks * c->q);
  p.total = p.state_bytes * (size_t)(p.nsnap + p.nsets * p.nsegslots + 3) + 2 * p.lam_bytes + p.partial_bytes;
  return p;
}

hipError_t fill_zero(double* p, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace

extern "C" {

size_t lbmrv_adjoint_workspace_bytes(const lbmrv_ctx* c, int64_t nsteps, int64_t K) {
  if (!c || nsteps < 1 || K < 1) return 0;
  return adj_plan(c, nsteps, K).total;
}

int lbmrv_adjoint(lbmrv_ctx* c, const void* f0, int ut_mode, double ut_alpha, const float* ut_field, int64_t nsteps,
                  int64_t K, const void* cot_fN, void* workspace, size_t workspace_bytes, void* f_N, void* grad_f0,
                  double* grad_s, double* grad_ut, void* hip_stream) {
  if (!c) return LBMRV_ERR_INVALID_ARG;
  if (ut_mode != LBMRV_UT_ZERO && ut_mode != LBMRV_UT_FLUID && ut_mode != LBMRV_UT_FIELD) return LBMRV_ERR_INVALID_ARG;
  if (!std::isfinite(ut_alpha)) return LBMRV_ERR_INVALID_ARG;
  if (nsteps < 1 || K < 1) return LBMRV_ERR_INVALID_ARG;
  if (c->wall_mask) return LBMRV_ERR_UNSUPPORTED;  // the adjoint covers periodic domains
  const size_t eb = elem_bytes(c->storage);
  const size_t tb = c->storage == LBMRV_F64 ? 8 : 4;
  int rc;
  if ((rc = check_ptr(f0, eb)) || (rc = check_ptr(cot_fN, tb)) || (rc = check_ptr(workspace, 256)) ||
      (rc = check_ptr(grad_f0, tb)) || (rc = check_ptr(grad_s, 8)))
    return rc;
  if (f_N && (rc = check_ptr(f_N, eb))) return rc;
  if (ut_mode == LBMRV_UT_FIELD && ((rc = check_ptr(ut_field, 4)) || (rc = check_ptr(grad_ut, 8)))) return rc;
  if ((rc = check_device(c))) return rc;
  const AdjPlan P = adj_plan(c, nsteps, K);
  if (workspace_bytes < P.total) return LBMRV_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);

  // Segments other than the last are recomputed from their first state on a
  // second stream, ahead of the reverse sweep on the caller's stream, so that
  // the two sweeps overlap on the GPU (needed only when there are several
  // segments with states inside them).
  const bool recompute_any = P.nseg > 1 && P.nsegslots > 0;
  const int64_t S = P.nsets;
  if (recompute_any) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LBMRV_ERR_HIP;
    if (c->astream && c->astream_dev != dev) return LBMRV_ERR_INVALID_ARG;  // bound to its first device
    if (!c->astream) {
      // all or nothing: a failure leaves no stream or event behind, so the
      // next call starts over
      bool ok = hipStreamCreateWithFlags(&c->astream, hipStreamNonBlocking) == hipSuccess;
      if (!ok) c->astream = nullptr;
      for (auto& ev : c->aev)
        if (ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
          ev = nullptr;
          ok = false;
        }
      if (!ok) {
        if (c->astream) (void)hipStreamDestroy(c->astream);
        c->astream = nullptr;
        for (auto& ev : c->aev) {
          if (ev) (void)hipEventDestroy(ev);
          ev = nullptr;
        }
        return LBMRV_ERR_HIP;
      }
      c->astream_dev = dev;
    }
  }
  hipStream_t st2 = c->astream;
  // aev[0]: a snapshot written; aev[1 + r mod 3]: segment r recomputed (on
  // st2); aev[4 + sg mod 3]: segment sg reversed (on st)
  hipEvent_t ev_snap = c->aev[0];
  auto ev_rec = [&](int64_t r) { return c->aev[1 + r % 3]; };
  auto ev_rev = [&](int64_t sg) { return c->aev[4 + sg % 3]; };

  char* w = static_cast<char*>(workspace);
  char* snaps = w;
  char* segs = snaps + P.state_bytes * P.nsnap;
  char* pingpong = segs + P.state_bytes * P.nsegslots * S;
  char* fscratch = pingpong + 2 * P.state_bytes;
  char* lam0 = fscratch + P.state_bytes;
  char* lam1 = lam0 + P.lam_bytes;
  double* partial = reinterpret_cast<double*>(lam1 + P.lam_bytes);
  void* fN = f_N ? f_N : fscratch;
  const int64_t last = P.nseg - 1;
  // state t as the reverse sweep reads it (and the recompute writes it)
  auto state = [&](int64_t t) -> void* {
    if (t == 0) return const_cast<void*>(f0);
    if (t == nsteps) return fN;
    if (t % K == 0) return snaps + P.state_bytes * (t / K - 1);
    return segs + P.state_bytes * (P.nsegslots * ((t / K) % S) + (t % K - 1));
  };
  // state t in the forward sweep: states inside earlier segments are not kept,
  // they alternate between two buffers that stay in the last-level cache
  auto fwd_state = [&](int64_t t) -> void* {
    if (t == 0 || t == nsteps || t % K == 0 || t / K == last) return state(t);
    return pingpong + P.state_bytes * (t % 2);
  };
  const Entry& E = kEntries[c->entry];
  hipError_t e;
  // Recompute the states inside segment r from its first state on st2, into
  // set r mod S.  The set's previous user, segment r + S, must have been
  // reversed first; ev_rev(r + S) is recorded before this is issued.
  auto issue_recompute = [&](int64_t r) -> hipError_t {
    hipError_t er;
    if (r + S <= last && (er = hipStreamWaitEvent(st2, ev_rev(r + S), 0)) != hipSuccess) return er;
    const int64_t t0 = r * K, t1 = (t0 + K < nsteps) ? t0 + K : nsteps;
    for (int64_t t = t0; t + 1 < t1; ++t)
      if ((er = run_kind(c, K_PUSH, state(t), state(t + 1), ut_mode, ut_alpha, ut_field, st2)) != hipSuccess)
        return er;
    return hipEventRecord(ev_rec(r), st2);
  };
  // forward sweep (scatter form, pre-collision states), keeping every K-th
  // state and the states of the last segment.  The S - 1 segments before the
  // last (whose sets the forward sweep does not touch) are recomputed on st2
  // as soon as their first state is written, alongside the rest of the sweep.
  for (int64_t t = 0; t < nsteps; ++t) {
    e = run_kind(c, K_PUSH, fwd_state(t), fwd_state(t + 1), ut_mode, ut_alpha, ut_field, st);
    if (e != hipSuccess) return LBMRV_ERR_HIP;
    const int64_t r = (t + 1) / K;
    if (recompute_any && (t + 1) % K == 0 && r < last && r >= last - (S - 1)) {
      if (hipEventRecord(ev_snap, st) != hipSuccess || hipStreamWaitEvent(st2, ev_snap, 0) != hipSuccess ||
          issue_recompute(r) != hipSuccess)
        return LBMRV_ERR_HIP;
    }
  }
  if (recompute_any && last - (S - 1) <= 0 && last >= 1) {
    // segment 0 among them: its first state is f0, present from the start
    if (issue_recompute(0) != hipSuccess) return LBMRV_ERR_HIP;
  }
  if ((e = fill_zero(partial, P.nblocks * c->q, st)) != hipSuccess) return LBMRV_ERR_HIP;
  if (ut_mode == LBMRV_UT_FIELD && (e = fill_zero(grad_ut, (uint64_t)c->d * c->N, st)) != hipSuccess)
    return LBMRV_ERR_HIP;
  AdjLaunch A{};
  A.mode = ut_mode;
  A.ut = ut_field;
  A.grad_ut = ut_mode == LBMRV_UT_FIELD ? grad_ut : nullptr;
  A.partial = partial;
  A.nx = c->nx;
  A.ny = c->ny;
  A.nz = c->nz;
  A.N = c->N;
  A.rho0 = c->rho0;
  A.inv_lambda = 1.0 / c->lambda;
  A.alpha = ut_alpha;
  for (int k = 0; k < 27; ++k) A.s[k] = k < c->q ? c->s[k] : 0.0;
  A.rnn = tab_ptr(c, 2);
  A.rnninv = tab_ptr(c, 3);
  A.xcd_remap = xcd_order(c);
  A.eq_maxwell = c->equilibrium == LBMRV_EQ_MAXWELLIAN ? 1u : 0u;
  A.stream = st;
  A.block = c->block;
  const bool two_step = has_adjoint2(c->d, c->sk) && c->N <= kAdj2MaxNodes;
  const void* lam_cur = cot_fN;
  // Reverse sweep, one segment of K steps at a time, last segment first (its
  // states are in place from the forward sweep).  Segment sg waits for its
  // recompute; once it is reversed its set is free, and segment sg - S is
  // recomputed into it on st2, S - 1 segments ahead of the reverse sweep.
  for (int64_t sg = last; sg >= 0; --sg) {
    if (recompute_any && sg < last && hipStreamWaitEvent(st, ev_rec(sg), 0) != hipSuccess) return LBMRV_ERR_HIP;
    const int64_t t0 = sg * K;
    const int64_t t1 = (t0 + K < nsteps) ? t0 + K : nsteps;
    // two steps per launch where the lattice has that kernel, the last step
    // of an odd count alone; the adjoint alternates between lam0 and lam1
    // (never written by the launch that reads it), the first step reads the
    // cotangent and the last one writes dJ/df0
    for (int64_t t = t1 - 1; t >= t0;) {
      const bool pair = two_step && t - 1 >= t0;
      const int64_t tl = pair ? t - 1 : t;  // the launch's last step
      A.f = state(t);
      A.f_prev = pair ? state(t - 1) : nullptr;
      A.lam_in = lam_cur;
      A.lam_out = tl == 0 ? static_cast<void*>(grad_f0) : (lam_cur == lam0 ? lam1 : lam0);
      if ((e = (pair ? E.adj2 : E.adj)[c->sk](A)) != hipSuccess) return LBMRV_ERR_HIP;
      lam_cur = A.lam_out;
      t = tl - 1;
    }
    if (recompute_any && sg - S >= 0) {
      if (hipEventRecord(ev_rev(sg), st) != hipSuccess || issue_recompute(sg - S) != hipSuccess)
        return LBMRV_ERR_HIP;
    }
  }
  hipLaunchKernelGGL(k_reduce_columns, dim3(1), dim3(kRedCols, kRedRows), 0, st, partial, P.nblocks, c->q, c->d, grad_s);
  return hipGetLastError() == hipSuccess ? LBMRV_OK : LBMRV_ERR_HIP;
}

void lbmrv_destroy(lbmrv_ctx* c) {
  if (!c) return;
  if (c->astream) (void)hipStreamDestroy(c->astream);
  for (auto& ev : c->aev)
    if (ev) (void)hipEventDestroy(ev);
  if (c->partial) (void)hipFree(c->partial);
  if (c->dtab) (void)hipFree(c->dtab);
  delete c;
}

const char* lbmrv_strerror(int code) {
  switch (code) {
    case LBMRV_OK: return "ok";
    case LBMRV_ERR_INVALID_ARG: return "invalid argument";
    case LBMRV_ERR_UNSUPPORTED: return "unsupported request";
    case LBMRV_ERR_HIP: return "HIP runtime error";
    case LBMRV_ERR_NONFINITE: return "non-finite population found";
    case LBMRV_ERR_ALIGNMENT: return "pointer not aligned to its element size";
  }
  return "unknown error code";
}

}  // extern "C"
