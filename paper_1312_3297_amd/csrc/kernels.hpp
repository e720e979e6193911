// HIP kernels of the relative-velocity lattice Boltzmann step (gfx950).
//
// One thread owns one lattice node per pass.  The per-node algebra (moments,
// shift into the moving frame, diagonal relaxation, shift back, inversion) is
// unrolled at compile time over the exact tables of tables.hpp and lives in
// registers; it is a handful of sparse q-vectors per node, not a contraction,
// so no matrix cores are involved.  Populations are SoA: f[j][z][y][x] with x
// fastest, so each population access of a wavefront is one contiguous run.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "tables.hpp"

namespace lbmrv {

// ------------------------------------------------------------------ helpers
template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// static_for: calls f(integral_constant<int, i>) for i = 0 .. N-1
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

template <class T>
__device__ __forceinline__ T fmac(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// y += C * x for a compile-time rational C (folds +-1 to add / sub)
template <Rat C, class T>
__device__ __forceinline__ void axpy_c(T& y, T x) {
  constexpr T cv = T(C.val());
  if constexpr (C == Rat(1)) y += x;
  else if constexpr (C == Rat(-1)) y -= x;
  else y = fmac(cv, x, y);
}

// Starting value of a sum: -0 is the additive identity for every x
// (x + -0 = x, -0 - x = -x, fma(a, b, -0) = a b), so the compiler drops the
// first add of each sum and the terms of moments known to vanish; +0 is not
// (-0 + +0 = +0), and would cost one add per sum.
template <class T>
__device__ __forceinline__ constexpr T zsum() {
  return T(-0.0);
}

template <Rat C, class T>
__device__ __forceinline__ constexpr T lit() {
  return T(C.val());
}

// storage element types
template <int ST>
struct Store;
template <>
struct Store<0> { using S = double; using T = double; };   // FP64
template <>
struct Store<1> { using S = float; using T = float; };     // FP32 (also FP32 deviations)
template <>
struct Store<2> { using S = _Float16; using T = float; };  // FP16 deviations, FP32 arithmetic

enum Mode { UT_ZERO = 0, UT_FLUID = 1, UT_FIELD = 2 };
// K_PULL    gather f*_j(x - c_j), collide, store at x        (post-collision kept)
// K_PUSH    load at x, collide, scatter to x + c_j           (pre-collision kept)
// K_COLLIDE load at x, collide, store at x
// K_STREAM  gather f_j(x - c_j), store at x (no collision)
// K_AA_EVEN load slot j at x, collide, store slot opp(j) at x         (in place)
// K_AA_ODD  load slot opp(j) at x - c_j, collide, store slot j at x + c_j (in place)
// K_AA_ODD_WALLS  the same with half-way bounce-back walls on paired faces
enum Kind { K_PULL = 0, K_PUSH = 1, K_COLLIDE = 2, K_STREAM = 3, K_AA_EVEN = 4, K_AA_ODD = 5, K_AA_ODD_WALLS = 6 };

template <class T>
struct StepArgs {
  const void* fin;
  void* fout;
  const float* ut;  // [d][N] relative-velocity field (physical units) or null
  uint32_t nx, ny, nz;
  uint64_t N;       // nodes
  T rho0;           // reference density subtracted in deviation storage (0 otherwise)
  T alpha;          // FLUID mode: u~ = alpha u
  T inv_lambda;     // FIELD mode: u~ is given in physical units
  T s[27];          // relaxation rates of the user basis
  uint32_t wall_mask;  // bit 2a+side: the low (0) / high (1) face of axis a is a wall
  T wall_coef[6][3];   // 6 rho_w u_w / lambda per wall face (half-way bounce-back)
  uint32_t eq_maxwell; // 1: equilibrium moments of the continuous Maxwellian
  const T* relax;      // run-time basis only: the non-conserved block of R^{-1} S R,
                       // (Q-D-1)^2 row-major, in the working basis
  uint32_t xcd_remap;  // 1: contiguous tile ranges per XCD (block_tile)
};

// ------------------------------------------------------------------ cube form
// When the velocities lie in {0, +1, -1}^3 and the working basis is a set of
// monomials X^a Y^b Z^e with a, b, e <= 2, M_W(0) is a restriction of the
// 27 x 27 tensor product of one 3 x 3 matrix per axis (rows 1, X, X^2 on the
// velocities 0, +1, -1), and both M_W(0) and its inverse apply as three
// one-axis passes over a 3 x 3 x 3 cube of cells.  Cells that hold no value
// (velocities the lattice lacks, monomials the basis lacks, the conserved
// moments, which vanish in the collision's moment change) are known at compile
// time and cost nothing.  The inverse is exact for a lattice smaller than the
// cube when every monomial missing from the basis vanishes on all of its
// velocities (D3Q19: the monomials with all three exponents >= 1): the cube
// moments of a population vector on such a lattice are its basis moments plus
// zeros, so the cube inverse of (moments, zeros) is that vector padded with
// zeros.
template <class B>
struct CubeForm {
  using L = typename B::Lat;
  static constexpr int Q = B::Q;
  struct Mask {
    bool m[27] = {};
  };
  static constexpr int node(int c) { return c == 0 ? 0 : (c > 0 ? 1 : 2); }
  static constexpr int cell(int a, int b, int e) { return (a * 3 + b) * 3 + e; }
  static constexpr int pop_cell(int j) { return cell(node(L::c[j].x), node(L::c[j].y), node(L::c[j].z)); }
  static constexpr int mom_cell(int k) {
    const Poly p = B::W(k);
    return cell(p.t[0].a, p.t[0].b, p.t[0].e);
  }
  static constexpr int ipow(int c, int n) { return n == 0 ? 1 : c * ipow(c, n - 1); }
  static constexpr bool applies() {
    for (int j = 0; j < Q; ++j) {
      const int c[3] = {L::c[j].x, L::c[j].y, L::c[j].z};
      for (int ax = 0; ax < 3; ++ax)
        if (c[ax] < -1 || c[ax] > 1) return false;
    }
    bool used[27] = {};
    for (int k = 0; k < Q; ++k) {
      const Poly p = B::W(k);
      if (p.n != 1 || !(p.t[0].c == Rat(1)) || p.t[0].a > 2 || p.t[0].b > 2 || p.t[0].e > 2) return false;
      if (used[mom_cell(k)]) return false;
      used[mom_cell(k)] = true;
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int e = 0; e < 3; ++e)
          if (!used[cell(a, b, e)])
            for (int j = 0; j < Q; ++j)
              if (ipow(L::c[j].x, a) * ipow(L::c[j].y, b) * ipow(L::c[j].z, e) != 0) return false;
    return true;
  }
  static constexpr int stride(int ax) { return ax == 0 ? 9 : (ax == 1 ? 3 : 1); }
  // first cell of line i (0..8) along axis ax
  static constexpr int line(int ax, int i) {
    const int u = i / 3, v = i % 3;
    return ax == 0 ? cell(0, u, v) : (ax == 1 ? cell(u, 0, v) : cell(u, v, 0));
  }
  // Which cells hold a value (all others are known zeros) before pass `stage`
  // (passes along x, y, z) of one of the four maps, by the rule each map's
  // one-axis step follows on a line of cells (p0, p+, p-) or (m0, m1, m2):
  //   kFwd  M_W(0):        (a|p|n, p|n, p|n)   from the populations
  //   kInv  its inverse:   (a|n,   p|n, p|n)   from the non-conserved moments
  //   kFwdT M_W(0)^T:      (a, a|p|n, a|p|n)   from the non-conserved moments
  //   kInvT its inverse^T: (a, p|n,   a|p|n)   from the populations
  enum { kFwd = 0, kInv = 1, kFwdT = 2, kInvT = 3 };
  static constexpr Mask mask(int map, int stage) {
    Mask m;
    if (map == kFwd || map == kInvT) {
      for (int j = 0; j < Q; ++j) m.m[pop_cell(j)] = true;
    } else {
      for (int k = L::D + 1; k < Q; ++k) m.m[mom_cell(k)] = true;
    }
    for (int ax = 0; ax < stage; ++ax)
      for (int i = 0; i < 9; ++i) {
        const int i0 = line(ax, i), i1 = i0 + stride(ax), i2 = i0 + 2 * stride(ax);
        const bool A = m.m[i0], P = m.m[i1], N = m.m[i2];
        const bool any = A || P || N;
        if (map == kFwd) {
          m.m[i0] = any;
          m.m[i1] = m.m[i2] = P || N;
        } else if (map == kInv) {
          m.m[i0] = A || N;
          m.m[i1] = m.m[i2] = P || N;
        } else if (map == kFwdT) {
          m.m[i1] = m.m[i2] = any;
        } else {
          m.m[i1] = P || N;
          m.m[i2] = any;
        }
      }
    return m;
  }
};

// m_k = sum_j W_k(c_j) h_j for every basis monomial (the conserved ones too).
// One axis: (p0, p+, p-) -> (p0 + p+ + p-, p+ - p-, p+ + p-).
template <class B, class T>
__device__ __forceinline__ void cube_moments(const T (&h)[B::Q], T (&m)[B::Q]) {
  using C = CubeForm<B>;
  T c[27];
  sfor<B::Q>([&](auto jj) { c[C::pop_cell(jj)] = h[jj]; });
  sfor<3>([&](auto ax) {
    constexpr int AX = ax;
    constexpr typename C::Mask M = C::mask(C::kFwd, AX);
    sfor<9>([&](auto ii) {
      constexpr int i0 = C::line(AX, ii), i1 = i0 + C::stride(AX), i2 = i0 + 2 * C::stride(AX);
      constexpr bool A = M.m[i0], P = M.m[i1], N = M.m[i2];
      if constexpr (P && N) {
        const T sum = c[i1] + c[i2], dif = c[i1] - c[i2];
        if constexpr (A) c[i0] = c[i0] + sum;
        else c[i0] = sum;
        c[i1] = dif;
        c[i2] = sum;
      } else if constexpr (P) {
        if constexpr (A) c[i0] = c[i0] + c[i1];
        else c[i0] = c[i1];
        c[i2] = c[i1];
      } else if constexpr (N) {
        if constexpr (A) c[i0] = c[i0] + c[i2];
        else c[i0] = c[i2];
        c[i1] = -c[i2];
      }
    });
  });
  constexpr typename C::Mask F = C::mask(C::kFwd, 3);
  sfor<B::Q>([&](auto kk) {
    // a basis monomial whose cell stayed empty would vanish on every velocity
    // (and M_W(0) would be singular)
    static_assert(F.m[C::mom_cell(kk)]);
    m[kk] = c[C::mom_cell(kk)];
  });
}

// dh_j = 2^{|c_j|^2} (M_W(0)^{-1} dm)_j for a moment change dm that vanishes on
// the conserved moments.  One axis of the inverse is
// (m0, m1, m2) -> (m0 - m2, (m1 + m2)/2, (m2 - m1)/2); the halves belong to
// the population index, so the passes leave them out and the caller applies
// 2^{-|c_j|^2} once per population.
template <class B, class T>
__device__ __forceinline__ void cube_populations(const T (&dm)[B::Q], T (&dh)[B::Q]) {
  using C = CubeForm<B>;
  constexpr int D = B::Lat::D;
  T c[27];
  sfor<B::Q>([&](auto kk) {
    if constexpr (kk > D) c[C::mom_cell(kk)] = dm[kk];
  });
  sfor<3>([&](auto ax) {
    constexpr int AX = ax;
    constexpr typename C::Mask M = C::mask(C::kInv, AX);
    sfor<9>([&](auto ii) {
      constexpr int i0 = C::line(AX, ii), i1 = i0 + C::stride(AX), i2 = i0 + 2 * C::stride(AX);
      constexpr bool A = M.m[i0], P = M.m[i1], N = M.m[i2];
      if constexpr (N) {
        const T q0 = c[i0], q1 = c[i1], q2 = c[i2];
        if constexpr (A) c[i0] = q0 - q2;
        else c[i0] = -q2;
        if constexpr (P) {
          c[i1] = q1 + q2;
          c[i2] = q2 - q1;
        } else {
          c[i1] = q2;
          c[i2] = q2;
        }
      } else if constexpr (P) {
        c[i2] = -c[i1];
      }
    });
  });
  constexpr typename C::Mask F = C::mask(C::kInv, 3);
  sfor<B::Q>([&](auto jj) {
    if constexpr (F.m[C::pop_cell(jj)]) dh[jj] = c[C::pop_cell(jj)];
    else dh[jj] = zsum<T>();
  });
}

// Transposes, for the adjoint.  M_W(0)^T z (moments -> populations), for z
// that vanishes on the conserved moments; one axis is
// (z0, z1, z2) -> (z0, z0 + z1 + z2, z0 - z1 + z2).  Exact for a lattice
// smaller than the cube: the basis moments it lacks enter as zeros.
template <class B, class T>
__device__ __forceinline__ void cube_moments_t(const T (&z)[B::Q], T (&y)[B::Q]) {
  using C = CubeForm<B>;
  constexpr int D = B::Lat::D;
  T c[27];
  sfor<B::Q>([&](auto kk) {
    if constexpr (kk > D) c[C::mom_cell(kk)] = z[kk];
  });
  sfor<3>([&](auto ax) {
    constexpr int AX = ax;
    constexpr typename C::Mask M = C::mask(C::kFwdT, AX);
    sfor<9>([&](auto ii) {
      constexpr int i0 = C::line(AX, ii), i1 = i0 + C::stride(AX), i2 = i0 + 2 * C::stride(AX);
      constexpr bool A = M.m[i0], P = M.m[i1], N = M.m[i2];
      if constexpr (A || P || N) {
        T sum;  // z0 + z2
        if constexpr (A && N) sum = c[i0] + c[i2];
        else if constexpr (A) sum = c[i0];
        else if constexpr (N) sum = c[i2];
        if constexpr ((A || N) && P) {
          c[i2] = sum - c[i1];
          c[i1] = sum + c[i1];
        } else if constexpr (A || N) {
          c[i1] = sum;
          c[i2] = sum;
        } else {
          c[i2] = -c[i1];
        }
      }
    });
  });
  constexpr typename C::Mask F = C::mask(C::kFwdT, 3);
  sfor<B::Q>([&](auto jj) {
    if constexpr (F.m[C::pop_cell(jj)]) y[jj] = c[C::pop_cell(jj)];
    else y[jj] = zsum<T>();
  });
}

// M_W(0)^{-T} g on the non-conserved moments (populations -> moments): the
// populations are first scaled by 2^{-|c_j|^2} (the inverse's halves), then
// one axis is (p0, p+, p-) -> (p0, p+ - p-, p+ + p- - p0).  The conserved
// entries (k <= d) are set to -0.
template <class B, class T>
__device__ __forceinline__ void cube_populations_t(const T (&g)[B::Q], T (&zm)[B::Q]) {
  using C = CubeForm<B>;
  using L = typename B::Lat;
  constexpr int D = L::D;
  T c[27];
  sfor<B::Q>([&](auto jj) {
    constexpr int J = jj;
    constexpr int c2 = L::c[J].x * L::c[J].x + L::c[J].y * L::c[J].y + L::c[J].z * L::c[J].z;
    if constexpr (c2 == 0) c[C::pop_cell(J)] = g[J];
    else c[C::pop_cell(J)] = T(1.0 / (1 << c2)) * g[J];
  });
  sfor<3>([&](auto ax) {
    constexpr int AX = ax;
    constexpr typename C::Mask M = C::mask(C::kInvT, AX);
    sfor<9>([&](auto ii) {
      constexpr int i0 = C::line(AX, ii), i1 = i0 + C::stride(AX), i2 = i0 + 2 * C::stride(AX);
      constexpr bool A = M.m[i0], P = M.m[i1], N = M.m[i2];
      if constexpr (P || N) {
        T sum, dif;
        if constexpr (P && N) {
          sum = c[i1] + c[i2];
          dif = c[i1] - c[i2];
        } else if constexpr (P) {
          sum = c[i1];
          dif = c[i1];
        } else {
          sum = c[i2];
          dif = -c[i2];
        }
        c[i1] = dif;
        if constexpr (A) c[i2] = sum - c[i0];
        else c[i2] = sum;
      } else if constexpr (A) {
        c[i2] = -c[i0];
      }
    });
  });
  constexpr typename C::Mask F = C::mask(C::kInvT, 3);
  sfor<B::Q>([&](auto kk) {
    constexpr int K = kk;
    if constexpr (K <= D || !F.m[C::mom_cell(K)]) zm[K] = zsum<T>();
    else zm[K] = c[C::mom_cell(K)];
  });
}

// ------------------------------------------------------------------ collision
// In-register collision at one node.  h holds the populations minus w_j rho0.
// After return h holds the post-collision values (same offset).
// RLX = 0: rates act on the built-in user basis (sparse compile-time R);
// RLX = 1: on a run-time basis P = R W of the same span, through the dense
// matrix a.relax = R^{-1} S R (non-conserved block).
template <class B, class T, int MODE, int RLX>
__device__ __forceinline__ void collide_node(T (&h)[B::Q], const StepArgs<T>& a, const T (&utf)[3]) {
  // Products are fused into sums only where the source says so (fmac) or
  // within one expression, never across statements: the pull, push and
  // in-place kernels inline this body into different code, and must round it
  // identically.
#pragma clang fp contract(on)
  using L = typename B::Lat;
  constexpr int Q = B::Q;
  constexpr int D = L::D;
  using Tb = Tab<B>;

  // monomial bases on {0, +-1}^d velocities: all working-basis moments of h
  // in three one-axis passes.  FP32 arithmetic only: with 8-byte values the
  // cube's live cells raise the register count (D3Q19: 96 -> 132 VGPRs, two
  // wavefronts per SIMD fewer), and the sparse rows measured 2.9 % faster.
  constexpr bool cube = CubeForm<B>::applies() && sizeof(T) == 4;
  T mw[cube ? Q : 1];
  if constexpr (cube) cube_moments<B>(h, mw);

  // conserved moments, eq. (rhoq): rho = rho0 + sum h, j = sum c h
  T drho, jm[3] = {zsum<T>(), zsum<T>(), zsum<T>()};
  if constexpr (cube) {
    drho = mw[0];
    sfor<3>([&](auto al) { jm[al] = mw[1 + al]; });
  } else {
    drho = h[0];
    sfor<Q - 1>([&](auto jj) { drho += h[jj + 1]; });
    sfor<Q>([&](auto jj) {
      constexpr int J = jj;
      if constexpr (L::c[J].x > 0) jm[0] += h[J];
      if constexpr (L::c[J].x < 0) jm[0] -= h[J];
      if constexpr (L::c[J].y > 0) jm[1] += h[J];
      if constexpr (L::c[J].y < 0) jm[1] -= h[J];
      if constexpr (L::c[J].z > 0) jm[2] += h[J];
      if constexpr (L::c[J].z < 0) jm[2] -= h[J];
    });
  }
  const T rho = a.rho0 + drho;
  const T irho = T(1) / rho;
  T u[3] = {jm[0] * irho, jm[1] * irho, D == 3 ? jm[2] * irho : T(0)};

  // relative velocity
  T ut[3] = {T(0), T(0), T(0)};
  if constexpr (MODE == UT_FLUID) {
    sfor<D>([&](auto al) { ut[al] = a.alpha * u[al]; });
  } else if constexpr (MODE == UT_FIELD) {
    sfor<D>([&](auto al) { ut[al] = utf[al]; });
  }

  // fixed-frame non-equilibrium moments in the working basis, dl = m^eq - m
  // (k > d only; the conserved entries are exactly zero because f^eq has the
  // same rho, j).  One uniform branch picks the equilibrium for all moments,
  // so neither form is evaluated and then discarded; each branch subtracts m
  // itself, so that every kernel rounds the difference the same way.
  T dl[Q];
  // m_K of the populations (k > d)
  T mh[Q];
  sfor<Q>([&](auto kk) {
    constexpr int K = kk;
    if constexpr (K <= D) {
      dl[K] = zsum<T>();
    } else if constexpr (cube) {
      mh[K] = mw[K];
    } else {
      mh[K] = zsum<T>();
      sfor<Tb::t.sMW[K].n>([&](auto i) {
        axpy_c<Tb::t.sMW[K].val[i]>(mh[K], h[Tb::t.sMW[K].col[i]]);
      });
    }
  });
  if (a.eq_maxwell != 0) {
    // Maxwellian option: per-axis moments E[xi^n] of N(u_a, cs2), cs2 = 1/3
    // in lattice units, n = 0..4; m^eq_K - rho0 a_K = rho E[W_K(xi)] - rho0 a_K
    // from the monomial terms of W_K
    T mu[3][kP];
    constexpr T cs2 = T(1) / T(3);
    sfor<3>([&](auto ax) {
      const T v = ax < D ? u[ax] : T(0);
      const T v2 = v * v;
      mu[ax][0] = T(1);
      mu[ax][1] = v;
      mu[ax][2] = v2 + cs2;
      mu[ax][3] = v * (v2 + T(3) * cs2);
      mu[ax][4] = v2 * (v2 + T(6) * cs2) + T(3) * cs2 * cs2;
    });
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      if constexpr (K > D) {
        constexpr Poly pk = B::W(K);
        T mk = zsum<T>();
        sfor<pk.n>([&](auto ti) {
          constexpr PTerm tm = pk.t[ti];
          mk = fmac(lit<tm.c, T>(), mu[0][tm.a] * mu[1][tm.b] * mu[2][tm.e], mk);
        });
        constexpr Rat ak = Tb::t.a[K];
        dl[K] = fmac(rho, mk, -(lit<ak, T>() * a.rho0)) - mh[K];
      }
    });
  } else {
    // second-order polynomial equilibrium: rho (b.u + u.C.u) + a drho
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      if constexpr (K > D) {
        T quad = zsum<T>();
        sfor<D>([&](auto al) {
          constexpr Rat bb = Tb::t.b[K][al];
          if constexpr (!bb.zero()) quad = fmac(lit<bb, T>(), u[al], quad);
          sfor<D>([&](auto be) {
            if constexpr (be >= al) {
              constexpr Rat cc = (be == al) ? Tb::t.C[K][al][be] : Tb::t.C[K][al][be] + Tb::t.C[K][be][al];
              if constexpr (!cc.zero()) quad = fmac(lit<cc, T>() * u[al], u[be], quad);
            }
          });
        });
        T eq = rho * quad;
        constexpr Rat ak = Tb::t.a[K];
        if constexpr (!ak.zero()) eq = fmac(lit<ak, T>(), drho, eq);
        dl[K] = eq - mh[K];
      }
    });
  }
  // shift into the frame moving at u~:  dl <- prod_a exp(-u~_a D_a) dl
  auto shift = [&](T sign) {
    sfor<D>([&](auto ax) {
      constexpr int AX = ax;
      constexpr int NM = Tb::t.nmax[AX];
      T pw[kP];
      pw[1] = sign * ut[AX];
      sfor<NM>([&](auto nn) {
        if constexpr (nn + 1 >= 2) pw[nn + 1] = pw[nn] * pw[1];
      });
      T out[Q];
      sfor<Q>([&](auto kk) {
        constexpr int K = kk;
        out[K] = dl[K];
        if constexpr (K > D) {
          sfor<NM>([&](auto nn) {
            constexpr int N = nn + 1;
            constexpr int NZ = Tb::t.sE[AX][N][K].n;
            if constexpr (NZ == 1) {
              // one term: the constant goes into the power, which the
              // compiler then shares between all rows with that constant
              constexpr Rat cv = Tb::t.sE[AX][N][K].val[0];
              out[K] = fmac(lit<cv, T>() * pw[N], dl[Tb::t.sE[AX][N][K].col[0]], out[K]);
            } else if constexpr (NZ > 1) {
              T acc = zsum<T>();
              sfor<NZ>([&](auto i) {
                axpy_c<Tb::t.sE[AX][N][K].val[i]>(acc, dl[Tb::t.sE[AX][N][K].col[i]]);
              });
              out[K] = fmac(pw[N], acc, out[K]);
            }
          });
        }
      });
      sfor<Q>([&](auto kk) { dl[kk] = out[kk]; });
    });
  };
  if constexpr (MODE != UT_ZERO) shift(T(-1));

  // diagonal relaxation in the user basis, eq. (relaxationu): r = Rinv S R dl
  if constexpr (RLX) {
    constexpr int NC = Q - D - 1;
    T r[NC];
    sfor<NC>([&](auto ii) {
      T acc = zsum<T>();
      sfor<NC>([&](auto jj) { acc = fmac(a.relax[ii * NC + jj], dl[D + 1 + jj], acc); });
      r[ii] = acc;
    });
    sfor<NC>([&](auto ii) { dl[D + 1 + ii] = r[ii]; });
  } else {
    T r[Q];
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      if constexpr (K > D) {
        T acc = zsum<T>();
        sfor<Tb::t.sR[K].n>([&](auto i) { axpy_c<Tb::t.sR[K].val[i]>(acc, dl[Tb::t.sR[K].col[i]]); });
        r[K] = acc * a.s[K];
      } else {
        r[K] = zsum<T>();
      }
    });
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      if constexpr (K > D) {
        T acc = zsum<T>();
        sfor<Tb::t.sRinv[K].n>([&](auto i) { axpy_c<Tb::t.sRinv[K].val[i]>(acc, r[Tb::t.sRinv[K].col[i]]); });
        dl[K] = acc;
      }
    });
  }

  // shift back: T(u~)^{-1} = T(-u~) (Prop. th:csd2q9)
  if constexpr (MODE != UT_ZERO) shift(T(1));

  // back to populations: h += M_W(0)^{-1} dm  (dm vanishes on the conserved block)
  if constexpr (cube) {
    T dh[Q];
    cube_populations<B>(dl, dh);
    sfor<Q>([&](auto jj) {
      constexpr int J = jj;
      constexpr int c2 = L::c[J].x * L::c[J].x + L::c[J].y * L::c[J].y + L::c[J].z * L::c[J].z;
      if constexpr (c2 == 0) h[J] += dh[J];
      else h[J] = fmac(T(1.0 / (1 << c2)), dh[J], h[J]);
    });
  } else {
    sfor<Q>([&](auto jj) {
      constexpr int J = jj;
      T acc = zsum<T>();
      sfor<Tb::t.sMWinv[J].n>([&](auto i) { axpy_c<Tb::t.sMWinv[J].val[i]>(acc, dl[Tb::t.sMWinv[J].col[i]]); });
      h[J] += acc;
    });
  }
}

// ------------------------------------------------------------------ step kernel
// Grid: (ceil(nx / blockDim.x), ceil(ny / blockDim.y), nz).  One thread = one
// node (x, y, z).  The forms that store at the node (pull, collide,
// transport, in-place even) may run blocks of up to 1024 threads spanning
// several consecutive rows (blockDim.y > 1), so that each block streams a few
// KB of every population array contiguously (512 for FP64 storage, whose D3Q27
// collision needs more than 128 registers); the launcher picks the shape.  The scatter forms (push,
// in-place odd) run one row of at most 256 threads, and their bound says so:
// with the 1024-thread bound the D3Q27 in-place odd step was held to 128
// registers and spilled to scratch.
constexpr bool scatter_kind(int kind) { return kind == K_PUSH || kind == K_AA_ODD || kind == K_AA_ODD_WALLS; }

template <int ST, int KIND>
constexpr int step_max_threads() {
  return scatter_kind(KIND) ? 256 : (ST == 0 ? 512 : 1024);
}

// Wavefronts per SIMD the register allocation must allow (1: no constraint).
// The D3Q27 step with FP16 storage at the node takes 97 VGPRs, one past the 96
// that let a SIMD hold 5 of its wavefronts: at 5 it spends ~9 % more
// instructions on moves but measured 3.5 % faster (6 would spill to scratch).
// The scatter forms are left unconstrained: with their destinations formed
// after the collision (late_dst below) the D3Q27 FP16 ones hold 93-96 VGPRs
// and five wavefronts anyway; before that change a request for 5 made the
// in-place odd step spill 216 bytes per lane.
template <class B, int ST, int KIND>
constexpr int step_min_waves() {
  return (B::Q == 27 && ST == 2 && !scatter_kind(KIND)) ? 5 : 1;
}

// Half-way bounce-back.  wall_face_in<L, J>: the wall face that the link from
// node pos - c_J to node pos passes (-1: none): for c_J[a] > 0 the low face of
// axis a when pos[a] == 0, for c_J[a] < 0 the high face when pos[a] is the
// last index; the first axis that matches decides.
template <class L, int J>
__device__ __forceinline__ int wall_face_in(uint32_t mask, const uint32_t (&pos)[3], const uint32_t (&ext)[3]) {
  constexpr int cj[3] = {L::c[J].x, L::c[J].y, L::c[J].z};
  int face = -1;
  sfor<L::D>([&](auto ax) {
    constexpr int c = cj[ax];
    if constexpr (c > 0) {
      if (face < 0 && ((mask >> (2 * ax)) & 1u) && pos[ax] == 0) face = 2 * ax;
    } else if constexpr (c < 0) {
      if (face < 0 && ((mask >> (2 * ax + 1)) & 1u) && pos[ax] == ext[ax] - 1) face = 2 * ax + 1;
    }
  });
  return face;
}

// The population of direction J that bounced off wall `face`: the reflected
// post-collision value plus the momentum a moving wall adds,
// w_J (c_J . coef[face]) with coef = 6 rho_w u_w / lambda.
template <class B, class T, int J>
__device__ __forceinline__ T bounce(const T (&coef)[6][3], int face, T reflected) {
  using L = typename B::Lat;
  constexpr int cj[3] = {L::c[J].x, L::c[J].y, L::c[J].z};
  constexpr T wj = lit<Tab<B>::t.w[J], T>();
  T cu = zsum<T>();
  sfor<L::D>([&](auto ax) {
    if constexpr (cj[ax] != 0) cu = fmac(T(cj[ax]), coef[face][ax], cu);
  });
  return fmac(wj, cu, reflected);
}

// Workgroups are dispatched to the eight XCDs round-robin by linear block
// index, and each XCD has its own L2.  With remap set, block p instead takes
// tile t so that every XCD receives one contiguous range of tiles: tiles that
// are neighbours along x share the cache lines straddling their common edge
// (the +-1 shifted accesses) and then meet in the same L2.  A bijection for
// any block count P: XCD k = p mod 8 holds tiles [k q + min(k, r), ...) with
// q = P / 8, r = P mod 8.  (Measured: worth it while the state stays largely in
// the 256 MB last-level cache; for larger grids the natural order, where the
// eight XCDs stream neighbouring addresses at any moment, is faster.  The host
// chooses.)
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint3 block_tile(uint32_t remap) {
  if (!remap) return make_uint3(blockIdx.x, blockIdx.y, blockIdx.z);
  const uint32_t gx = gridDim.x, gy = gridDim.y;
  const uint32_t P = gx * gy * gridDim.z;
  const uint32_t p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const uint32_t k = p % kXcds, q = P / kXcds, r = P % kXcds;
  const uint32_t t = k * q + (k < r ? k : r) + p / kXcds;
  return make_uint3(t % gx, (t / gx) % gy, t / (gx * gy));
}

template <class B, int ST, int MODE, int KIND, int RLX>
__global__ __launch_bounds__((step_max_threads<ST, KIND>()))
__attribute__((amdgpu_waves_per_eu(step_min_waves<B, ST, KIND>()))) void k_step(StepArgs<typename Store<ST>::T> a) {
  using L = typename B::Lat;
  using S = typename Store<ST>::S;
  using T = typename Store<ST>::T;
  constexpr int Q = B::Q;
  constexpr int D = L::D;

  const uint3 tile = block_tile(a.xcd_remap);
  const uint32_t x = tile.x * blockDim.x + threadIdx.x;
  const uint32_t y = tile.y * blockDim.y + threadIdx.y, z = tile.z;
  if (x >= a.nx || y >= a.ny) return;
  const uint32_t nx = a.nx, ny = a.ny, nz = a.nz;
  const uint32_t xm = x == 0 ? nx - 1 : x - 1;
  const uint32_t xp = x == nx - 1 ? 0 : x + 1;
  const uint32_t ym = y == 0 ? ny - 1 : y - 1;
  const uint32_t yp = y == ny - 1 ? 0 : y + 1;
  const uint32_t zm = z == 0 ? nz - 1 : z - 1;
  const uint32_t zp = z == nz - 1 ? 0 : z + 1;
  const uint32_t own = (z * ny + y) * nx + x;

  // node offset of x + dir * c_j (dir = -1: upstream for pull, +1: downstream for push)
  auto nbr = [&](auto jj, auto dirc) -> uint32_t {
    constexpr int J = jj;
    constexpr int dir = dirc;
    constexpr int cx = dir * L::c[J].x, cy = dir * L::c[J].y, cz = dir * L::c[J].z;
    const uint32_t xx = cx == 0 ? x : (cx > 0 ? xp : xm);
    const uint32_t yy = cy == 0 ? y : (cy > 0 ? yp : ym);
    const uint32_t zz = cz == 0 ? z : (cz > 0 ? zp : zm);
    return (zz * ny + yy) * nx + xx;
  };
  // Destination node of direction j for the scatter forms.  For D3Q27 with
  // FP16 storage the compiler otherwise forms all 27 destination offsets
  // before the collision and keeps them live through it: 148 VGPRs, three
  // wavefronts per SIMD, too few loads in flight for 2-byte populations.
  // Node coordinates that an empty asm statement claims to rewrite after the
  // collision keep that work behind it (96 VGPRs, five wavefronts; in-place
  // odd step 187 -> 167 us at 192^3).  FP32 D3Q27 and D3Q19 ran 2-3 % slower
  // at their higher occupancy this way, so they keep the early form.
  constexpr bool late_dst = scatter_kind(KIND) && Q == 27 && ST == 2;
  auto dst_node = [&](auto jj, uint32_t px, uint32_t py, uint32_t pz) -> uint32_t {
    if constexpr (!late_dst) {
      return nbr(jj, std::integral_constant<int, 1>{});
    } else {
      constexpr int J = jj;
      constexpr int cx = L::c[J].x, cy = L::c[J].y, cz = L::c[J].z;
      const uint32_t xx = cx == 0 ? px : (cx > 0 ? (px == nx - 1 ? 0 : px + 1) : (px == 0 ? nx - 1 : px - 1));
      const uint32_t yy = cy == 0 ? py : (cy > 0 ? (py == ny - 1 ? 0 : py + 1) : (py == 0 ? ny - 1 : py - 1));
      const uint32_t zz = cz == 0 ? pz : (cz > 0 ? (pz == nz - 1 ? 0 : pz + 1) : (pz == 0 ? nz - 1 : pz - 1));
      return (zz * ny + yy) * nx + xx;
    }
  };

  const S* fin = static_cast<const S*>(a.fin);  // may alias fout for in-place collision
  S* fout = static_cast<S*>(a.fout);
  const uint64_t N = a.N;

  constexpr bool aa_odd = KIND == K_AA_ODD || KIND == K_AA_ODD_WALLS;
  constexpr bool gather = KIND == K_PULL || KIND == K_STREAM || aa_odd;
  const uint32_t pos[3] = {x, y, z}, ext[3] = {nx, ny, nz};
  T h[Q];
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    constexpr int slot = aa_odd ? opposite<L>(J) : J;
    if constexpr (KIND == K_AA_ODD_WALLS) {
      // in place, with walls: a population whose source lies beyond a wall is
      // read from this node's slot J, where the even step left the opposite
      // post-collision population (the periodic source slot is another node's
      // to rewrite in this pass, so it is not read)
      if (a.wall_mask) {
        const int face = wall_face_in<L, J>(a.wall_mask, pos, ext);
        if (face >= 0) {
          h[J] = bounce<B, T, J>(a.wall_coef, face, T(fin[(uint64_t)J * N + own]));
          return;
        }
      }
    }
    uint32_t src = own;
    if constexpr (gather) src = nbr(jj, std::integral_constant<int, -1>{});
    // loads that are aligned with the wavefront (own node, or a neighbour in y
    // or z only) bypass the caches; the +-1 shifted ones along x share cache
    // lines with the neighbouring wavefront and go through L2.  D3Q27's
    // two-array gathers stream all 27 past the caches (18 of its populations
    // are x-shifted): +2.6 % at 192^3 FP32, where D3Q19 and D2Q9 lost 2-3 %.
    constexpr bool all_nt = Q == 27 && (KIND == K_PULL || KIND == K_STREAM);
    constexpr bool aligned = KIND == K_COLLIDE || KIND == K_AA_EVEN || (gather && (L::c[J].x == 0 || all_nt));
    if constexpr (aligned) h[J] = T(__builtin_nontemporal_load(&fin[(uint64_t)slot * N + src]));
    else h[J] = T(fin[(uint64_t)slot * N + src]);
  });
  // half-way bounce-back on wall faces (two-array pull forms): a population
  // whose source lies beyond a wall is the node's own post-collision opposite
  // population, kept in slot opp(J) at the node, plus the momentum of a
  // moving wall
  if constexpr (KIND == K_PULL || KIND == K_STREAM) {
    if (a.wall_mask) {
      sfor<Q>([&](auto jj) {
        constexpr int J = jj;
        const int face = wall_face_in<L, J>(a.wall_mask, pos, ext);
        if (face >= 0) h[J] = bounce<B, T, J>(a.wall_coef, face, T(fin[(uint64_t)opposite<L>(J) * N + own]));
      });
    }
  }

  if constexpr (KIND != K_STREAM) {
    T utf[3] = {T(0), T(0), T(0)};
    if constexpr (MODE == UT_FIELD) {
      sfor<D>([&](auto al) { utf[al] = T(a.ut[(uint64_t)al * N + own]) * a.inv_lambda; });
    }
    collide_node<B, T, MODE, RLX>(h, a, utf);
  }
  uint32_t px = x, py = y, pz = z;
  if constexpr (late_dst) asm volatile("" : "+v"(px), "+v"(py), "+v"(pz));

  // Stores: the gather forms write their own node (aligned, contiguous per
  // wavefront) and are streamed past the caches with non-temporal stores, which
  // measured ~5% faster on MI355X for arrays far larger than L2 and MALL.  The
  // scatter forms do the same for the populations without an x-shift and use
  // plain stores for the +-1 shifted ones, whose partial lines L2 then merges.
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    if constexpr (KIND == K_AA_ODD_WALLS) {
      // in-place form with walls: a population whose destination lies beyond a
      // wall returns to this node as direction opp(J), bounced, into slot
      // opp(J) here (the slot this node's read of that link would have used)
      if (a.wall_mask) {
        constexpr int O = opposite<L>(J);
        const int face = wall_face_in<L, O>(a.wall_mask, pos, ext);
        if (face >= 0) {
          fout[(uint64_t)O * N + own] = S(bounce<B, T, O>(a.wall_coef, face, h[J]));
          return;
        }
      }
    }
    if constexpr (KIND == K_PUSH || aa_odd) {
      S* dst = &fout[(uint64_t)J * N + dst_node(jj, px, py, pz)];
      if constexpr (L::c[J].x == 0) __builtin_nontemporal_store(S(h[J]), dst);  // aligned with the wavefront
      else *dst = S(h[J]);
    } else {
      constexpr int slot = KIND == K_AA_EVEN ? opposite<L>(J) : J;
      __builtin_nontemporal_store(S(h[J]), &fout[(uint64_t)slot * N + own]);
    }
  });
}

// ------------------------------------------------------------------ in place, FP16, node pairs
// The even in-place step with FP16 storage on D3Q19, two nodes per thread:
// nodes x and x + 1 of a row, x even (the host launches this form for even
// nx).  The even step reads and writes only its own nodes, so each
// population of the pair is one aligned 4-byte word, loaded and stored
// non-temporally; the pair shares the address arithmetic and issues half the
// memory instructions, which matters because the FP16 step is bound by the
// vector ALU about as much as by HBM.  Each node's collision (collide_node)
// and FP16 rounding are those of k_step, so both kernels store the same bits.
// (Measured on D3Q19 256^3: 220 -> 194 us.  The odd step's x-shifted pairs
// would need 2-byte-aligned dword accesses, which measured slower than the
// single-node kernel (254 -> 353 us), and D3Q27's pair needs ~175 registers,
// two wavefronts per SIMD: 150 -> 162 us; both keep k_step.)
__device__ __forceinline__ void unpack_f16x2(uint32_t w, float& lo, float& hi) {
  lo = float(__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)));
  hi = float(__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)));
}
__device__ __forceinline__ uint32_t pack_f16x2(float lo, float hi) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)lo) | ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)hi) << 16);
}

template <class B, int MODE, int RLX>
__global__ __launch_bounds__(256) void k_aa_even_pair(StepArgs<float> a) {
  using L = typename B::Lat;
  using S = _Float16;
  using T = float;
  constexpr int Q = B::Q;
  constexpr int D = L::D;

  const uint3 tile = block_tile(a.xcd_remap);
  const uint32_t x = 2 * (tile.x * blockDim.x + threadIdx.x);  // first node of the pair
  const uint32_t y = tile.y * blockDim.y + threadIdx.y, z = tile.z;
  if (x >= a.nx || y >= a.ny) return;
  const uint32_t own = (z * a.ny + y) * a.nx + x;
  const uint64_t N = a.N;
  const S* fin = static_cast<const S*>(a.fin);
  S* fout = static_cast<S*>(a.fout);

  T h0[Q], h1[Q];
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    const uint32_t w = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(&fin[(uint64_t)J * N + own]));
    unpack_f16x2(w, h0[J], h1[J]);
  });
  T u0[3] = {T(0), T(0), T(0)}, u1[3] = {T(0), T(0), T(0)};
  if constexpr (MODE == UT_FIELD) {
    sfor<D>([&](auto al) {
      u0[al] = T(a.ut[(uint64_t)al * N + own]) * a.inv_lambda;
      u1[al] = T(a.ut[(uint64_t)al * N + own + 1]) * a.inv_lambda;
    });
  }
  collide_node<B, T, MODE, RLX>(h0, a, u0);
  collide_node<B, T, MODE, RLX>(h1, a, u1);
  // slot opp(J) at the pair's own nodes
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    __builtin_nontemporal_store(pack_f16x2(h0[J], h1[J]),
                                reinterpret_cast<uint32_t*>(&fout[(uint64_t)opposite<L>(J) * N + own]));
  });
}

// After an even-form in-place step the array holds f*_j(x) in slot opp(j) at x;
// the natural layout needs f_j(x) = f*_j(x - c_j).  Slots (j at x) and (opp(j)
// at x - c_j) trade places, so one thread per node swaps one pair per
// direction j with c_j > 0 in lexicographic order (each pair exactly once).
// With walls (on both faces of an axis), a pair whose link passes a wall is
// not swapped: each of its two slots already holds its node's bounced
// population, which only gains the moving-wall term.
struct FinArgs {
  uint32_t wall_mask;
  double wall_coef[6][3];
};

template <class B, int ST>
__global__ __launch_bounds__(256) void k_aa_finish(void* fp, uint32_t nx, uint32_t ny, uint32_t nz, uint64_t N,
                                                   FinArgs w) {
  using L = typename B::Lat;
  using S = typename Store<ST>::S;
  using T = typename Store<ST>::T;
  constexpr int Q = B::Q;
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t y = blockIdx.y, z = blockIdx.z;
  if (x >= nx) return;
  S* f = static_cast<S*>(fp);
  const uint32_t own = (z * ny + y) * nx + x;
  const uint32_t pos[3] = {x, y, z}, ext[3] = {nx, ny, nz};
  T coef[6][3];
  for (int i = 0; i < 6; ++i)
    for (int ax = 0; ax < 3; ++ax) coef[i][ax] = T(w.wall_coef[i][ax]);
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    const int face = w.wall_mask ? wall_face_in<L, J>(w.wall_mask, pos, ext) : -1;
    if (face >= 0) {
      S* p = &f[(uint64_t)J * N + own];
      *p = S(bounce<B, T, J>(coef, face, T(*p)));
      return;
    }
    constexpr int cx = L::c[J].x, cy = L::c[J].y, cz = L::c[J].z;
    constexpr bool positive = cz > 0 || (cz == 0 && (cy > 0 || (cy == 0 && cx > 0)));
    if constexpr (positive) {
      const uint32_t xs = cx == 0 ? x : (cx > 0 ? (x == 0 ? nx - 1 : x - 1) : (x == nx - 1 ? 0 : x + 1));
      const uint32_t ys = cy == 0 ? y : (cy > 0 ? (y == 0 ? ny - 1 : y - 1) : (y == ny - 1 ? 0 : y + 1));
      const uint32_t zs = cz == 0 ? z : (cz > 0 ? (z == 0 ? nz - 1 : z - 1) : (z == nz - 1 ? 0 : z + 1));
      S* p = &f[(uint64_t)J * N + own];
      S* q = &f[(uint64_t)opposite<L>(J) * N + (zs * ny + ys) * nx + xs];
      const S t = *p;
      *p = *q;
      *q = t;
    }
  });
}

// ------------------------------------------------------------------ moments
template <class T>
struct MomArgs {
  const void* f;
  void* rho;   // [N]
  void* u;     // [d][N]
  void* m0;    // [q][N] or null
  uint64_t N;
  T rho0, lambda;
  const T* rmat;  // run-time basis only: R of P = R W, Q x Q row-major (m0 then in xi = X / lambda units)
};

// rho, u (physical units) and optionally the fixed-frame user moments
// m(0) = M(0) f (eq. (matort) for the D2Q9 paper basis), all per node.
template <class B, int ST>
__global__ __launch_bounds__(256) void k_moments(MomArgs<typename Store<ST>::T> a) {
  using L = typename B::Lat;
  using S = typename Store<ST>::S;
  using T = typename Store<ST>::T;
  using O = T;  // output element type
  constexpr int Q = B::Q;
  constexpr int D = L::D;
  using Tb = Tab<B>;
  const uint64_t n = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  const S* f = static_cast<const S*>(a.f);
  T h[Q];
  sfor<Q>([&](auto jj) { h[jj] = T(f[(uint64_t)jj * a.N + n]); });
  T drho = h[0];
  sfor<Q - 1>([&](auto jj) { drho += h[jj + 1]; });
  T jm[3] = {T(0), T(0), T(0)};
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    if constexpr (L::c[J].x != 0) jm[0] += T(L::c[J].x) * h[J];
    if constexpr (L::c[J].y != 0) jm[1] += T(L::c[J].y) * h[J];
    if constexpr (L::c[J].z != 0) jm[2] += T(L::c[J].z) * h[J];
  });
  const T rho = a.rho0 + drho;
  static_cast<O*>(a.rho)[n] = O(rho);
  sfor<D>([&](auto al) { static_cast<O*>(a.u)[(uint64_t)al * a.N + n] = O(a.lambda * jm[al] / rho); });
  if (a.m0 && a.rmat) {
    // run-time basis: m0 = R M_W(0) f
    T mw[Q];
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      T acc = T(0);
      sfor<Tb::t.sMW[K].n>([&](auto i) { axpy_c<Tb::t.sMW[K].val[i]>(acc, h[Tb::t.sMW[K].col[i]]); });
      constexpr Rat restK = [] {
        Rat r;
        for (int j = 0; j < Q; ++j) r = r + Tb::t.MW.m[K][j] * Tb::t.w[j];
        return r;
      }();
      if constexpr (!restK.zero()) acc = fmac(lit<restK, T>(), a.rho0, acc);
      mw[K] = acc;
    });
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      T acc = T(0);
      sfor<Q>([&](auto ll) { acc = fmac(a.rmat[K * Q + ll], mw[ll], acc); });
      static_cast<O*>(a.m0)[(uint64_t)K * a.N + n] = O(acc);
    });
  } else if (a.m0) {
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      T acc = T(0);
      sfor<Tb::t.sMP[K].n>([&](auto i) { axpy_c<Tb::t.sMP[K].val[i]>(acc, h[Tb::t.sMP[K].col[i]]); });
      constexpr Rat restK = Tb::t.restP[K];
      if constexpr (!restK.zero()) acc = fmac(lit<restK, T>(), a.rho0, acc);
      T sc = T(1);
      sfor<Tb::t.lam_deg[K]>([&](auto) { sc *= a.lambda; });
      static_cast<O*>(a.m0)[(uint64_t)K * a.N + n] = O(acc * sc);
    });
  }
}

// ------------------------------------------------------------------ initial state
// f_j = f^eq_j(rho, u) + amp * noise_j in FP64 (equilibrium of section 1.2 with
// the second-order polynomial form), stored minus w_j rho0 in the storage type.
// rho [N], u [d][N] (physical units), noise [q][N] or null.
template <class B, int ST>
__global__ __launch_bounds__(256) void k_init_eq(const double* rho, const double* u, const double* noise, double amp,
                                                 double rho0, double lambda, uint64_t N, void* fout) {
  using L = typename B::Lat;
  using S = typename Store<ST>::S;
  using Tb = Tab<B>;
  constexpr int Q = B::Q;
  constexpr int D = L::D;
  const uint64_t n = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double r = rho[n];
  double uu[3] = {0, 0, 0};
  sfor<D>([&](auto al) { uu[al] = u[(uint64_t)al * N + n] / lambda; });
  const double u2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
  S* f = static_cast<S*>(fout);
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    constexpr double w = Tb::t.w[J].val();
    const double cu = double(L::c[J].x) * uu[0] + double(L::c[J].y) * uu[1] + double(L::c[J].z) * uu[2];
    double fe = w * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u2);
    if (noise) fe += amp * noise[(uint64_t)J * N + n];
    f[(uint64_t)J * N + n] = S(fe - w * rho0);
  });
}

// Storage <-> FP64 conversion: f64 = stored + w_j rho0, stored = rn(f64 - w_j rho0).
template <class B, int ST>
__global__ __launch_bounds__(256) void k_convert(const void* in, void* out, double rho0, uint64_t N, int to_storage) {
  using S = typename Store<ST>::S;
  using Tb = Tab<B>;
  constexpr int Q = B::Q;
  const uint64_t n = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  sfor<Q>([&](auto jj) {
    constexpr double w = Tb::t.w[jj].val();
    const uint64_t i = (uint64_t)jj * N + n;
    if (to_storage) static_cast<S*>(out)[i] = S(static_cast<const double*>(in)[i] - w * rho0);
    else static_cast<double*>(out)[i] = double(static_cast<const S*>(in)[i]) + w * rho0;
  });
}

// ------------------------------------------------------------------ conservation
// FP64 block partial sums of (sum h, sum c h, non-finite count) per block.
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

template <class B, int ST>
__global__ __launch_bounds__(kRedThreads) void k_conserve_partial(const void* fp, uint64_t N, double* partial) {
  using L = typename B::Lat;
  using S = typename Store<ST>::S;
  constexpr int Q = B::Q;
  const S* f = static_cast<const S*>(fp);
  double acc[5] = {0, 0, 0, 0, 0};
  for (uint64_t n = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (uint64_t)gridDim.x * blockDim.x) {
    sfor<Q>([&](auto jj) {
      constexpr int J = jj;
      const double v = double(f[(uint64_t)J * N + n]);
      if (!__builtin_isfinite(v)) acc[4] += 1.0;
      acc[0] += v;
      if constexpr (L::c[J].x != 0) acc[1] += double(L::c[J].x) * v;
      if constexpr (L::c[J].y != 0) acc[2] += double(L::c[J].y) * v;
      if constexpr (L::c[J].z != 0) acc[3] += double(L::c[J].z) * v;
    });
  }
  __shared__ double red[5][kRedThreads];
  for (int i = 0; i < 5; ++i) red[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int i = 0; i < 5; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int i = 0; i < 5; ++i) partial[(uint64_t)blockIdx.x * 5 + i] = red[i][0];
}

// Distance from a uniform reference state, for the growth rate of small
// perturbations (linear stability).  ref[j] is the reference population in the
// stored representation (f_ref_j - w_j rho0 for the deviation storages).
struct DevRef {
  double r[27];
};

// Squared distance sum_j (f_j - ref_j)^2 per node, block partial sums in FP64
// in the 5-slot layout of k_conserve_partial (slot 0: the sum, slot 4: count
// of non-finite values, slots 1-3: zero).
template <class B, int ST>
__global__ __launch_bounds__(kRedThreads) void k_dev_partial(const void* fp, uint64_t N, DevRef ref, double* partial) {
  using S = typename Store<ST>::S;
  constexpr int Q = B::Q;
  const S* f = static_cast<const S*>(fp);
  double acc = 0.0, bad = 0.0;
  for (uint64_t n = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (uint64_t)gridDim.x * blockDim.x) {
    sfor<Q>([&](auto jj) {
      constexpr int J = jj;
      const double v = double(f[(uint64_t)J * N + n]);
      if (!__builtin_isfinite(v)) bad += 1.0;
      const double d = v - ref.r[J];
      acc = __builtin_fma(d, d, acc);
    });
  }
  __shared__ double red[2][kRedThreads];
  red[0][threadIdx.x] = acc;
  red[1][threadIdx.x] = bad;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 5) {
    const double v = threadIdx.x == 0 ? red[0][0] : threadIdx.x == 4 ? red[1][0] : 0.0;
    partial[(uint64_t)blockIdx.x * 5 + threadIdx.x] = v;
  }
}

// f_j <- ref_j + factor (f_j - ref_j) at every node (FP64, then the storage's
// arithmetic type and rounding).
template <class B, int ST>
__global__ __launch_bounds__(256) void k_dev_scale(void* fp, uint64_t N, DevRef ref, double factor) {
  using S = typename Store<ST>::S;
  using T = typename Store<ST>::T;
  constexpr int Q = B::Q;
  const uint64_t n = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  S* f = static_cast<S*>(fp);
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    const uint64_t i = (uint64_t)J * N + n;
    const double v = ref.r[J] + factor * (double(f[i]) - ref.r[J]);
    f[i] = S(T(v));
  });
}

// Sums kRedBlocks partials in a fixed order (one block), deterministic.
__global__ __launch_bounds__(kRedThreads) void k_conserve_final(const double* partial, double* out, double add0,
                                                                double scale, int d);

}  // namespace lbmrv
