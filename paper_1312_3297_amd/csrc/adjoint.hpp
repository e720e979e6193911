// Adjoint of one time step (relaxation in the moving frame, then transport),
// for a relative velocity that is zero, a given field, or alpha times the local
// fluid velocity (then u~ depends on f and its derivative enters lambda).
//
// Forward step at node x (scatter form, pre-collision states):
//   f^{n+1}_j(x + c_j) = f*_j(x),
//   f* = f + M_W^{-1} T(-u~) R^{-1} S R T(u~) d0,   d0 = m^eq_W(rho, u) - M_W f
// (eq. (relaxationu) written on increments, T(u~) = prod_a exp(-u~_a D_a)).
// With g_j = lambda^{n+1}_j(x + c_j) (the transpose of the transport), the
// transpose of the collision Jacobian is, with the working vectors
//   z1 = M_W^{-T} g,  z2 = T(-u~)^T z1,  z3 = R^{-T} z2,  z5 = R^T S z3,
//   z6 = T(u~)^T z5,  y = M_W^T z6:
//   lambda^n_i = g_i - y_i + dm^eq/dh_i . z6
//   dJ/ds_k   += z3_k (R T(u~) d0)_k
//   dJ/du~_a  += z2 . D_a (R^{-1} S R v) - z5 . D_a v,   v = T(u~) d0
// using d/du~_a T(u~) = -D_a T(u~) and that the D_a commute with T.
// With u~ = alpha u(f): du~_a/dh_i = alpha (c_ia - u_a) / rho, so dJ/du~_a
// (lattice units) is folded into lambda instead of being accumulated.
#pragma once

#include "kernels.hpp"

namespace lbmrv {

template <class T>
struct AdjArgs {
  const void* f;       // f^n, storage type, [q][N]
  const T* lam_in;     // lambda^{n+1} [q][N]
  T* lam_out;          // lambda^n [q][N]
  const float* ut;     // [d][N] u~ field in physical units (FIELD) or null
  double* grad_ut;     // [d][N] FP64 accumulators (FIELD) or null
  double* partial;     // [nblocks][Q] FP64 accumulators of dJ/ds, one row per block
  uint32_t nx, ny, nz;
  uint64_t N;
  T rho0, inv_lambda, alpha;
  T s[27];
  const void* f_prev;  // two-step kernel: f^{n-1}, storage type, [q][N] (f is then f^n)
  const T* rnn;     // run-time basis only: non-conserved block of R (P = R W), (Q-D-1)^2 row-major
  const T* rnninv;  // and its inverse
  uint32_t xcd_remap;  // block order, as for the step kernels (block_tile)
  uint32_t eq_maxwell; // 1: equilibrium moments of the continuous Maxwellian
};

// The adjoint of one time step at one node (the transpose of the collision
// Jacobian, with the equations at the top of this file): from the node's
// populations h (stored values), the gathered adjoint g_j = lambda^{n+1}_j(x +
// c_j) and, for a given field, u~ in lattice units, it returns lambda^n at the
// node, the node's dJ/du~ in lattice units (a field; folded into lambda for
// u~ = alpha u), and z3, r whose products z3_k r_k are the node's dJ/ds_k.
template <class B, int ST, int MODE, int RLX>
__device__ __forceinline__ void adjoint_node(const AdjArgs<typename Store<ST>::T>& a,
                                             const typename Store<ST>::T (&h)[B::Q],
                                             const typename Store<ST>::T (&g)[B::Q],
                                             const typename Store<ST>::T (&utf)[3],
                                             typename Store<ST>::T (&lam_out)[B::Q],
                                             typename Store<ST>::T (&gut_out)[3],
                                             typename Store<ST>::T (&z3_out)[B::Q],
                                             typename Store<ST>::T (&r_out)[B::Q]) {
  using L = typename B::Lat;
  using T = typename Store<ST>::T;
  using Tb = Tab<B>;
  constexpr int Q = B::Q;
  constexpr int D = L::D;

  // ---- forward quantities at this node (monomial bases on {0, +-1}^d with
  // FP32 arithmetic: all moments, and below the two transposed maps, by the
  // cube passes of the forward kernel)
  constexpr bool cube = CubeForm<B>::applies() && sizeof(T) == 4;
  T mw[cube ? Q : 1];
  if constexpr (cube) cube_moments<B>(h, mw);
  T drho, jm[3] = {zsum<T>(), zsum<T>(), zsum<T>()};
  if constexpr (cube) {
    drho = mw[0];
    sfor<D>([&](auto al) { jm[al] = mw[1 + al]; });
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
  const T u[3] = {jm[0] * irho, jm[1] * irho, D == 3 ? jm[2] * irho : T(0)};
  T ut[3] = {T(0), T(0), T(0)};
  if constexpr (MODE == UT_FIELD) {
    sfor<D>([&](auto al) { ut[al] = utf[al]; });
  } else if constexpr (MODE == UT_FLUID) {
    sfor<D>([&](auto al) { ut[al] = a.alpha * u[al]; });
  }

  // Maxwellian option: per-axis moments E[xi^n] of N(u_a, cs2) (cs2 = 1/3 in
  // lattice units, the same expressions as the forward kernel) and their
  // derivatives with respect to u_a
  const bool maxwell = a.eq_maxwell != 0;
  T mu[3][kP], dmu[3][kP];
  if (maxwell) {
    constexpr T cs2 = T(1) / T(3);
    sfor<3>([&](auto ax) {
      const T w = ax < D ? u[ax] : T(0);
      const T w2 = w * w;
      mu[ax][0] = T(1);
      mu[ax][1] = w;
      mu[ax][2] = w2 + cs2;
      mu[ax][3] = w * (w2 + T(3) * cs2);
      mu[ax][4] = w2 * (w2 + T(6) * cs2) + T(3) * cs2 * cs2;
      dmu[ax][0] = T(0);
      dmu[ax][1] = T(1);
      dmu[ax][2] = T(2) * w;
      dmu[ax][3] = T(3) * (w2 + cs2);
      dmu[ax][4] = T(4) * w * (w2 + T(3) * cs2);
    });
  }
  // E_K = E[W_K(xi)] (so m^eq_K = rho E_K) and dE_K / du
  auto maxwell_moment = [&](auto kk, T (&dek)[3]) -> T {
    constexpr Poly pk = B::W(decltype(kk)::value);
    T ek = zsum<T>();
    sfor<3>([&](auto al) { dek[al] = zsum<T>(); });
    sfor<pk.n>([&](auto ti) {
      constexpr PTerm tm = pk.t[ti];
      constexpr int ex[3] = {tm.a, tm.b, tm.e};
      const T c = lit<tm.c, T>();
      ek = fmac(c, mu[0][tm.a] * mu[1][tm.b] * mu[2][tm.e], ek);
      sfor<D>([&](auto al) {
        if constexpr (ex[al] > 0) {
          T prod = dmu[al][ex[al]];
          sfor<3>([&](auto bx) {
            if constexpr (bx != al) prod *= mu[bx][ex[bx]];
          });
          dek[al] = fmac(c, prod, dek[al]);
        }
      });
    });
    return ek;
  };

  T v[Q];  // d0, then T(u~) d0
  T mh[Q];
  sfor<Q>([&](auto kk) {
    constexpr int K = kk;
    if constexpr (K <= D) {
      v[K] = zsum<T>();
    } else if constexpr (cube) {
      mh[K] = mw[K];
    } else {
      mh[K] = zsum<T>();
      sfor<Tb::t.sMW[K].n>([&](auto i) { axpy_c<Tb::t.sMW[K].val[i]>(mh[K], h[Tb::t.sMW[K].col[i]]); });
    }
  });
  // one uniform branch for all moments (neither equilibrium is evaluated and
  // then discarded)
  if (maxwell) {
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      if constexpr (K > D) {
        T dek[3];
        const T ek = maxwell_moment(kk, dek);
        constexpr Rat ak = Tb::t.a[K];
        v[K] = fmac(rho, ek, -(lit<ak, T>() * a.rho0)) - mh[K];
      }
    });
  } else {
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
        v[K] = eq - mh[K];
      }
    });
  }

  // out = prod_a exp(sign u~_a D_a) in (rows: transposed or not), non-conserved block
  auto apply_shift = [&](T (&w)[Q], T sign, auto transposed) {
    constexpr bool TR = decltype(transposed)::value;
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
        out[K] = w[K];
        if constexpr (K > D) {
          sfor<NM>([&](auto nn) {
            constexpr int NN = nn + 1;
            constexpr auto row = TR ? Tb::t.tE[AX][NN][K] : Tb::t.sE[AX][NN][K];
            if constexpr (row.n == 1) {
              // one term: its constant goes into the (shared) power
              out[K] = fmac(lit<row.val[0], T>() * pw[NN], w[row.col[0]], out[K]);
            } else if constexpr (row.n > 1) {
              T acc = zsum<T>();
              sfor<row.n>([&](auto i) { axpy_c<row.val[i]>(acc, w[row.col[i]]); });
              out[K] = fmac(pw[NN], acc, out[K]);
            }
          });
        }
      });
      sfor<Q>([&](auto kk) { w[kk] = out[kk]; });
    });
  };
  if constexpr (MODE != UT_ZERO) apply_shift(v, T(-1), std::false_type{});

  constexpr int NC = Q - D - 1;
  // y = M x (or M^T x) on the non-conserved block for a run-time NC x NC matrix
  auto dense = [&](const T* m, const T (&x)[Q], T (&y)[Q], auto transposed, auto scale_by_s) {
    constexpr bool TR = decltype(transposed)::value;
    constexpr bool SC = decltype(scale_by_s)::value;
    sfor<D + 1>([&](auto kk) { y[kk] = zsum<T>(); });
    sfor<NC>([&](auto ii) {
      T acc = zsum<T>();
      sfor<NC>([&](auto jj) {
        const T xv = SC ? x[D + 1 + jj] * a.s[D + 1 + jj] : x[D + 1 + jj];
        acc = fmac(TR ? m[jj * NC + ii] : m[ii * NC + jj], xv, acc);
      });
      y[D + 1 + ii] = acc;
    });
  };

  T r[Q], am[Q];  // r = R v (user basis), am = R^{-1} S r
  if constexpr (RLX) {
    dense(a.rnn, v, r, std::false_type{}, std::false_type{});
    dense(a.rnninv, r, am, std::false_type{}, std::true_type{});
  } else {
  sfor<Q>([&](auto kk) {
    constexpr int K = kk;
    T acc = zsum<T>();
    if constexpr (K > D) sfor<Tb::t.sR[K].n>([&](auto i) { axpy_c<Tb::t.sR[K].val[i]>(acc, v[Tb::t.sR[K].col[i]]); });
    r[K] = acc;
  });
  sfor<Q>([&](auto kk) {
    constexpr int K = kk;
    T acc = zsum<T>();
    if constexpr (K > D)
      sfor<Tb::t.sRinv[K].n>([&](auto i) {
        constexpr int l = Tb::t.sRinv[K].col[i];
        axpy_c<Tb::t.sRinv[K].val[i]>(acc, r[l] * a.s[l]);
      });
    am[K] = acc;
  });
  }

  // ---- adjoint
  T zz[Q];  // z1 = M_W(0)^{-T} g, then z2 (in place through the shift)
  if constexpr (cube) {
    cube_populations_t<B>(g, zz);
  } else {
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      T acc = zsum<T>();
      if constexpr (K > D)
        sfor<Tb::t.tMWinv[K].n>([&](auto i) { axpy_c<Tb::t.tMWinv[K].val[i]>(acc, g[Tb::t.tMWinv[K].col[i]]); });
      zz[K] = acc;
    });
  }
  if constexpr (MODE != UT_ZERO) apply_shift(zz, T(1), std::true_type{});  // z2 = T(-u~)^T z1

  T z3[Q], z5[Q];  // z3 = R^{-T} z2, z5 = R^T S z3
  if constexpr (RLX) {
    dense(a.rnninv, zz, z3, std::true_type{}, std::false_type{});
    dense(a.rnn, z3, z5, std::true_type{}, std::true_type{});
  } else {
  sfor<Q>([&](auto kk) {
    constexpr int K = kk;
    T acc = zsum<T>();
    if constexpr (K > D)
      sfor<Tb::t.tRinv[K].n>([&](auto i) { axpy_c<Tb::t.tRinv[K].val[i]>(acc, zz[Tb::t.tRinv[K].col[i]]); });
    z3[K] = acc;
  });
  sfor<Q>([&](auto kk) {
    constexpr int K = kk;
    T acc = zsum<T>();
    if constexpr (K > D)
      sfor<Tb::t.tR[K].n>([&](auto i) {
        constexpr int l = Tb::t.tR[K].col[i];
        axpy_c<Tb::t.tR[K].val[i]>(acc, z3[l] * a.s[l]);
      });
    z5[K] = acc;
  });
  }

  // dJ/du~_a = z2 . D_a am - z5 . D_a v (lattice units): accumulated per node in
  // physical units for a given field, folded into lambda for u~ = alpha u
  T gut[3] = {T(0), T(0), T(0)};
  if constexpr (MODE != UT_ZERO) {
    sfor<D>([&](auto ax) {
      constexpr int AX = ax;
      T gsum = zsum<T>();
      sfor<Q>([&](auto kk) {
        constexpr int K = kk;
        constexpr auto row = Tb::t.sE[AX][1][K];
        if constexpr (K > D && row.n > 0) {
          T da = zsum<T>(), dv = zsum<T>();
          sfor<row.n>([&](auto i) {
            axpy_c<row.val[i]>(da, am[row.col[i]]);
            axpy_c<row.val[i]>(dv, v[row.col[i]]);
          });
          gsum = fmac(zz[K], da, gsum);
          gsum = fmac(-z5[K], dv, gsum);
        }
      });
      gut[AX] = gsum;
    });
  }

  // z6 = T(u~)^T z5
  if constexpr (MODE != UT_ZERO) apply_shift(z5, T(-1), std::true_type{});

  // lambda^n = g - M_W^T z6 + (d m^eq / d h)^T z6
  T A0 = zsum<T>(), Bv[3] = {zsum<T>(), zsum<T>(), zsum<T>()};
  if (maxwell) {
    // d(rho E_K)/dh_j = E_K + sum_a dE_K/du_a (c_ja - u_a)
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      if constexpr (K > D) {
        T dek[3];
        const T ek = maxwell_moment(kk, dek);
        A0 = fmac(z5[K], ek, A0);
        sfor<D>([&](auto al) { Bv[al] = fmac(z5[K], dek[al], Bv[al]); });
      }
    });
  } else {
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      if constexpr (K > D) {
        T quad = zsum<T>();
        sfor<D>([&](auto al) {
          constexpr Rat bb = Tb::t.b[K][al];
          T dq = zsum<T>();
          if constexpr (!bb.zero()) {
            quad = fmac(lit<bb, T>(), u[al], quad);
            dq = lit<bb, T>();
          }
          sfor<D>([&](auto be) {
            constexpr Rat cab = Tb::t.C[K][al][be];
            constexpr Rat csym = Tb::t.C[K][al][be] + Tb::t.C[K][be][al];
            if constexpr (!cab.zero()) quad = fmac(lit<cab, T>() * u[al], u[be], quad);
            if constexpr (!csym.zero()) dq = fmac(lit<csym, T>(), u[be], dq);
          });
          Bv[al] = fmac(z5[K], dq, Bv[al]);
        });
        constexpr Rat ak = Tb::t.a[K];
        A0 = fmac(z5[K], lit<ak, T>() + quad, A0);
      }
    });
  }
  if constexpr (MODE == UT_FLUID) {
    sfor<D>([&](auto al) { Bv[al] = fmac(a.alpha * irho, gut[al], Bv[al]); });
  }
  T yt[cube ? Q : 1];  // M_W(0)^T z6
  if constexpr (cube) cube_moments_t<B>(z5, yt);
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    T yv = zsum<T>();
    if constexpr (cube) {
      yv = yt[J];
    } else {
      sfor<Tb::t.tMW[J].n>([&](auto i) { axpy_c<Tb::t.tMW[J].val[i]>(yv, z5[Tb::t.tMW[J].col[i]]); });
    }
    T lam = g[J] - yv + A0;
    sfor<D>([&](auto al) {
      constexpr int cj = al == 0 ? L::c[J].x : al == 1 ? L::c[J].y : L::c[J].z;
      lam = fmac(Bv[al], T(cj) - u[al], lam);
    });
    lam_out[J] = lam;
  });
  sfor<3>([&](auto ax) { gut_out[ax] = gut[ax]; });
  sfor<Q>([&](auto kk) {
    z3_out[kk] = z3[kk];
    r_out[kk] = r[kk];
  });

}

template <class B, int ST, int MODE, int RLX>
__global__ __launch_bounds__(256) void k_adjoint(AdjArgs<typename Store<ST>::T> a) {
  using L = typename B::Lat;
  using S = typename Store<ST>::S;
  using T = typename Store<ST>::T;
  constexpr int Q = B::Q;
  constexpr int D = L::D;

  const uint3 tile = block_tile(a.xcd_remap);
  const uint32_t xr = tile.x * blockDim.x + threadIdx.x;
  const bool active = xr < a.nx;
  const uint32_t x = active ? xr : a.nx - 1;  // inactive lanes recompute a valid node, store nothing
  const uint32_t y = tile.y, z = tile.z;
  const uint32_t nx = a.nx, ny = a.ny, nz = a.nz;
  const uint32_t xp = x == nx - 1 ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
  const uint32_t yp = y == ny - 1 ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
  const uint32_t zp = z == nz - 1 ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;
  const uint32_t own = (z * ny + y) * nx + x;
  const uint64_t N = a.N;
  const S* f = static_cast<const S*>(a.f);

  T h[Q], g[Q];
  sfor<Q>([&](auto jj) {
    constexpr int J = jj;
    constexpr int cx = L::c[J].x, cy = L::c[J].y, cz = L::c[J].z;
    const uint32_t xx = cx == 0 ? x : (cx > 0 ? xp : xm);
    const uint32_t yy = cy == 0 ? y : (cy > 0 ? yp : ym);
    const uint32_t zz = cz == 0 ? z : (cz > 0 ? zp : zm);
    // accesses aligned with the wavefront stream past the caches; the +-1
    // shifted gathers along x share lines with the neighbouring wavefront
    h[J] = T(__builtin_nontemporal_load(&f[(uint64_t)J * N + own]));
    const T* src = &a.lam_in[(uint64_t)J * N + (zz * ny + yy) * nx + xx];
    if constexpr (cx == 0) g[J] = __builtin_nontemporal_load(src);
    else g[J] = *src;
  });

  T utf[3] = {T(0), T(0), T(0)};
  if constexpr (MODE == UT_FIELD) {
    sfor<D>([&](auto al) { utf[al] = T(a.ut[(uint64_t)al * N + own]) * a.inv_lambda; });
  }
  T lam[Q], gut[3], z3[Q], r[Q];
  adjoint_node<B, ST, MODE, RLX>(a, h, g, utf, lam, gut, z3, r);
  if constexpr (MODE == UT_FIELD) {
    if (active) sfor<D>([&](auto ax) { a.grad_ut[(uint64_t)ax * N + own] += double(gut[ax] * a.inv_lambda); });
  }
  if (active) {
    sfor<Q>([&](auto jj) { __builtin_nontemporal_store(lam[jj], &a.lam_out[(uint64_t)jj * N + own]); });
  }

  // dJ/ds_k: block sum of z3_k r_k in FP64, added to this block's row
  __shared__ double red[4][Q];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // one row per tile (not per workgroup), so the sums do not depend on the block order
  const uint32_t bid = tile.x + gridDim.x * (tile.y + gridDim.y * tile.z);
  sfor<Q>([&](auto kk) {
    constexpr int K = kk;
    if constexpr (K > D) {
      double c = active ? double(z3[K]) * double(r[K]) : 0.0;
      for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
      if (lane == 0) red[wave][K] = c;
    }
  });
  __syncthreads();
  if (threadIdx.x < Q && (int)threadIdx.x > D) {
    double sum = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) sum += red[w][threadIdx.x];
    a.partial[(uint64_t)bid * Q + threadIdx.x] += sum;
  }
}

// Two reverse steps in one launch (two-dimensional lattices, FP32
// arithmetic): lambda^{n-1} from lambda^{n+1}, f^n and f^{n-1}, with lambda^n
// kept in LDS.  A block owns a tile of kA2X x kA2Y nodes.  It stages
// lambda^{n+1} on the tile and a two-node halo (periodic), computes lambda^n on
// the tile and a one-node ring (the ring is also computed by the neighbouring
// blocks: 29 % more adjoint work per step pair for 64 x 8 tiles), then
// lambda^{n-1} on the tile.  Each node's arithmetic is adjoint_node, as in
// k_adjoint, so lambda^{n-1} and dJ/du~ (added to the FP64 accumulator in the
// same order, step n first) are bit for bit those of two single steps; the
// dJ/ds partial sums go to one row per tile of this grid and differ from the
// single steps only in the order of the FP64 additions.  Small grids are
// bound by the latency and the fixed cost of each launch, which this halves;
// on large grids lambda^n never goes to HBM.
constexpr int kA2X = 64, kA2Y = 8;
constexpr int kA2RX = kA2X + 2, kA2RY = kA2Y + 2;  // ring region: lambda^n
constexpr int kA2HX = kA2X + 4, kA2HY = kA2Y + 4;  // halo region: lambda^{n+1}

__device__ __forceinline__ int wrap_index(int i, int n) {
  int m = i % n;
  return m < 0 ? m + n : m;
}

template <class B, int ST, int MODE, int RLX>
__global__ __launch_bounds__(kA2X* kA2Y) void k_adjoint2(AdjArgs<typename Store<ST>::T> a) {
  using L = typename B::Lat;
  using S = typename Store<ST>::S;
  using T = typename Store<ST>::T;
  constexpr int Q = B::Q;
  constexpr int D = L::D;
  static_assert(D == 2 && sizeof(T) == 4, "the two-step adjoint is for 2-D lattices with FP32 arithmetic");
  constexpr int NT = kA2X * kA2Y;
  __shared__ T lh[Q][kA2HY * kA2HX];  // lambda^{n+1}, halo region
  __shared__ T lr[Q][kA2RY * kA2RX];  // lambda^n, ring region
  __shared__ T gr[D][NT];             // step n's dJ/du~ at the owned nodes (field mode)
  __shared__ double red[NT / 64][Q];

  const uint3 tile = block_tile(a.xcd_remap);
  const int tid = threadIdx.x;
  const int nx = (int)a.nx, ny = (int)a.ny;
  const int x0 = (int)tile.x * kA2X, y0 = (int)tile.y * kA2Y;
  const uint64_t N = a.N;
  const S* fn = static_cast<const S*>(a.f);
  const S* fp = static_cast<const S*>(a.f_prev);

  // lambda^{n+1} on the halo region
  for (int i = tid; i < kA2HY * kA2HX; i += NT) {
    const int ix = i % kA2HX, iy = i / kA2HX;
    const uint64_t node = (uint64_t)wrap_index(y0 - 2 + iy, ny) * nx + wrap_index(x0 - 2 + ix, nx);
    sfor<Q>([&](auto jj) { lh[jj][i] = a.lam_in[(uint64_t)jj * N + node]; });
  }
  __syncthreads();

  double sacc[Q];
  sfor<Q>([&](auto kk) { sacc[kk] = 0.0; });
  // step n on the ring region
  for (int i = tid; i < kA2RY * kA2RX; i += NT) {
    const int ix = i % kA2RX, iy = i / kA2RX;  // tile coordinates ix - 1, iy - 1
    const int gx = wrap_index(x0 - 1 + ix, nx), gy = wrap_index(y0 - 1 + iy, ny);
    const uint64_t node = (uint64_t)gy * nx + gx;
    T h[Q], g[Q], utf[3] = {T(0), T(0), T(0)};
    sfor<Q>([&](auto jj) {
      constexpr int J = jj;
      h[J] = T(fn[(uint64_t)J * N + node]);
      g[J] = lh[J][(iy + 1 + L::c[J].y) * kA2HX + (ix + 1 + L::c[J].x)];
    });
    if constexpr (MODE == UT_FIELD) {
      sfor<D>([&](auto al) { utf[al] = T(a.ut[(uint64_t)al * N + node]) * a.inv_lambda; });
    }
    T lam[Q], gut[3], z3[Q], r[Q];
    adjoint_node<B, ST, MODE, RLX>(a, h, g, utf, lam, gut, z3, r);
    sfor<Q>([&](auto jj) { lr[jj][i] = lam[jj]; });
    const bool owned = ix >= 1 && ix <= kA2X && iy >= 1 && iy <= kA2Y && x0 + ix - 1 < nx && y0 + iy - 1 < ny;
    if (owned) {
      sfor<Q>([&](auto kk) {
        constexpr int K = kk;
        if constexpr (K > D) sacc[K] += double(z3[K]) * double(r[K]);
      });
      if constexpr (MODE == UT_FIELD) {
        sfor<D>([&](auto al) { gr[al][(iy - 1) * kA2X + (ix - 1)] = gut[al]; });
      }
    }
  }
  __syncthreads();

  // step n - 1 on the owned tile
  const int tx = tid % kA2X, ty = tid / kA2X;
  const int x = x0 + tx, y = y0 + ty;
  if (x < nx && y < ny) {
    const uint64_t node = (uint64_t)y * nx + x;
    T h[Q], g[Q], utf[3] = {T(0), T(0), T(0)};
    sfor<Q>([&](auto jj) {
      constexpr int J = jj;
      h[J] = T(__builtin_nontemporal_load(&fp[(uint64_t)J * N + node]));
      g[J] = lr[J][(ty + 1 + L::c[J].y) * kA2RX + (tx + 1 + L::c[J].x)];
    });
    if constexpr (MODE == UT_FIELD) {
      sfor<D>([&](auto al) { utf[al] = T(a.ut[(uint64_t)al * N + node]) * a.inv_lambda; });
    }
    T lam[Q], gut[3], z3[Q], r[Q];
    adjoint_node<B, ST, MODE, RLX>(a, h, g, utf, lam, gut, z3, r);
    sfor<Q>([&](auto jj) { __builtin_nontemporal_store(lam[jj], &a.lam_out[(uint64_t)jj * N + node]); });
    sfor<Q>([&](auto kk) {
      constexpr int K = kk;
      if constexpr (K > D) sacc[K] += double(z3[K]) * double(r[K]);
    });
    if constexpr (MODE == UT_FIELD) {
      sfor<D>([&](auto al) {
        double* gp = &a.grad_ut[(uint64_t)al * N + node];
        double v = *gp;
        v += double(gr[al][tid] * a.inv_lambda);
        v += double(gut[al] * a.inv_lambda);
        *gp = v;
      });
    }
  }

  // dJ/ds_k: block sum, added to this tile's row
  const int lane = tid & 63, wave = tid >> 6;
  sfor<Q>([&](auto kk) {
    constexpr int K = kk;
    if constexpr (K > D) {
      double c = sacc[K];
      for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
      if (lane == 0) red[wave][K] = c;
    }
  });
  __syncthreads();
  if (tid < Q && tid > D) {
    double sum = 0.0;
    for (int w = 0; w < NT / 64; ++w) sum += red[w][tid];
    const uint32_t bid = tile.x + gridDim.x * (tile.y + gridDim.y * tile.z);
    a.partial[(uint64_t)bid * Q + tid] += sum;
  }
}

}  // namespace lbmrv
