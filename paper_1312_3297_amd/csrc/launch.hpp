// Host-side launchers for one (lattice, basis) pair.  Each per-lattice
// translation unit instantiates these once; the C-ABI layer dispatches to them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "adjoint.hpp"
#include "kernels.hpp"

namespace lbmrv {

enum StorageKind { SK_F64 = 0, SK_F32 = 1, SK_F16 = 2 };

struct StepLaunch {
  int sk;      // StorageKind
  int mode;    // Mode
  int kind;    // Kind
  const void* fin;
  void* fout;
  const float* ut;
  uint32_t nx, ny, nz;
  uint64_t N;
  double rho0, alpha, inv_lambda;
  double s[27];
  uint32_t wall_mask;
  double wall_coef[6][3];
  uint32_t eq_maxwell;
  const void* relax;  // run-time basis: R^{-1} S R block in the arithmetic type, or null
  uint32_t xcd_remap; // block order (see block_tile)
  hipStream_t stream;
  int block;   // threads per block along x
};

struct MomLaunch {
  int sk;
  const void* f;
  void* rho;
  void* u;
  void* m0;
  uint64_t N;
  double rho0, lambda;
  const void* rmat;  // run-time basis: R (Q x Q) in the arithmetic type, or null
  hipStream_t stream;
};

// LDS per compute unit on gfx950 (CDNA4), and per-block reservations that let
// at most n blocks share a CU: a multiple of 4 KB between kLdsPerCu / (n + 1)
// and kLdsPerCu / n with room on both sides (53 KB, for three blocks, was
// measured to admit only two: the allocation is coarser than 1 KB)
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr size_t lds_for_blocks(size_t n) {
  return ((kLdsPerCu / n + kLdsPerCu / (n + 1)) / 2) / 4096 * 4096;
}
static_assert(lds_for_blocks(4) == 36 * 1024 && lds_for_blocks(3) == 44 * 1024, "LDS reservations");

template <class B, int ST, int MODE, int KIND, int RLX>
hipError_t launch_step_t(const StepLaunch& L) {
  using T = typename Store<ST>::T;
  StepArgs<T> a{};
  a.fin = L.fin;
  a.fout = L.fout;
  a.ut = L.ut;
  a.nx = L.nx;
  a.ny = L.ny;
  a.nz = L.nz;
  a.N = L.N;
  a.rho0 = T(L.rho0);
  a.alpha = T(L.alpha);
  a.inv_lambda = T(L.inv_lambda);
  for (int k = 0; k < 27; ++k) a.s[k] = T(L.s[k]);
  a.wall_mask = L.wall_mask;
  a.eq_maxwell = L.eq_maxwell;
  a.relax = static_cast<const T*>(L.relax);
  a.xcd_remap = L.xcd_remap;
  for (int f = 0; f < 6; ++f)
    for (int ax = 0; ax < 3; ++ax) a.wall_coef[f][ax] = T(L.wall_coef[f][ax]);
  // D3Q19 with FP16 storage, even in-place step: node pairs (k_aa_even_pair),
  // up to 128 pairs of a row per block and as many rows as fill 256 threads
  if constexpr (ST == 2 && KIND == K_AA_EVEN && B::Q == 19) {
    // whole words: nx even (so N is even and every slot starts on a word) and
    // the arrays 4-byte aligned (the interface asks for 2)
    if (L.nx % 2 == 0 && reinterpret_cast<uintptr_t>(L.fin) % 4 == 0 && reinterpret_cast<uintptr_t>(L.fout) % 4 == 0) {
      const uint32_t npx = L.nx / 2;
      const uint32_t bxp = npx >= 128u ? 128u : npx;
      uint32_t byp = 256u / bxp;
      if (byp > L.ny) byp = L.ny;
      dim3 grid((npx + bxp - 1) / bxp, (L.ny + byp - 1) / byp, L.nz);
      hipLaunchKernelGGL((k_aa_even_pair<B, MODE, RLX>), grid, dim3(bxp, byp), 0, L.stream, a);
      return hipGetLastError();
    }
  }
  // block: whole wavefronts along x, and as many rows as fit in
  // step_max_threads threads.  The gather forms take rows up to that width
  // (1024-wide rows measured 1-2 % faster than 256 on 2048^2 and 4096^2 D2Q9
  // grids); the scatter and in-place forms keep 256.
  // D3Q19 keeps 256-wide rows (four per block in FP32) on wider grids too:
  // at 512^3 that measured 6.9 % faster than 512-wide rows in FP32, 3.9 % in
  // FP64 and the same in FP16.
  constexpr bool wide = KIND == K_PULL || KIND == K_STREAM || KIND == K_COLLIDE;
  const uint32_t bx_max = !wide ? 256u : (B::Q == 19 ? 256u : (uint32_t)step_max_threads<ST, KIND>());
  const uint32_t bx = L.nx >= bx_max ? bx_max : ((L.nx + 63u) / 64u) * 64u;
  // (FP16 storage measured faster with one row per block)
  uint32_t by = (KIND == K_PUSH || KIND == K_AA_ODD || KIND == K_AA_ODD_WALLS || ST == 2)
                    ? 1u
                    : (uint32_t)step_max_threads<ST, KIND>() / bx;
  // D3Q27's step holds ~90 VGPRs, so at most 5 wavefronts per SIMD: one
  // 15-wavefront block of five 192-wide rows per CU leaves slots idle, blocks
  // of two rows pack better (measured +2.6 % at 192^3 FP32; one row and three
  // to five rows were slower, and D3Q19 stays fastest at four rows)
  if (B::Q == 27 && by > 2u) by = 2u;
  // D3Q19 with 4-byte populations, in-place even step (and the pull step on
  // rows wider than one block): one 256-wide row per block and at most four
  // blocks per CU, four wavefronts per SIMD as the odd step runs.  The cap is
  // an LDS reservation the kernel never touches (lds_for_blocks).
  // Same-GPU A/B: in place +1.1 % at 256^3 and +7.9 % at 512^3, pull +11 % at
  // 512^3 (-0.4 % at 256^3, so 256-wide grids keep four-row blocks there);
  // one-row blocks without the cap (seven per CU) lost 0.8 % at 256^3, and
  // FP16, FP64, D3Q27 and D2Q9 gained nothing from either.  The odd step
  // (four wavefronts per SIMD by its registers) runs at most three blocks per
  // CU where a row fits one block: in place +1.2 to +1.4 % at 256^3, odd step
  // 420 -> 406-410 us (two blocks: -2 %; three at 512^3, rows of two blocks:
  // -1.8 %).
  size_t lds_cap = 0;
  if constexpr (B::Q == 19 && ST == 1 && (KIND == K_AA_EVEN || KIND == K_PULL)) {
    if (KIND == K_AA_EVEN || L.nx > bx) {
      by = 1u;
      lds_cap = lds_for_blocks(4);
    }
  }
  if constexpr (B::Q == 19 && ST == 1 && KIND == K_AA_ODD) {
    if (L.nx <= bx) lds_cap = lds_for_blocks(3);
  }
  if (by > L.ny) by = L.ny;
  dim3 grid((L.nx + bx - 1) / bx, (L.ny + by - 1) / by, L.nz);
  hipLaunchKernelGGL((k_step<B, ST, MODE, KIND, RLX>), grid, dim3(bx, by), lds_cap, L.stream, a);
  return hipGetLastError();
}

template <class B, int ST, int MODE>
hipError_t launch_step_m(const StepLaunch& L) {
  if (L.relax) {  // run-time basis: the two-array forms
    switch (L.kind) {
      case K_PULL: return launch_step_t<B, ST, MODE, K_PULL, 1>(L);
      case K_PUSH: return launch_step_t<B, ST, MODE, K_PUSH, 1>(L);
      case K_COLLIDE: return launch_step_t<B, ST, MODE, K_COLLIDE, 1>(L);
      case K_STREAM: return launch_step_t<B, ST, UT_ZERO, K_STREAM, 0>(L);
    }
    return hipErrorInvalidValue;
  }
  switch (L.kind) {
    case K_PULL: return launch_step_t<B, ST, MODE, K_PULL, 0>(L);
    case K_PUSH: return launch_step_t<B, ST, MODE, K_PUSH, 0>(L);
    case K_COLLIDE: return launch_step_t<B, ST, MODE, K_COLLIDE, 0>(L);
    case K_STREAM: return launch_step_t<B, ST, UT_ZERO, K_STREAM, 0>(L);
    case K_AA_EVEN: return launch_step_t<B, ST, MODE, K_AA_EVEN, 0>(L);
    case K_AA_ODD: return launch_step_t<B, ST, MODE, K_AA_ODD, 0>(L);
    case K_AA_ODD_WALLS: return launch_step_t<B, ST, MODE, K_AA_ODD_WALLS, 0>(L);
  }
  return hipErrorInvalidValue;
}

template <class B, int ST>
hipError_t launch_aa_finish_t(void* f, uint32_t nx, uint32_t ny, uint32_t nz, uint64_t N, const FinArgs& w,
                              hipStream_t st) {
  const uint32_t bx = nx >= 256 ? 256u : ((nx + 63u) / 64u) * 64u;
  hipLaunchKernelGGL((k_aa_finish<B, ST>), dim3((nx + bx - 1) / bx, ny, nz), dim3(bx), 0, st, f, nx, ny, nz, N, w);
  return hipGetLastError();
}

template <class B, int ST>
hipError_t launch_step_s(const StepLaunch& L) {
  switch (L.mode) {
    case UT_ZERO: return launch_step_m<B, ST, UT_ZERO>(L);
    case UT_FLUID: return launch_step_m<B, ST, UT_FLUID>(L);
    case UT_FIELD: return launch_step_m<B, ST, UT_FIELD>(L);
  }
  return hipErrorInvalidValue;
}

template <class B, int ST>
hipError_t launch_moments_t(const MomLaunch& L) {
  using T = typename Store<ST>::T;
  MomArgs<T> a{};
  a.f = L.f;
  a.rho = L.rho;
  a.u = L.u;
  a.m0 = L.m0;
  a.N = L.N;
  a.rho0 = T(L.rho0);
  a.lambda = T(L.lambda);
  a.rmat = static_cast<const T*>(L.rmat);
  const unsigned grid = (unsigned)((L.N + 255) / 256);
  hipLaunchKernelGGL((k_moments<B, ST>), dim3(grid), dim3(256), 0, L.stream, a);
  return hipGetLastError();
}

template <class B, int ST>
hipError_t launch_conserve_partial(const void* f, uint64_t N, double* partial, hipStream_t st) {
  hipLaunchKernelGGL((k_conserve_partial<B, ST>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, f, N, partial);
  return hipGetLastError();
}

template <class B, int ST>
hipError_t launch_devnorm_t(const void* f, uint64_t N, const DevRef& ref, double* partial, hipStream_t st) {
  hipLaunchKernelGGL((k_dev_partial<B, ST>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, f, N, ref, partial);
  return hipGetLastError();
}

template <class B, int ST>
hipError_t launch_devscale_t(void* f, uint64_t N, const DevRef& ref, double factor, hipStream_t st) {
  hipLaunchKernelGGL((k_dev_scale<B, ST>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, f, N, ref, factor);
  return hipGetLastError();
}

struct InitLaunch {
  const double* rho;
  const double* u;
  const double* noise;
  double amp, rho0, lambda;
  uint64_t N;
  void* fout;
  hipStream_t stream;
};

template <class B, int ST>
hipError_t launch_init_t(const InitLaunch& L) {
  const unsigned grid = (unsigned)((L.N + 255) / 256);
  hipLaunchKernelGGL((k_init_eq<B, ST>), dim3(grid), dim3(256), 0, L.stream, L.rho, L.u, L.noise, L.amp, L.rho0, L.lambda,
                     L.N, L.fout);
  return hipGetLastError();
}

template <class B, int ST>
hipError_t launch_convert_t(const void* in, void* out, double rho0, uint64_t N, int to_storage, hipStream_t st) {
  const unsigned grid = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL((k_convert<B, ST>), dim3(grid), dim3(256), 0, st, in, out, rho0, N, to_storage);
  return hipGetLastError();
}

struct AdjLaunch {
  int mode;  // UT_ZERO, UT_FLUID or UT_FIELD
  const void* f;
  const void* f_prev;  // two-step kernel only: f^{n-1} (f is f^n)
  const void* lam_in;
  void* lam_out;
  const float* ut;
  double* grad_ut;
  double* partial;
  uint32_t nx, ny, nz;
  uint64_t N;
  double rho0, inv_lambda, alpha;
  double s[27];
  const void* rnn;     // run-time basis: non-conserved block of R and its inverse, or null
  const void* rnninv;
  uint32_t xcd_remap;
  uint32_t eq_maxwell;
  hipStream_t stream;
  int block;
};

template <class B, int ST, int MODE, int RLX>
hipError_t launch_adjoint_t(const AdjLaunch& L) {
  using T = typename Store<ST>::T;
  AdjArgs<T> a{};
  a.f = L.f;
  a.lam_in = static_cast<const T*>(L.lam_in);
  a.lam_out = static_cast<T*>(L.lam_out);
  a.ut = L.ut;
  a.grad_ut = L.grad_ut;
  a.partial = L.partial;
  a.nx = L.nx;
  a.ny = L.ny;
  a.nz = L.nz;
  a.N = L.N;
  a.rho0 = T(L.rho0);
  a.inv_lambda = T(L.inv_lambda);
  a.alpha = T(L.alpha);
  for (int k = 0; k < 27; ++k) a.s[k] = T(L.s[k]);
  a.f_prev = L.f_prev;
  a.rnn = static_cast<const T*>(L.rnn);
  a.rnninv = static_cast<const T*>(L.rnninv);
  a.xcd_remap = L.xcd_remap;
  a.eq_maxwell = L.eq_maxwell;
  const int bx = L.block;
  dim3 grid((L.nx + bx - 1) / bx, L.ny, L.nz);
  hipLaunchKernelGGL((k_adjoint<B, ST, MODE, RLX>), grid, dim3(bx), 0, L.stream, a);
  return hipGetLastError();
}

template <class B, int ST, int RLX>
hipError_t launch_adjoint_r(const AdjLaunch& L) {
  if (L.mode == UT_ZERO) return launch_adjoint_t<B, ST, UT_ZERO, RLX>(L);
  if (L.mode == UT_FLUID) return launch_adjoint_t<B, ST, UT_FLUID, RLX>(L);
  if (L.mode == UT_FIELD) return launch_adjoint_t<B, ST, UT_FIELD, RLX>(L);
  return hipErrorInvalidValue;
}

template <class B, int ST>
hipError_t launch_adjoint_s(const AdjLaunch& L) {
  return L.rnn ? launch_adjoint_r<B, ST, 1>(L) : launch_adjoint_r<B, ST, 0>(L);
}

// Two reverse steps per launch (k_adjoint2): two-dimensional lattices with
// FP32 arithmetic only; blocks of kA2X x kA2Y nodes.
template <class B, int ST, int MODE, int RLX>
hipError_t launch_adjoint2_t(const AdjLaunch& L) {
  using T = typename Store<ST>::T;
  AdjArgs<T> a{};
  a.f = L.f;
  a.f_prev = L.f_prev;
  a.lam_in = static_cast<const T*>(L.lam_in);
  a.lam_out = static_cast<T*>(L.lam_out);
  a.ut = L.ut;
  a.grad_ut = L.grad_ut;
  a.partial = L.partial;
  a.nx = L.nx;
  a.ny = L.ny;
  a.nz = L.nz;
  a.N = L.N;
  a.rho0 = T(L.rho0);
  a.inv_lambda = T(L.inv_lambda);
  a.alpha = T(L.alpha);
  for (int k = 0; k < 27; ++k) a.s[k] = T(L.s[k]);
  a.rnn = static_cast<const T*>(L.rnn);
  a.rnninv = static_cast<const T*>(L.rnninv);
  a.xcd_remap = L.xcd_remap;
  a.eq_maxwell = L.eq_maxwell;
  dim3 grid((L.nx + kA2X - 1) / kA2X, (L.ny + kA2Y - 1) / kA2Y, 1);
  hipLaunchKernelGGL((k_adjoint2<B, ST, MODE, RLX>), grid, dim3(kA2X * kA2Y), 0, L.stream, a);
  return hipGetLastError();
}

template <class B, int ST, int RLX>
hipError_t launch_adjoint2_r(const AdjLaunch& L) {
  if (L.mode == UT_ZERO) return launch_adjoint2_t<B, ST, UT_ZERO, RLX>(L);
  if (L.mode == UT_FLUID) return launch_adjoint2_t<B, ST, UT_FLUID, RLX>(L);
  if (L.mode == UT_FIELD) return launch_adjoint2_t<B, ST, UT_FIELD, RLX>(L);
  return hipErrorInvalidValue;
}

template <class B, int ST>
hipError_t launch_adjoint2_s(const AdjLaunch& L) {
  if constexpr (B::Lat::D == 2 && ST != 0) {
    return L.rnn ? launch_adjoint2_r<B, ST, 1>(L) : launch_adjoint2_r<B, ST, 0>(L);
  } else {
    (void)L;
    return hipErrorInvalidValue;
  }
}

// Whether a lattice and storage have the two-step reverse kernel.
constexpr bool has_adjoint2(int d, int sk) { return d == 2 && sk != SK_F64; }

// Per-(lattice, basis, storage) entry points, defined in the lattice translation
// units (one unit per lattice and storage type, so they compile in parallel).
#define LBMRV_DECLARE_LAUNCHERS(NAME, SKN)                                                  \
  hipError_t launch_step_##NAME##_##SKN(const StepLaunch& L);                               \
  hipError_t launch_moments_##NAME##_##SKN(const MomLaunch& L);                             \
  hipError_t launch_conserve_##NAME##_##SKN(const void* f, uint64_t N, double* partial,     \
                                            hipStream_t st);                                \
  hipError_t launch_init_##NAME##_##SKN(const InitLaunch& L);                               \
  hipError_t launch_adjoint_##NAME##_##SKN(const AdjLaunch& L);                             \
  hipError_t launch_adjoint2_##NAME##_##SKN(const AdjLaunch& L);                            \
  hipError_t launch_aa_finish_##NAME##_##SKN(void* f, uint32_t nx, uint32_t ny, uint32_t nz, uint64_t N, \
                                             const FinArgs& w, hipStream_t st);              \
  hipError_t launch_convert_##NAME##_##SKN(const void* in, void* out, double rho0, uint64_t N, \
                                           int to_storage, hipStream_t st);                  \
  hipError_t launch_devnorm_##NAME##_##SKN(const void* f, uint64_t N, const DevRef& ref,    \
                                           double* partial, hipStream_t st);                \
  hipError_t launch_devscale_##NAME##_##SKN(void* f, uint64_t N, const DevRef& ref, double factor, \
                                            hipStream_t st);

#define LBMRV_DEFINE_LAUNCHERS(NAME, BASIS, SKN, ST)                                        \
  hipError_t launch_step_##NAME##_##SKN(const StepLaunch& L) { return launch_step_s<BASIS, ST>(L); } \
  hipError_t launch_moments_##NAME##_##SKN(const MomLaunch& L) {                            \
    return launch_moments_t<BASIS, ST>(L);                                                  \
  }                                                                                         \
  hipError_t launch_conserve_##NAME##_##SKN(const void* f, uint64_t N, double* partial,     \
                                            hipStream_t st) {                               \
    return launch_conserve_partial<BASIS, ST>(f, N, partial, st);                           \
  }                                                                                         \
  hipError_t launch_init_##NAME##_##SKN(const InitLaunch& L) { return launch_init_t<BASIS, ST>(L); } \
  hipError_t launch_adjoint_##NAME##_##SKN(const AdjLaunch& L) { return launch_adjoint_s<BASIS, ST>(L); } \
  hipError_t launch_adjoint2_##NAME##_##SKN(const AdjLaunch& L) { return launch_adjoint2_s<BASIS, ST>(L); } \
  hipError_t launch_aa_finish_##NAME##_##SKN(void* f, uint32_t nx, uint32_t ny, uint32_t nz, uint64_t N, \
                                             const FinArgs& w, hipStream_t st) {             \
    return launch_aa_finish_t<BASIS, ST>(f, nx, ny, nz, N, w, st);                          \
  }                                                                                         \
  hipError_t launch_convert_##NAME##_##SKN(const void* in, void* out, double rho0, uint64_t N, \
                                           int to_storage, hipStream_t st) {               \
    return launch_convert_t<BASIS, ST>(in, out, rho0, N, to_storage, st);                   \
  }                                                                                         \
  hipError_t launch_devnorm_##NAME##_##SKN(const void* f, uint64_t N, const DevRef& ref,    \
                                           double* partial, hipStream_t st) {               \
    return launch_devnorm_t<BASIS, ST>(f, N, ref, partial, st);                             \
  }                                                                                         \
  hipError_t launch_devscale_##NAME##_##SKN(void* f, uint64_t N, const DevRef& ref, double factor, \
                                            hipStream_t st) {                               \
    return launch_devscale_t<BASIS, ST>(f, N, ref, factor, st);                             \
  }

#define LBMRV_DECLARE_ALL(NAME) \
  LBMRV_DECLARE_LAUNCHERS(NAME, f64) LBMRV_DECLARE_LAUNCHERS(NAME, f32) LBMRV_DECLARE_LAUNCHERS(NAME, f16)

LBMRV_DECLARE_ALL(d2q9_paper)
LBMRV_DECLARE_ALL(d2q9_geier)
LBMRV_DECLARE_ALL(d3q19)
LBMRV_DECLARE_ALL(d3q27)

}  // namespace lbmrv
