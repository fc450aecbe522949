// a2a_reduce.h -- deterministic per-slot global reductions in FP64 and the BiCGStab and
// CGNR scalar updates that consume them.
//
// A reducing kernel block works on one site block of one or more slots (right-hand sides).
// It reduces its per-thread FP64 values with a fixed shuffle tree and stores the block
// partial to partials[slot][block] with plain stores.  A separate finalize launch (one
// block per slot, ordered after the kernel on the same stream, so no fences or atomics
// are needed across the per-XCD L2 caches) sums the partials in block order and applies
// the scalar update.  Results are bitwise reproducible and independent of what else
// shares the launch.
#pragma once

#include "a2a_device.h"

namespace a2a {

enum RedKind {
  RED_NONE = 0,
  RED_ALPHA,   // v = (rhat, v)            -> alpha = rho / v
  RED_OMEGA,   // v = (t, s), |t|^2        -> omega
  RED_RHO,     // v = (rhat, r), |r|^2     -> beta, rho
  RED_INIT,    // v = (rhat, r), |r|^2     -> fresh BiCGStab state
  RED_RU,      // v = (rhat, r), |r|^2     -> state after a reliable update
  RED_R64,     // v = |r64|^2
  RED_ETA,     // v = |eta|^2
  RED_RES_E,   // v = |r_e|^2
  RED_RES_O,   // v = |r_o|^2
  RED_NORM,    // v = |out|^2 into SC_TMP
  // CG on the normal equations; gamma = |z|^2 of z = M^dag r lives in SC_RHO (real)
  RED_CG_ALPHA,  // v[2] = |q|^2, q = M p          -> alpha = gamma / |q|^2
  RED_CG_R,      // v[2] = |r|^2                   -> iterated residual norm
  RED_CG_BETA,   // v[2] = |M gamma5 r|^2 = |z'|^2 -> beta = |z'|^2 / gamma, gamma = |z'|^2
  RED_CG_INIT,   // v[2] = |r|^2                   -> fresh CGNR state (beta = 0 next)
  RED_CG_RU,     // v[2] = |r|^2                   -> state after a reliable update
};

constexpr int RED_NV = 3;  // values stored per block partial

struct RedBuf {
  double* partials;  // [slot id][maxblk][RED_NV]
  int maxblk;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sums of N values per thread (BS threads).  On return thread k < N holds the
// block total of value k in v[k] (other entries unspecified).
template <int N, int BS>
__device__ __forceinline__ void block_sum_n(double (&v)[N]) {
  __shared__ double lds[N * (BS / 64)];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) lds[k * (BS / 64) + w] = v[k];
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < BS / 64; ++j) s += lds[threadIdx.x * (BS / 64) + j];
#pragma unroll
    for (int k = 0; k < N; ++k)
      if (k == (int)threadIdx.x) v[k] = s;
  }
}

// Block-wide sums of N values per thread; thread 0 receives all N totals in v.
template <int N, int BS>
__device__ __forceinline__ void block_sum_all(double (&v)[N]) {
  __shared__ double lds[N * (BS / 64)];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) lds[k * (BS / 64) + w] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = 0.0;
      for (int j = 0; j < BS / 64; ++j) s += lds[k * (BS / 64) + j];
      v[k] = s;
    }
}

// store the block partial of value k (thread k) for slot `sid`, block `blk`
__device__ __forceinline__ void store_partial(const RedBuf& rb, int sid, int blk, int k, double val) {
  rb.partials[((size_t)sid * rb.maxblk + blk) * RED_NV + k] = val;
}

__device__ __forceinline__ void cdiv(double ar, double ai, double br, double bi, double& cr, double& ci) {
  double d = br * br + bi * bi;
  cr = (ar * br + ai * bi) / d;
  ci = (ai * br - ar * bi) / d;
}
__device__ __forceinline__ void cmul(double ar, double ai, double br, double bi, double& cr, double& ci) {
  cr = ar * br - ai * bi;
  ci = ar * bi + ai * br;
}

// New inner-vector scale at a reliable update.  The residual is brought back to unit RMS
// per component, but the scale may shrink by at most RU_MAX_RATIO per update: the search
// directions p, v are carried over multiplied by sigma_old / sigma_new, and an unbounded
// ratio (after a fast drop of the residual) would push FP16 intermediates past 65504.
constexpr double RU_MAX_RATIO = 16.0;
__host__ __device__ inline double ru_scale(double r64n2, double sigma_old, int hv) {
  const double s = sqrt(r64n2 / (12.0 * hv));
  return fmax(s, sigma_old / RU_MAX_RATIO);
}

// scalar update for one slot from the fully reduced values v[]; hv = sites per parity
__device__ inline void finalize_slot(int kind, double* sc, const double* v, int hv) {
  switch (kind) {
    case RED_ALPHA: {
      double ar, ai;
      if (v[0] == 0.0 && v[1] == 0.0) {
        sc[SC_FLAGS] = 1.0;
        ar = ai = 0.0;
      } else {
        cdiv(sc[SC_RHO], sc[SC_RHO + 1], v[0], v[1], ar, ai);
      }
      sc[SC_ALPHA] = ar;
      sc[SC_ALPHA + 1] = ai;
    } break;
    case RED_OMEGA: {
      if (v[2] == 0.0) {
        sc[SC_FLAGS] = 2.0;
        sc[SC_OMEGA] = 0.0;
        sc[SC_OMEGA + 1] = 0.0;
      } else {
        sc[SC_OMEGA] = v[0] / v[2];
        sc[SC_OMEGA + 1] = v[1] / v[2];
      }
    } break;
    case RED_RHO: {
      double qr, qi, ar, ai, br, bi;
      if ((sc[SC_RHO] == 0.0 && sc[SC_RHO + 1] == 0.0) || (sc[SC_OMEGA] == 0.0 && sc[SC_OMEGA + 1] == 0.0)) {
        sc[SC_FLAGS] = 3.0;
        br = bi = 0.0;
      } else {
        cdiv(v[0], v[1], sc[SC_RHO], sc[SC_RHO + 1], qr, qi);
        cdiv(sc[SC_ALPHA], sc[SC_ALPHA + 1], sc[SC_OMEGA], sc[SC_OMEGA + 1], ar, ai);
        cmul(qr, qi, ar, ai, br, bi);
      }
      sc[SC_BETA] = br;
      sc[SC_BETA + 1] = bi;
      sc[SC_RHOPREV] = sc[SC_RHO];
      sc[SC_RHOPREV + 1] = sc[SC_RHO + 1];
      sc[SC_RHO] = v[0];
      sc[SC_RHO + 1] = v[1];
      sc[SC_RNORM2] = v[2];
    } break;
    case RED_INIT: {
      sc[SC_RHO] = v[0];
      sc[SC_RHO + 1] = v[1];
      sc[SC_RHOPREV] = v[0];
      sc[SC_RHOPREV + 1] = v[1];
      sc[SC_ALPHA] = 1.0;
      sc[SC_ALPHA + 1] = 0.0;
      sc[SC_OMEGA] = 1.0;
      sc[SC_OMEGA + 1] = 0.0;
      sc[SC_BETA] = 0.0;
      sc[SC_BETA + 1] = 0.0;
      sc[SC_RNORM2] = v[2];
      sc[SC_SIGMA] = sqrt(sc[SC_R64N2] / (12.0 * hv));
      sc[SC_FLAGS] = 0.0;
    } break;
    case RED_RU: {
      double snew = ru_scale(sc[SC_R64N2], sc[SC_SIGMA], hv);
      double ratio = sc[SC_SIGMA] / snew;  // old units -> new units
      double pr = sc[SC_RHOPREV] * ratio, pi = sc[SC_RHOPREV + 1] * ratio;
      double qr, qi, ar, ai, br, bi;
      if (pr == 0.0 && pi == 0.0) {
        br = bi = 0.0;
      } else {
        cdiv(v[0], v[1], pr, pi, qr, qi);
        cdiv(sc[SC_ALPHA], sc[SC_ALPHA + 1], sc[SC_OMEGA], sc[SC_OMEGA + 1], ar, ai);
        cmul(qr, qi, ar, ai, br, bi);
      }
      sc[SC_BETA] = br;
      sc[SC_BETA + 1] = bi;
      sc[SC_RHO] = v[0];
      sc[SC_RHO + 1] = v[1];
      sc[SC_RNORM2] = v[2];
      sc[SC_SIGMA] = snew;
    } break;
    case RED_CG_ALPHA: {
      if (v[2] == 0.0) {
        sc[SC_FLAGS] = 1.0;
        sc[SC_ALPHA] = 0.0;
      } else {
        sc[SC_ALPHA] = sc[SC_RHO] / v[2];
      }
      sc[SC_ALPHA + 1] = 0.0;
    } break;
    case RED_CG_R: sc[SC_RNORM2] = v[2]; break;
    case RED_CG_BETA: {  // gamma == 0 marks a fresh start: p = z
      sc[SC_BETA] = sc[SC_RHO] == 0.0 ? 0.0 : v[2] / sc[SC_RHO];
      sc[SC_BETA + 1] = 0.0;
      sc[SC_RHO] = v[2];
      sc[SC_RHO + 1] = 0.0;
    } break;
    case RED_CG_INIT: {
      sc[SC_RHO] = sc[SC_RHO + 1] = 0.0;
      sc[SC_ALPHA] = sc[SC_ALPHA + 1] = 0.0;
      sc[SC_BETA] = sc[SC_BETA + 1] = 0.0;
      sc[SC_RNORM2] = v[2];
      sc[SC_SIGMA] = sqrt(sc[SC_R64N2] / (12.0 * hv));
      sc[SC_FLAGS] = 0.0;
    } break;
    case RED_CG_RU: {  // z and p carry over in the new units: gamma scales with the ratio squared
      double snew = ru_scale(sc[SC_R64N2], sc[SC_SIGMA], hv);
      double ratio = sc[SC_SIGMA] / snew;
      sc[SC_RHO] *= ratio * ratio;
      sc[SC_RNORM2] = v[2];
      sc[SC_SIGMA] = snew;
    } break;
    case RED_R64: sc[SC_R64N2] = v[0]; break;
    case RED_ETA: sc[SC_ETAN2] = v[0]; break;
    case RED_RES_E: sc[SC_RES_E] = v[0]; break;
    case RED_RES_O: sc[SC_RES_O] = v[0]; break;
    case RED_NORM: sc[SC_TMP] = v[0]; break;
    default: break;
  }
}

}  // namespace a2a
