// a2a_reduce.h -- deterministic per-slot global reductions in FP64 and the BiCGStab scalar
// updates that consume them.
//
// Every block of a reducing kernel works on one slot (right-hand side) and one block of
// sites.  It reduces its per-thread FP64 values with a fixed shuffle tree, writes the block
// partial to partials[slot][block], and counts itself in on the slot's counter.  The block
// that arrives last sums the partials in block order (fixed, independent of scheduling),
// applies the scalar update for that slot and re-arms the counter.  Results are therefore
// bitwise reproducible run to run and independent of what else shares the launch.
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
};

HD int red_nv(int kind) {
  switch (kind) {
    case RED_NONE: return 0;
    case RED_ALPHA: return 2;
    case RED_OMEGA: case RED_RHO: case RED_INIT: case RED_RU: return 3;
    default: return 1;
  }
}

struct RedBuf {
  double* partials;    // [slot][maxblk][4]
  unsigned* counters;  // [slot]
  int maxblk;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum of NV values per thread for BS threads; result valid on thread 0
template <int NV, int BS>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* NV * BS/64 */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k * (BS / 64) + w] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0;
      for (int j = 0; j < BS / 64; ++j) s += lds[k * (BS / 64) + j];
      v[k] = s;
    }
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
      double snew = sqrt(sc[SC_R64N2] / (12.0 * hv));
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
    case RED_R64: sc[SC_R64N2] = v[0]; break;
    case RED_ETA: sc[SC_ETAN2] = v[0]; break;
    case RED_RES_E: sc[SC_RES_E] = v[0]; break;
    case RED_RES_O: sc[SC_RES_O] = v[0]; break;
    case RED_NORM: sc[SC_TMP] = v[0]; break;
    default: break;
  }
}

// Block-level epilogue of a reducing kernel: v[] holds this thread's contribution for one
// slot.  Must be called by every thread of the block (BS threads).
template <int NV, int BS>
__device__ inline void reduce_slot(double (&v)[NV], int kind, int slot /* stable id */, int blk, int nblk,
                                   double* scal, int hv, const RedBuf& rb) {
  __shared__ double lds[4 * (BS / 64)];
  __shared__ int is_last;
  block_sum<NV, BS>(v, lds);
  if (threadIdx.x == 0) {
    double* p = rb.partials + ((size_t)slot * rb.maxblk + blk) * 4;
#pragma unroll
    for (int k = 0; k < NV; ++k) p[k] = v[k];
    __threadfence();
    unsigned prev = atomicAdd(rb.counters + slot, 1u);
    is_last = (prev == (unsigned)(nblk - 1));
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const volatile double* p = rb.partials + (size_t)slot * rb.maxblk * 4;
  for (int b = threadIdx.x; b < nblk; b += BS)
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] += p[(size_t)b * 4 + k];
  block_sum<NV, BS>(acc, lds);
  if (threadIdx.x == 0) {
    finalize_slot(kind, scal, acc, hv);
    rb.counters[slot] = 0u;
    __threadfence();
  }
}

}  // namespace a2a
