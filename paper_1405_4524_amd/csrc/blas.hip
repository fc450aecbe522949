// blas.hip -- BiCGStab vector updates with fused FP64 reductions, the reliable-update
// (mixed-precision defect correction) kernels and site-local clover application.
//
// All kernels run over per-slot tiles {slot, site block}; one thread owns one site of one
// slot.  Inner vectors live in the slot's working-precision arena, FP64 vectors in its
// FP64 arena; the inner vectors carry a per-slot scale sigma (inner = true / sigma) so
// that FP16 storage stays well inside its normal range whatever the residual norm.
#include "a2a_kernels.h"

namespace a2a {

template <typename A>
__device__ __forceinline__ cx<A> scal_c(const double* sc, int k) {
  return mk((A)sc[k], (A)sc[k + 1]);
}

template <class P>
__global__ __launch_bounds__(BS) void k_vec(VecArgs a) {
  using S = typename P::S;
  using A = typename P::A;
  const int2 tile = a.tiles[blockIdx.x];
  const int slot = tile.x;
  const SlotDev& sd = a.slots[slot];
  const OpDev& op = a.ops[sd.op];
  const int hv = op.g.hv;
  const int site = tile.y * BS + (int)threadIdx.x;
  const bool valid = site < hv;
  char* lo = sd.arena[0];
  char* hi = sd.arena[1];
  const long long vl = sd.vstride[0], vh = sd.vstride[1];
  double* sc = sd.scal;
#define LO(v) (lo + (size_t)(v) * vl)
#define HI(v) (hi + (size_t)(v) * vh)

  switch (a.kind) {
    case VK_BICG_S: {  // s = r - alpha v
      if (!valid) return;
      const cx<A> al = scal_c<A>(sc, SC_ALPHA);
      Spinor<A> r, v;
      load_spinor<S, A>(LO(VL_R), hv, site, r);
      load_spinor<S, A>(LO(VL_V), hv, site, v);
#pragma unroll
      for (int k = 0; k < 12; ++k) r.v[k] = r.v[k] - al * v.v[k];
      store_spinor<S, A>(LO(VL_S), hv, site, r);
    } break;
    case VK_BICG_P: {  // p = r + beta (p - omega v)
      if (!valid) return;
      const cx<A> be = scal_c<A>(sc, SC_BETA), om = scal_c<A>(sc, SC_OMEGA);
      Spinor<A> r, p, v;
      load_spinor<S, A>(LO(VL_R), hv, site, r);
      load_spinor<S, A>(LO(VL_P), hv, site, p);
      load_spinor<S, A>(LO(VL_V), hv, site, v);
#pragma unroll
      for (int k = 0; k < 12; ++k) p.v[k] = r.v[k] + be * (p.v[k] - om * v.v[k]);
      store_spinor<S, A>(LO(VL_P), hv, site, p);
    } break;
    case VK_BICG_XR: {  // x += alpha p + omega s; r = s - omega t; (rhat, r), |r|^2
      double v3[3] = {0.0, 0.0, 0.0};
      if (valid) {
        const cx<A> al = scal_c<A>(sc, SC_ALPHA), om = scal_c<A>(sc, SC_OMEGA);
        Spinor<A> x, p, s, t;
        load_spinor<S, A>(LO(VL_X), hv, site, x);
        load_spinor<S, A>(LO(VL_P), hv, site, p);
        load_spinor<S, A>(LO(VL_S), hv, site, s);
        load_spinor<S, A>(LO(VL_T), hv, site, t);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          x.v[k] = x.v[k] + al * p.v[k] + om * s.v[k];
          s.v[k] = s.v[k] - om * t.v[k];
        }
        store_spinor<S, A>(LO(VL_X), hv, site, x);
        store_spinor<S, A>(LO(VL_R), hv, site, s);
        load_spinor<S, A>(LO(VL_R), hv, site, s);  // reduce the stored values
        Spinor<A> rh;
        load_spinor<S, A>(LO(VL_RHAT), hv, site, rh);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          v3[0] += (double)rh.v[k].re * s.v[k].re + (double)rh.v[k].im * s.v[k].im;
          v3[1] += (double)rh.v[k].re * s.v[k].im - (double)rh.v[k].im * s.v[k].re;
          v3[2] += (double)s.v[k].re * s.v[k].re + (double)s.v[k].im * s.v[k].im;
        }
      }
      reduce_slot<3, BS>(v3, RED_RHO, sd.sid, tile.y, sd.nblk, sc, hv, a.rb);
    } break;
    case VK_RU_ACCUM: {  // x64 += sigma x_lo; x_lo = 0
      if (!valid) return;
      const double sg = sc[SC_SIGMA];
      Spinor<A> xl;
      Spinor<double> xh;
      load_spinor<S, A>(LO(VL_X), hv, site, xl);
      load_spinor<double, double>(HI(VH_X), hv, site, xh);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        xh.v[k].re += sg * (double)xl.v[k].re;
        xh.v[k].im += sg * (double)xl.v[k].im;
        xl.v[k] = mk((A)0, (A)0);
      }
      store_spinor<double, double>(HI(VH_X), hv, site, xh);
      store_spinor<S, A>(LO(VL_X), hv, site, xl);
    } break;
    case VK_RU_RESCALE:
    case VK_INIT: {
      double v3[3] = {0.0, 0.0, 0.0};
      const double snew = sqrt(sc[SC_R64N2] / (12.0 * hv));
      const double inv = (snew > 0.0) ? 1.0 / snew : 0.0;
      if (valid) {
        Spinor<double> rh64;
        load_spinor<double, double>(HI(VH_R), hv, site, rh64);
        Spinor<A> r;
#pragma unroll
        for (int k = 0; k < 12; ++k) r.v[k] = mk((A)(rh64.v[k].re * inv), (A)(rh64.v[k].im * inv));
        store_spinor<S, A>(LO(VL_R), hv, site, r);
        load_spinor<S, A>(LO(VL_R), hv, site, r);
        Spinor<A> rh;
        if (a.kind == VK_INIT) {
          Spinor<A> z;
#pragma unroll
          for (int k = 0; k < 12; ++k) z.v[k] = mk((A)0, (A)0);
          store_spinor<S, A>(LO(VL_RHAT), hv, site, r);
          store_spinor<S, A>(LO(VL_P), hv, site, r);
          store_spinor<S, A>(LO(VL_V), hv, site, z);
          store_spinor<S, A>(LO(VL_X), hv, site, z);
          rh = r;
        } else {
          const A ratio = (A)(sc[SC_SIGMA] * inv);
          Spinor<A> p, v;
          load_spinor<S, A>(LO(VL_P), hv, site, p);
          load_spinor<S, A>(LO(VL_V), hv, site, v);
#pragma unroll
          for (int k = 0; k < 12; ++k) {
            p.v[k] = ratio * p.v[k];
            v.v[k] = ratio * v.v[k];
          }
          store_spinor<S, A>(LO(VL_P), hv, site, p);
          store_spinor<S, A>(LO(VL_V), hv, site, v);
          load_spinor<S, A>(LO(VL_RHAT), hv, site, rh);
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          v3[0] += (double)rh.v[k].re * r.v[k].re + (double)rh.v[k].im * r.v[k].im;
          v3[1] += (double)rh.v[k].re * r.v[k].im - (double)rh.v[k].im * r.v[k].re;
          v3[2] += (double)r.v[k].re * r.v[k].re + (double)r.v[k].im * r.v[k].im;
        }
      }
      reduce_slot<3, BS>(v3, a.kind == VK_INIT ? RED_INIT : RED_RU, sd.sid, tile.y, sd.nblk, sc, hv, a.rb);
    } break;
    case VK_CLOVER: {  // FP64: hi[vout] = C hi[vin], C = A or A^{-1} of parity par
      if (!valid) return;
      const void* C = a.use_inv ? op.Ai[1][a.par] : op.A[1][a.par];
      Spinor<double> in, out;
      load_spinor<double, double>(HI(a.vin), hv, site, in);
      clover_apply_mem<double, double>(C, hv, site, in, out);
      store_spinor<double, double>(HI(a.vout), hv, site, out);
    } break;
    case VK_ZERO_HI: {
      if (!valid) return;
      Spinor<double> z;
#pragma unroll
      for (int k = 0; k < 12; ++k) z.v[k] = mk(0.0, 0.0);
      store_spinor<double, double>(HI(a.vout), hv, site, z);
    } break;
    case VK_ZERO_LO:
    case VK_FILL_LO: {
      if (!valid) return;
      Spinor<A> z;
      uint32_t h = (uint32_t)site * 2654435761u + (uint32_t)sd.sid * 40503u + 12345u;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        if (a.kind == VK_ZERO_LO) {
          z.v[k] = mk((A)0, (A)0);
        } else {
          h = h * 1664525u + 1013904223u;
          A re = (A)((double)(h >> 8) * (1.0 / 16777216.0) - 0.5);
          h = h * 1664525u + 1013904223u;
          A im = (A)((double)(h >> 8) * (1.0 / 16777216.0) - 0.5);
          z.v[k] = mk(re, im);
        }
      }
      store_spinor<S, A>(LO(a.vout), hv, site, z);
    } break;
    default: break;
  }
#undef LO
#undef HI
}

void launch_vec(int prec, const VecArgs& a, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return;
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_vec<PrecF64>, dim3(ntiles), dim3(BS), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_vec<PrecF32>, dim3(ntiles), dim3(BS), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_vec<PrecF16>, dim3(ntiles), dim3(BS), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_vec<PrecB16>, dim3(ntiles), dim3(BS), 0, s, a); break;
    default: break;
  }
}

// ------------------------------------------------------------------------------------
// canonical <-> even-odd layout (per slot), optional gamma_5, optional |in|^2
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BS) void k_layout_in(LayoutArgs a) {
  using S = typename P::S;
  using A = typename P::A;
  const int2 tile = a.tiles[blockIdx.x];
  const int slot = tile.x;
  const SlotDev& sd = a.slots[slot];
  const Geo g = a.ops[sd.op].g;
  const int hv = g.hv;
  const int site = tile.y * BS + (int)threadIdx.x;
  double nn = 0.0;
  if (site < hv) {
    const double* src = a.which_in ? sd.x0 : sd.src;
    char* base = sd.arena[a.psel];
    const long long vs = sd.vstride[a.psel];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      int c[4];
      cb_coords(g, site, par, c);
      const double* p = src + lex_index(g, c) * 24;
      Spinor<A> s;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        double re = p[2 * k], im = p[2 * k + 1];
        nn += re * re + im * im;
        double sgn = (a.gamma5 && k >= 6) ? -1.0 : 1.0;
        s.v[k] = mk((A)(sgn * re), (A)(sgn * im));
      }
      store_spinor<S, A>(base + (size_t)(par ? a.v_odd : a.v_even) * vs, hv, site, s);
    }
  }
  if (a.red != RED_NONE) {
    double v[1] = {nn};
    reduce_slot<1, BS>(v, a.red, sd.sid, tile.y, sd.nblk, sd.scal, hv, a.rb);
  }
}

template <class P>
__global__ __launch_bounds__(BS) void k_layout_out(LayoutArgs a) {
  using S = typename P::S;
  using A = typename P::A;
  const int2 tile = a.tiles[blockIdx.x];
  const int slot = tile.x;
  const SlotDev& sd = a.slots[slot];
  const Geo g = a.ops[sd.op].g;
  const int hv = g.hv;
  const int site = tile.y * BS + (int)threadIdx.x;
  if (site >= hv) return;
  double* dst = sd.sol;
  const char* base = sd.arena[a.psel];
  const long long vs = sd.vstride[a.psel];
#pragma unroll
  for (int par = 0; par < 2; ++par) {
    int c[4];
    cb_coords(g, site, par, c);
    double* p = dst + lex_index(g, c) * 24;
    Spinor<A> s;
    load_spinor<S, A>(base + (size_t)(par ? a.v_odd : a.v_even) * vs, hv, site, s);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      double sgn = (a.gamma5 && k >= 6) ? -1.0 : 1.0;
      p[2 * k] = sgn * (double)s.v[k].re;
      p[2 * k + 1] = sgn * (double)s.v[k].im;
    }
  }
}

void launch_layout_in(int prec, const LayoutArgs& a, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return;
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_layout_in<PrecF64>, dim3(ntiles), dim3(BS), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_layout_in<PrecF32>, dim3(ntiles), dim3(BS), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_layout_in<PrecF16>, dim3(ntiles), dim3(BS), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_layout_in<PrecB16>, dim3(ntiles), dim3(BS), 0, s, a); break;
    default: break;
  }
}

void launch_layout_out(int prec, const LayoutArgs& a, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return;
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_layout_out<PrecF64>, dim3(ntiles), dim3(BS), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_layout_out<PrecF32>, dim3(ntiles), dim3(BS), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_layout_out<PrecF16>, dim3(ntiles), dim3(BS), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_layout_out<PrecB16>, dim3(ntiles), dim3(BS), 0, s, a); break;
    default: break;
  }
}

}  // namespace a2a
