// blas.hip -- BiCGStab vector updates with fused FP64 block reductions, the reliable-update
// (mixed-precision defect correction) kernels, site-local clover application, the
// canonical <-> even-odd layout kernels and the reduction finalize kernel.
//
// All kernels run over per-slot tiles {slot, site block}; one thread owns one site of one
// slot.  Inner vectors live in the slot's working-precision arena, FP64 vectors in its
// FP64 arena; the inner vectors carry a per-slot scale sigma (inner = true / sigma) so
// that FP16 storage stays well inside its normal range whatever the residual norm.
// Each vector operation is its own kernel instantiation, so the simple updates keep a
// small register footprint and high occupancy.
#include "a2a_kernels.h"

namespace a2a {

template <typename A>
__device__ __forceinline__ cx<A> scal_c(const double* sc, int k) {
  return mk((A)sc[k], (A)sc[k + 1]);
}

template <typename A>
__device__ __forceinline__ void dot3(const Spinor<A>& a, const Spinor<A>& b, double* v) {
  // v[0] + i v[1] += (a, b) = sum conj(a) b;  v[2] += |b|^2
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    v[0] += (double)a.v[k].re * b.v[k].re + (double)a.v[k].im * b.v[k].im;
    v[1] += (double)a.v[k].re * b.v[k].im - (double)a.v[k].im * b.v[k].re;
    v[2] += (double)b.v[k].re * b.v[k].re + (double)b.v[k].im * b.v[k].im;
  }
}

template <class P, int KIND>
__global__ __launch_bounds__(BS) void k_vec(VecArgs a) {
  using S = typename P::S;
  using SX = typename P::SX;
  using A = typename P::A;
  const int2 tile = a.tiles[blockIdx.x];
  const SlotDev& sd = a.slots[tile.x];
  const int hv = a.ops[sd.op].g.hv;
  const int site = tile.y * BS + (int)threadIdx.x;
  const bool valid = site < hv;
  char* lo = sd.arena[0];
  char* hi = sd.arena[1];
  const long long vl = sd.vstride[0], vh = sd.vstride[1];
  const double* sc = sd.scal;
#define LO(v) (lo + (size_t)(v) * vl)
#define HI(v) (hi + (size_t)(v) * vh)

  if (KIND == VK_BICG_S) {  // s = r - alpha v
    if (!valid) return;
    const cx<A> al = scal_c<A>(sc, SC_ALPHA);
    Spinor<A> r, v;
    load_spinor<S, A>(LO(VL_R), hv, site, r);
    load_spinor<S, A>(LO(VL_V), hv, site, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) r.v[k] = r.v[k] - al * v.v[k];
    store_spinor<S, A>(LO(VL_S), hv, site, r);
  } else if (KIND == VK_BICG_P) {  // p = r + beta (p - omega v)
    if (!valid) return;
    const cx<A> be = scal_c<A>(sc, SC_BETA), om = scal_c<A>(sc, SC_OMEGA);
    Spinor<A> r, p, v;
    load_spinor<S, A>(LO(VL_R), hv, site, r);
    load_spinor<S, A>(LO(VL_P), hv, site, p);
    load_spinor<S, A>(LO(VL_V), hv, site, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) p.v[k] = r.v[k] + be * (p.v[k] - om * v.v[k]);
    store_spinor<S, A>(LO(VL_P), hv, site, p);
  } else if (KIND == VK_BICG_XR) {  // x += alpha p + omega s; r = s - omega t; (rhat, r), |r|^2
    double v3[3] = {0.0, 0.0, 0.0};
    if (valid) {
      const cx<A> al = scal_c<A>(sc, SC_ALPHA), om = scal_c<A>(sc, SC_OMEGA);
      Spinor<A> x, p, s, t;
      load_spinor<SX, A>(LO(VL_X), hv, site, x);
      load_spinor<S, A>(LO(VL_P), hv, site, p);
      load_spinor<S, A>(LO(VL_S), hv, site, s);
      load_spinor<S, A>(LO(VL_T), hv, site, t);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        x.v[k] = x.v[k] + al * p.v[k] + om * s.v[k];
        s.v[k] = s.v[k] - om * t.v[k];
      }
      store_spinor<SX, A>(LO(VL_X), hv, site, x);
      store_spinor<S, A>(LO(VL_R), hv, site, s);
      load_spinor<S, A>(LO(VL_R), hv, site, s);  // reduce the stored values
      Spinor<A> rh;
      load_spinor<S, A>(LO(VL_RHAT), hv, site, rh);
      dot3(rh, s, v3);
    }
    block_sum_n<3, BS>(v3);
    if (threadIdx.x < 3)
      store_partial(a.rb, sd.sid, tile.y, threadIdx.x, threadIdx.x == 0 ? v3[0] : threadIdx.x == 1 ? v3[1] : v3[2]);
  } else if (KIND == VK_RU_ACCUM) {  // x64 += sigma x_lo; x_lo = 0
    if (!valid) return;
    const double sg = sc[SC_SIGMA];
    Spinor<A> xl;
    Spinor<double> xh;
    load_spinor<SX, A>(LO(VL_X), hv, site, xl);
    load_spinor<double, double>(HI(VH_X), hv, site, xh);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      xh.v[k].re += sg * (double)xl.v[k].re;
      xh.v[k].im += sg * (double)xl.v[k].im;
      xl.v[k] = mk((A)0, (A)0);
    }
    store_spinor<double, double>(HI(VH_X), hv, site, xh);
    store_spinor<SX, A>(LO(VL_X), hv, site, xl);
  } else if (KIND == VK_RU_RESCALE || KIND == VK_INIT) {
    double v3[3] = {0.0, 0.0, 0.0};
    const double snew =
        KIND == VK_INIT ? sqrt(sc[SC_R64N2] / (12.0 * hv)) : ru_scale(sc[SC_R64N2], sc[SC_SIGMA], hv);
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
      if (KIND == VK_INIT) {
        Spinor<A> z;
#pragma unroll
        for (int k = 0; k < 12; ++k) z.v[k] = mk((A)0, (A)0);
        store_spinor<S, A>(LO(VL_RHAT), hv, site, r);
        store_spinor<S, A>(LO(VL_P), hv, site, r);
        store_spinor<S, A>(LO(VL_V), hv, site, z);
        store_spinor<SX, A>(LO(VL_X), hv, site, z);
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
      dot3(rh, r, v3);
    }
    block_sum_n<3, BS>(v3);
    if (threadIdx.x < 3)
      store_partial(a.rb, sd.sid, tile.y, threadIdx.x, threadIdx.x == 0 ? v3[0] : threadIdx.x == 1 ? v3[1] : v3[2]);
  } else if (KIND == VK_CLOVER) {  // FP64: hi[vout] = C hi[vin], C = A or A^{-1} of parity par
    if (!valid) return;
    const OpDev& op = a.ops[sd.op];
    const void* C = a.use_inv ? op.Ai[1][a.par] : op.A[1][a.par];
    Spinor<double> in, out;
    load_spinor<double, double>(HI(a.vin), hv, site, in);
    clover_apply_mem<double, double>(C, hv, site, in, out);
    store_spinor<double, double>(HI(a.vout), hv, site, out);
  } else if (KIND == VK_ZERO_X) {
    if (!valid) return;
    Spinor<A> z;
#pragma unroll
    for (int k = 0; k < 12; ++k) z.v[k] = mk((A)0, (A)0);
    store_spinor<SX, A>(LO(VL_X), hv, site, z);
  } else if (KIND == VK_ZERO_HI) {
    if (!valid) return;
    Spinor<double> z;
#pragma unroll
    for (int k = 0; k < 12; ++k) z.v[k] = mk(0.0, 0.0);
    store_spinor<double, double>(HI(a.vout), hv, site, z);
  } else if (KIND == VK_ZERO_LO || KIND == VK_FILL_LO) {
    if (!valid) return;
    Spinor<A> z;
    uint32_t h = (uint32_t)site * 2654435761u + (uint32_t)sd.sid * 40503u + 12345u;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      if (KIND == VK_ZERO_LO) {
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
  }
#undef LO
#undef HI
}

template <class P>
static void launch_vec_p(const VecArgs& a, int n, hipStream_t s) {
  const dim3 g(n), b(BS);
  switch (a.kind) {
    case VK_BICG_S: hipLaunchKernelGGL((k_vec<P, VK_BICG_S>), g, b, 0, s, a); break;
    case VK_BICG_XR: hipLaunchKernelGGL((k_vec<P, VK_BICG_XR>), g, b, 0, s, a); break;
    case VK_BICG_P: hipLaunchKernelGGL((k_vec<P, VK_BICG_P>), g, b, 0, s, a); break;
    case VK_RU_ACCUM: hipLaunchKernelGGL((k_vec<P, VK_RU_ACCUM>), g, b, 0, s, a); break;
    case VK_RU_RESCALE: hipLaunchKernelGGL((k_vec<P, VK_RU_RESCALE>), g, b, 0, s, a); break;
    case VK_INIT: hipLaunchKernelGGL((k_vec<P, VK_INIT>), g, b, 0, s, a); break;
    case VK_CLOVER: hipLaunchKernelGGL((k_vec<P, VK_CLOVER>), g, b, 0, s, a); break;
    case VK_ZERO_HI: hipLaunchKernelGGL((k_vec<P, VK_ZERO_HI>), g, b, 0, s, a); break;
    case VK_ZERO_X: hipLaunchKernelGGL((k_vec<P, VK_ZERO_X>), g, b, 0, s, a); break;
    case VK_ZERO_LO: hipLaunchKernelGGL((k_vec<P, VK_ZERO_LO>), g, b, 0, s, a); break;
    case VK_FILL_LO: hipLaunchKernelGGL((k_vec<P, VK_FILL_LO>), g, b, 0, s, a); break;
    default: break;
  }
}

void launch_vec(int prec, const VecArgs& a, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return;
  switch (prec) {
    case 0: launch_vec_p<PrecF64>(a, ntiles, s); break;
    case 1: launch_vec_p<PrecF32>(a, ntiles, s); break;
    case 2: launch_vec_p<PrecF16>(a, ntiles, s); break;
    case 3: launch_vec_p<PrecB16>(a, ntiles, s); break;
    default: break;
  }
}

// ------------------------------------------------------------------------------------
// reduction finalize: one 64-thread block per slot, partials summed in block order
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_finalize(int kind, const OpDev* ops, const SlotDev* slots, const int* list,
                                                  RedBuf rb) {
  const int idx = list ? list[blockIdx.x] : (int)blockIdx.x;
  const SlotDev& sd = slots[idx];
  const double* p = rb.partials + (size_t)sd.sid * rb.maxblk * RED_NV;
  double v[RED_NV] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < sd.nblk; b += 64)
#pragma unroll
    for (int k = 0; k < RED_NV; ++k) v[k] += p[(size_t)b * RED_NV + k];
#pragma unroll
  for (int k = 0; k < RED_NV; ++k) v[k] = wave_sum(v[k]);
  if (threadIdx.x == 0) finalize_slot(kind, sd.scal, v, ops[sd.op].g.hv);
}

void launch_finalize(int kind, const OpDev* ops, const SlotDev* slots, const int* list, int n, RedBuf rb,
                     hipStream_t s) {
  if (n <= 0 || kind == RED_NONE) return;
  hipLaunchKernelGGL(k_finalize, dim3(n), dim3(64), 0, s, kind, ops, slots, list, rb);
}

// ------------------------------------------------------------------------------------
// canonical <-> even-odd layout (per slot), optional gamma_5, optional |in|^2
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BS) void k_layout_in(LayoutArgs a) {
  using S = typename P::S;
  using A = typename P::A;
  const int2 tile = a.tiles[blockIdx.x];
  const SlotDev& sd = a.slots[tile.x];
  const Geo g = a.ops[sd.op].g;
  const int hv = g.hv;
  const int site = tile.y * BS + (int)threadIdx.x;
  double nn[1] = {0.0};
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
        nn[0] += re * re + im * im;
        double sgn = (a.gamma5 && k >= 6) ? -1.0 : 1.0;
        s.v[k] = mk((A)(sgn * re), (A)(sgn * im));
      }
      store_spinor<S, A>(base + (size_t)(par ? a.v_odd : a.v_even) * vs, hv, site, s);
    }
  }
  if (a.red != RED_NONE) {
    block_sum_n<1, BS>(nn);
    if (threadIdx.x == 0) store_partial(a.rb, sd.sid, tile.y, 0, nn[0]);
  }
}

template <class P>
__global__ __launch_bounds__(BS) void k_layout_out(LayoutArgs a) {
  using S = typename P::S;
  using A = typename P::A;
  const int2 tile = a.tiles[blockIdx.x];
  const SlotDev& sd = a.slots[tile.x];
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
