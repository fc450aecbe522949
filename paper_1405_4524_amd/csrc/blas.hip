// blas.hip -- BiCGStab and CGNR vector updates with fused FP64 block reductions, the reliable-update
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

// a spinor rounded to the storage format, as a store followed by a load would give it
template <typename S, typename A>
__device__ __forceinline__ void round_to(Spinor<A>& s) {
#pragma unroll
  for (int k = 0; k < 12; ++k)
    s.v[k] = mk(Conv<S>::template to<A>(Conv<S>::from(s.v[k].re)), Conv<S>::template to<A>(Conv<S>::from(s.v[k].im)));
}

// kinds whose result feeds a reduction
template <int KIND>
struct VecRed {
  static constexpr bool on = KIND == VK_BICG_XR || KIND == VK_RU_RESCALE || KIND == VK_INIT || KIND == VK_CG_XR ||
                             KIND == VK_CG_INIT || KIND == VK_CG_RESCALE;
};

// One site of one slot.  Reducing kinds add their (rhat, r), |r|^2 contributions to v3.
// NT: streaming (non-temporal) loads and stores of the inner vectors and of the FP64 vectors of the
// reliable-update kinds (lane-interleaved kernels: each value is touched once)
template <class P, int KIND, bool NT = false>
__device__ __forceinline__ void vec_site(const VecArgs& a, const SlotDev& sd, int hv, int site, double (&v3)[3]) {
  using S = typename P::S;
  using SX = typename P::SX;
  using A = typename P::A;
  const VView lw = lo_view(sd);
  const VView hw = hi_view(sd, hv);  // the slot's FP64 vectors (chunk planes)
  char* hi = sd.arena[1];
  const long long vh = sd.vstride[1];
  const double* sc = sd.scal;
#define HI(v) (hi + (size_t)(v) * vh)
  if (KIND == VK_BICG_S) {  // s = r - alpha v
    const cx<A> al = scal_c<A>(sc, SC_ALPHA);
    Spinor<A> r, v;
    vload<S, A, NT>(lw, VL_R, site, r);
    vload<S, A, NT>(lw, VL_V, site, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) r.v[k] = r.v[k] - al * v.v[k];
    vstore<S, A, NT>(lw, VL_S, site, r);
  } else if (KIND == VK_BICG_P) {  // p = r + beta (p - omega v)
    const cx<A> be = scal_c<A>(sc, SC_BETA), om = scal_c<A>(sc, SC_OMEGA);
    Spinor<A> r, p, v;
    vload<S, A, NT>(lw, VL_R, site, r);
    vload<S, A, NT>(lw, VL_P, site, p);
    vload<S, A, NT>(lw, VL_V, site, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) p.v[k] = r.v[k] + be * (p.v[k] - om * v.v[k]);
    vstore<S, A, NT>(lw, VL_P, site, p);
  } else if (KIND == VK_BICG_XR) {  // x += alpha p + omega s; r = s - omega t; (rhat, r), |r|^2
    const cx<A> al = scal_c<A>(sc, SC_ALPHA), om = scal_c<A>(sc, SC_OMEGA);
    Spinor<A> x, p, s, t;
    xload<SX, A, NT>(sd, VL_X, site, x);
    vload<S, A, NT>(lw, VL_P, site, p);
    vload<S, A, NT>(lw, VL_S, site, s);
    vload<S, A, NT>(lw, VL_T, site, t);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      x.v[k] = x.v[k] + al * p.v[k] + om * s.v[k];
      s.v[k] = s.v[k] - om * t.v[k];
    }
    xstore<SX, A, NT>(sd, VL_X, site, x);
    vstore<S, A, NT>(lw, VL_R, site, s);
    round_to<S>(s);  // reduce the values as stored
    Spinor<A> rh;
    vload<S, A, NT>(lw, VL_RHAT, site, rh);
    dot3(rh, s, v3);
  } else if (KIND == VK_CG_XR) {  // x += alpha p; r' -= alpha gamma5 q; |r'|^2
    const A al = (A)sc[SC_ALPHA];
    Spinor<A> x, p, r, q;
    xload<SX, A, NT>(sd, VL_X, site, x);
    vload<S, A, NT>(lw, VL_P, site, p);
    vload<S, A, NT>(lw, VL_R, site, r);
    vload<S, A, NT>(lw, VL_V, site, q);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      x.v[k] = x.v[k] + al * p.v[k];
      r.v[k] = k < 6 ? r.v[k] - al * q.v[k] : r.v[k] + al * q.v[k];
    }
    xstore<SX, A, NT>(sd, VL_X, site, x);
    vstore<S, A, NT>(lw, VL_R, site, r);
    round_to<S>(r);
    dot3(r, r, v3);
  } else if (KIND == VK_CG_P) {  // p = gamma5 u + beta p
    const A be = (A)sc[SC_BETA];
    Spinor<A> u, p;
    vload<S, A, NT>(lw, VL_S, site, u);
    vload<S, A, NT>(lw, VL_P, site, p);
#pragma unroll
    for (int k = 0; k < 12; ++k) p.v[k] = (k < 6 ? u.v[k] : mk(-u.v[k].re, -u.v[k].im)) + be * p.v[k];
    vstore<S, A, NT>(lw, VL_P, site, p);
  } else if (KIND == VK_CG_INIT || KIND == VK_CG_RESCALE) {  // r' = gamma5 r64 / sigma'
    const double snew =
        KIND == VK_CG_INIT ? sqrt(sc[SC_R64N2] / (12.0 * hv)) : ru_scale(sc[SC_R64N2], sc[SC_SIGMA], hv);
    const double inv = (snew > 0.0) ? 1.0 / snew : 0.0;
    Spinor<double> rh64;
    vload<double, double, NT>(hw, a.vin >= 0 ? a.vin : VH_R, site, rh64);
    Spinor<A> r;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double f = k < 6 ? inv : -inv;
      r.v[k] = mk((A)(rh64.v[k].re * f), (A)(rh64.v[k].im * f));
    }
    vstore<S, A, NT>(lw, VL_R, site, r);
    round_to<S>(r);
    Spinor<A> p;
    if (KIND == VK_CG_INIT) {
#pragma unroll
      for (int k = 0; k < 12; ++k) p.v[k] = mk((A)0, (A)0);
      xstore<SX, A, NT>(sd, VL_X, site, p);
    } else {
      const A ratio = (A)(sc[SC_SIGMA] * inv);
      vload<S, A, NT>(lw, VL_P, site, p);
#pragma unroll
      for (int k = 0; k < 12; ++k) p.v[k] = ratio * p.v[k];
    }
    vstore<S, A, NT>(lw, VL_P, site, p);
    dot3(r, r, v3);
  } else if (KIND == VK_RU_ACCUM) {  // x64 += sigma x_lo; x_lo = 0
    const double sg = sc[SC_SIGMA];
    Spinor<A> xl;
    Spinor<double> xh;
    xload<SX, A, NT>(sd, VL_X, site, xl);
    vload<double, double, NT>(hw, VH_X, site, xh);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      xh.v[k].re += sg * (double)xl.v[k].re;
      xh.v[k].im += sg * (double)xl.v[k].im;
      xl.v[k] = mk((A)0, (A)0);
    }
    vstore<double, double, NT>(hw, VH_X, site, xh);
    xstore<SX, A, NT>(sd, VL_X, site, xl);
  } else if (KIND == VK_RU_RESCALE || KIND == VK_INIT) {
    const double snew =
        KIND == VK_INIT ? sqrt(sc[SC_R64N2] / (12.0 * hv)) : ru_scale(sc[SC_R64N2], sc[SC_SIGMA], hv);
    const double inv = (snew > 0.0) ? 1.0 / snew : 0.0;
    Spinor<double> rh64;
    vload<double, double, NT>(hw, a.vin >= 0 ? a.vin : VH_R, site, rh64);
    if (a.use_inv) {  // symmetric Schur form: the inner right-hand side is A_oo^{-1} r64
      Spinor<double> t;
      clover_apply_mem<double, double>(a.ops[sd.op].Ai[1][1], hv, site, rh64, t);
      rh64 = t;
    }
    Spinor<A> r;
#pragma unroll
    for (int k = 0; k < 12; ++k) r.v[k] = mk((A)(rh64.v[k].re * inv), (A)(rh64.v[k].im * inv));
    vstore<S, A, NT>(lw, VL_R, site, r);
    round_to<S>(r);  // the values as stored
    Spinor<A> rh;
    if (KIND == VK_INIT) {
      Spinor<A> z;
#pragma unroll
      for (int k = 0; k < 12; ++k) z.v[k] = mk((A)0, (A)0);
      vstore<S, A, NT>(lw, VL_RHAT, site, r);
      vstore<S, A, NT>(lw, VL_P, site, r);
      vstore<S, A, NT>(lw, VL_V, site, z);
      xstore<SX, A, NT>(sd, VL_X, site, z);
      rh = r;
    } else {
      const A ratio = (A)(sc[SC_SIGMA] * inv);
      Spinor<A> p, v;
      vload<S, A, NT>(lw, VL_P, site, p);
      vload<S, A, NT>(lw, VL_V, site, v);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        p.v[k] = ratio * p.v[k];
        v.v[k] = ratio * v.v[k];
      }
      vstore<S, A, NT>(lw, VL_P, site, p);
      vstore<S, A, NT>(lw, VL_V, site, v);
      vload<S, A, NT>(lw, VL_RHAT, site, rh);
    }
    dot3(rh, r, v3);
  } else if (KIND == VK_CLOVER) {  // FP64: hi[vout] = C hi[vin], C = A or A^{-1} of parity par
    const OpDev& op = a.ops[sd.op];
    const void* C = a.use_inv ? op.Ai[1][a.par] : op.A[1][a.par];
    Spinor<double> in, out;
    load_spinor<double, double>(HI(a.vin), hv, site, in);
    clover_apply_mem<double, double>(C, hv, site, in, out);
    store_spinor<double, double>(HI(a.vout), hv, site, out);
  } else if (KIND == VK_ZERO_X) {
    Spinor<A> z;
#pragma unroll
    for (int k = 0; k < 12; ++k) z.v[k] = mk((A)0, (A)0);
    xstore<SX, A, NT>(sd, VL_X, site, z);
  } else if (KIND == VK_ZERO_HI) {
    Spinor<double> z;
#pragma unroll
    for (int k = 0; k < 12; ++k) z.v[k] = mk(0.0, 0.0);
    store_spinor<double, double>(HI(a.vout), hv, site, z);
  } else if (KIND == VK_COPY_HI) {
    Spinor<double> z;
    load_spinor<double, double>(HI(a.vin), hv, site, z);
    store_spinor<double, double>(HI(a.vout), hv, site, z);
  } else if (KIND == VK_ZERO_LO || KIND == VK_FILL_LO) {
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
    vstore<S, A, NT>(lw, a.vout, site, z);
  }
#undef HI
}

// per-slot mapping: tiles {slot, block of BS sites}, one site per thread
template <class P, int KIND>
__global__ __launch_bounds__(BS) void k_vec(VecArgs a) {
  const int2 tile = a.tiles[blockIdx.x];
  const SlotDev& sd = a.slots[tile.x];
  const int hv = a.ops[sd.op].g.hv;
  const int site = tile.y * BS + (int)threadIdx.x;
  double v3[3] = {0.0, 0.0, 0.0};
  if (site < hv) vec_site<P, KIND>(a, sd, hv, site, v3);
  if (VecRed<KIND>::on) {
    block_sum_n<3, BS>(v3);
    if (threadIdx.x < 3)
      store_partial(a.rb, sd.sid, tile.y, threadIdx.x, threadIdx.x == 0 ? v3[0] : threadIdx.x == 1 ? v3[1] : v3[2]);
  }
}

// interleaved mapping: tiles {16-lane group tile, block of BS sites}; BSI threads as (lane n,
// row q) visit sites block*BS + 64 i + q, and a block keeps 16 waves of loads in flight.
// Kinds on inner vectors only give a wave 4 sites x 16 lanes (4 contiguous 256-byte runs per
// chunk).  Kinds that also touch the slots' FP64 vectors, whose chunk planes are per slot
// ([chunk][site]), give a wave 8 sites x 8 lanes instead: 8 full 128-byte lines of the
// interleaved arena per chunk, and for each of its 8 slots 8 consecutive FP64 chunks = one full
// line (4 sites x 16 lanes used half lines there).  Reductions are per lane (slot) and land in
// the same partial slots as the per-slot mapping (block index = site block of BS sites).
constexpr int BSI = 1024;

template <int KIND>
struct VecWide {
  static constexpr bool on = KIND == VK_RU_ACCUM || KIND == VK_RU_RESCALE || KIND == VK_INIT || KIND == VK_CG_INIT ||
                             KIND == VK_CG_RESCALE;
};

template <class P, int KIND>
__global__ __launch_bounds__(BSI) void k_vec_il(VecArgs a) {
  constexpr bool wide = VecWide<KIND>::on;
  const int2 tile = a.tiles[blockIdx.x];
  const int t = threadIdx.x;
  // wide: thread bits [0..2] lane, [3..8] row, [9] lane bit 3; else [0..3] lane, [4..9] row
  const int n = wide ? (t & 7) | ((t >> 9) << 3) : t & 15;
  const int q = wide ? (t >> 3) & 63 : t >> 4;
  const int slot = a.ilslots[tile.x * 16 + n];
  double v3[3] = {0.0, 0.0, 0.0};
  if (slot >= 0) {
    const SlotDev& sd = a.slots[slot];
    const int hv = a.ops[sd.op].g.hv;
#pragma unroll
    for (int i = 0; i < BS / (BSI / 16); ++i) {
      const int site = tile.y * BS + (BSI / 16) * i + q;
      if (site < hv) vec_site<P, KIND, true>(a, sd, hv, site, v3);
    }
  }
  if (VecRed<KIND>::on) {
    // per wave: sum the lanes of equal n (wide: 8 lanes, each on 8 sites; else 16 lanes on 4)
    __shared__ double red[BSI / 64][16][3];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (wide) v3[k] += __shfl_xor(v3[k], 8, 64);
      v3[k] += __shfl_xor(v3[k], 16, 64);
      v3[k] += __shfl_xor(v3[k], 32, 64);
    }
    if (lane < (wide ? 8 : 16))
#pragma unroll
      for (int k = 0; k < 3; ++k) red[w][lane][k] = v3[k];
    __syncthreads();
    if (threadIdx.x < 48) {
      const int m = threadIdx.x & 15, k = threadIdx.x >> 4;
      const int sl = a.ilslots[tile.x * 16 + m];
      if (sl >= 0) {
        double s = 0.0;
        if (wide) {  // lane m lives in waves 8 (m >> 3) .. 8 (m >> 3) + 7 at wave lane m & 7
#pragma unroll
          for (int j = 0; j < BSI / 128; ++j) s += red[8 * (m >> 3) + j][m & 7][k];
        } else {
#pragma unroll
          for (int j = 0; j < BSI / 64; ++j) s += red[j][m][k];
        }
        store_partial(a.rb, a.slots[sl].sid, tile.y, k, s);
      }
    }
  }
}

template <class P>
static void launch_vec_il_p(const VecArgs& a, int n, hipStream_t s) {
  const dim3 g(n), b(BSI);
  switch (a.kind) {
    case VK_BICG_S: hipLaunchKernelGGL((k_vec_il<P, VK_BICG_S>), g, b, 0, s, a); break;
    case VK_BICG_XR: hipLaunchKernelGGL((k_vec_il<P, VK_BICG_XR>), g, b, 0, s, a); break;
    case VK_BICG_P: hipLaunchKernelGGL((k_vec_il<P, VK_BICG_P>), g, b, 0, s, a); break;
    case VK_RU_ACCUM: hipLaunchKernelGGL((k_vec_il<P, VK_RU_ACCUM>), g, b, 0, s, a); break;
    case VK_RU_RESCALE: hipLaunchKernelGGL((k_vec_il<P, VK_RU_RESCALE>), g, b, 0, s, a); break;
    case VK_INIT: hipLaunchKernelGGL((k_vec_il<P, VK_INIT>), g, b, 0, s, a); break;
    case VK_ZERO_X: hipLaunchKernelGGL((k_vec_il<P, VK_ZERO_X>), g, b, 0, s, a); break;
    case VK_ZERO_LO: hipLaunchKernelGGL((k_vec_il<P, VK_ZERO_LO>), g, b, 0, s, a); break;
    case VK_FILL_LO: hipLaunchKernelGGL((k_vec_il<P, VK_FILL_LO>), g, b, 0, s, a); break;
    case VK_CG_XR: hipLaunchKernelGGL((k_vec_il<P, VK_CG_XR>), g, b, 0, s, a); break;
    case VK_CG_P: hipLaunchKernelGGL((k_vec_il<P, VK_CG_P>), g, b, 0, s, a); break;
    case VK_CG_INIT: hipLaunchKernelGGL((k_vec_il<P, VK_CG_INIT>), g, b, 0, s, a); break;
    case VK_CG_RESCALE: hipLaunchKernelGGL((k_vec_il<P, VK_CG_RESCALE>), g, b, 0, s, a); break;
    default: break;
  }
}

bool vec_kind_il(int kind) {
  return kind == VK_BICG_S || kind == VK_BICG_XR || kind == VK_BICG_P || kind == VK_RU_ACCUM ||
         kind == VK_RU_RESCALE || kind == VK_INIT || kind == VK_ZERO_X || kind == VK_ZERO_LO || kind == VK_FILL_LO ||
         kind == VK_CG_XR || kind == VK_CG_P || kind == VK_CG_INIT || kind == VK_CG_RESCALE;
}

void launch_vec_il(int prec, const VecArgs& a, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return;
  switch (prec) {
    case 2: launch_vec_il_p<PrecF16>(a, ntiles, s); break;
    case 3: launch_vec_il_p<PrecB16>(a, ntiles, s); break;
    default: break;
  }
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
    case VK_COPY_HI: hipLaunchKernelGGL((k_vec<P, VK_COPY_HI>), g, b, 0, s, a); break;
    case VK_ZERO_X: hipLaunchKernelGGL((k_vec<P, VK_ZERO_X>), g, b, 0, s, a); break;
    case VK_ZERO_LO: hipLaunchKernelGGL((k_vec<P, VK_ZERO_LO>), g, b, 0, s, a); break;
    case VK_FILL_LO: hipLaunchKernelGGL((k_vec<P, VK_FILL_LO>), g, b, 0, s, a); break;
    case VK_CG_XR: hipLaunchKernelGGL((k_vec<P, VK_CG_XR>), g, b, 0, s, a); break;
    case VK_CG_P: hipLaunchKernelGGL((k_vec<P, VK_CG_P>), g, b, 0, s, a); break;
    case VK_CG_INIT: hipLaunchKernelGGL((k_vec<P, VK_CG_INIT>), g, b, 0, s, a); break;
    case VK_CG_RESCALE: hipLaunchKernelGGL((k_vec<P, VK_CG_RESCALE>), g, b, 0, s, a); break;
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
    const VView w = view_of(sd, a.psel, hv);
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
      vstore<S, A>(w, par ? a.v_odd : a.v_even, site, s);
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
  const VView w = view_of(sd, a.psel, hv);
#pragma unroll
  for (int par = 0; par < 2; ++par) {
    int c[4];
    cb_coords(g, site, par, c);
    double* p = dst + lex_index(g, c) * 24;
    Spinor<A> s;
    vload<S, A>(w, par ? a.v_odd : a.v_even, site, s);
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
