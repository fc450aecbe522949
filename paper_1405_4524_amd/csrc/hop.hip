// hop.hip -- the Wilson hopping stencil with fused clover / axpy / reduction epilogues.
//
// One thread owns one output site of one parity and R right-hand sides (a "group"), so
// each link is loaded once per thread and applied to R spinors: the multi-RHS blocks of
// the batched solver share link and clover traffic.  Neighbours are found from the
// site's coordinates (no index tables), and the fermion time-boundary sign is applied
// on the hops that wrap in t.  Blocks come from a tile list {group, site block} that the
// host orders so that each XCD sweeps a contiguous slab of the lattice for all groups.  With
// several groups per site block, a site block is a 4D brick of the lattice (x fastest inside),
// so that most neighbours of a block's sites are read by the same block at about the same
// time (FP64 stencils over 24 two-RHS groups: 7% faster); a single group keeps whole (x, y)
// planes per block, whose z and t neighbours are read by blocks in flight at the same time
// (bricks made that case 5-8% slower).
#include <type_traits>

#include "a2a_kernels.h"

namespace a2a {

// EPI_INVA: o = aux2 + A^{-1} (gam H in), the symmetric Schur operator's second stencil
enum { EPI_PLAIN = 0, EPI_CLOV = 1, EPI_INV = 2, EPI_INVA = 3 };

// LOM (FP64 stencils of the correction-form reliable update): 1 = the hopping input, 2 = the
// clover input aux2 is the slot's inner vector in storage SI, scaled by the slot's sigma (the
// inner vectors hold the true vector / sigma), read through the slot's inner layout.
template <class P, int R, int EPI, int LOM = 0, typename SI = typename P::S>
__global__ __launch_bounds__(BS) void k_hop(HopArgs a) {
  using S = typename P::S;
  using A = typename P::A;
  // FP64 stencils: the site's own operands and the output are touched once (streaming access),
  // and the output's reductions come from the registers (the stored values are the same)
  constexpr bool NTX = std::is_same<S, double>::value;
  const int2 tile = a.tiles[blockIdx.x];
  const int* grp = a.groups + (size_t)tile.x * R;
  const int slot0 = grp[0];
  const OpDev& op = a.ops[a.slots[slot0].op];
  Geo g = op.g;
  if (a.by > 0 && g.Y % a.by == 0 && g.Z % a.bz == 0 && g.T % a.bt == 0) {  // the launch's own brick
    g.by = (unsigned char)a.by;
    g.bz = (unsigned char)a.bz;
    g.bt = (unsigned char)a.bt;
  }
  const int hv = g.hv;
  const int pos = tile.y * BS + (int)threadIdx.x;  // position in the brick sweep
  const bool valid = pos < hv;
  const int site = !valid ? 0 : a.brick ? brick_site<false>(g, pos) : pos;
  const int sel = a.psel;
  const int po = a.out_par, pi = 1 - po;

  VView w[R], wl[R];
  A sgm[R];  // the slot's sigma for LOM terms
  bool on[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int sl = grp[r];
    on[r] = sl >= 0;
    const SlotDev& sd = a.slots[on[r] ? sl : slot0];
    w[r] = view_of(sd, sel, hv);
    wl[r] = lo_view(sd);
    sgm[r] = LOM != 0 ? (A)sd.scal[SC_SIGMA] : (A)1;
  }

  Spinor<A> acc[R];
  Spinor<A> resid[R];  // the reconstruction's r_e (EPI_INV with RED_RES_E)
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[r].v[k] = resid[r].v[k] = mk((A)0, (A)0);

  if (valid) {
    int c[4];
    cb_coords(g, site, po, c);
    const char* Uo = (const char*)op.U[sel][po];
    const char* Ui = (const char*)op.U[sel][pi];
    const size_t lb = LinkF<S>::bytes(hv);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      {  // forward: (1 - gamma_mu) U_mu(x) psi(x + mu)
        const int nf = neighbor(g, c, mu, +1);
        const A ph = (mu == 3 && c[3] == g.T - 1) ? (A)g.tbc : (A)1;
        Su3<A> U;
        LinkF<S>::template load<A>(Uo + mu * lb, hv, site, (A*)U.m);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!on[r]) continue;
          Spinor<A> p;
          if (LOM == 1)
            vload<SI, A>(wl[r], a.vin, nf, p);
          else
            vload<S, A>(w[r], a.vin, nf, p);
          cx<A> h[6], uh[6];
          project(mu, 1, p, h);
          su3_mul_half(U, h, uh);
          reconstruct_acc(mu, 1, uh, ph, acc[r]);
        }
      }
      {  // backward: (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
        const int nb = neighbor(g, c, mu, -1);
        const A ph = (mu == 3 && c[3] == 0) ? (A)g.tbc : (A)1;
        Su3<A> U;
        LinkF<S>::template load<A>(Ui + mu * lb, hv, nb, (A*)U.m);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!on[r]) continue;
          Spinor<A> p;
          if (LOM == 1)
            vload<SI, A>(wl[r], a.vin, nb, p);
          else
            vload<S, A>(w[r], a.vin, nb, p);
          cx<A> h[6], uh[6];
          project(mu, 0, p, h);
          su3_dag_mul_half(U, h, uh);
          reconstruct_acc(mu, 0, uh, ph, acc[r]);
        }
      }
    }
  }

  // ---- epilogue: acc <- gam * acc + ca * aux1 (+ cb * A aux2) (then A^{-1} .)
  double kp = 1.0;
  for (int i = 0; i < a.gpow; ++i) kp *= op.kappa;
  const A gam = (A)(a.gsign * kp);
  const A ca = (A)a.ca, cbv = (A)a.cb;
  if (valid) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!on[r]) continue;
      const A gr = LOM == 1 ? gam * sgm[r] : gam;
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[r].v[k] = gr * acc[r].v[k];
      if (a.vaux1 >= 0) {
        Spinor<A> x1;
        vload<S, A, NTX>(w[r], a.vaux1, site, x1);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[r].v[k] = acc[r].v[k] + ca * x1.v[k];
      }
    }
    // EPI_INV with RED_RES_E (the reconstruction): also r_e = y - A x_e, y the input of A^{-1}
    // (eta_e + kappa H_eo x_o) and x_e the output as stored, and its |r_e|^2
    const bool res_e = EPI == EPI_INV && std::is_same<S, double>::value && a.red == RED_RES_E;
    if (EPI != EPI_PLAIN) {
      const void* cbase = (EPI == EPI_CLOV) ? op.A[sel][po] : op.Ai[sel][po];
      Spinor<A> x3[R];  // EPI_INVA: the identity term
      if (EPI == EPI_INVA) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (on[r]) vload<S, A, NTX>(w[r], a.vaux2, site, x3[r]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        A blk[36];
        CloverBlkF<S>::template load<A>((const char*)cbase + b * CloverBlkF<S>::bytes(hv), hv, site, blk);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!on[r]) continue;
          cx<A> i6[6], o6[6];
          if (EPI == EPI_CLOV) {
            Spinor<A> x2;
            if (LOM == 2)
              vload<SI, A, NTX>(wl[r], a.vaux2, site, x2);
            else
              vload<S, A, NTX>(w[r], a.vaux2, site, x2);
            const A cr = LOM == 2 ? cbv * sgm[r] : cbv;
#pragma unroll
            for (int k = 0; k < 6; ++k) i6[k] = x2.v[b * 6 + k];
            clover_apply_block(blk, i6, o6);
#pragma unroll
            for (int k = 0; k < 6; ++k) acc[r].v[b * 6 + k] = acc[r].v[b * 6 + k] + cr * o6[k];
          } else {
#pragma unroll
            for (int k = 0; k < 6; ++k) i6[k] = acc[r].v[b * 6 + k];
            clover_apply_block(blk, i6, o6);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
              if (res_e) resid[r].v[b * 6 + k] = i6[k];  // y, kept for r_e
              acc[r].v[b * 6 + k] = EPI == EPI_INVA ? x3[r].v[b * 6 + k] + o6[k] : o6[k];
            }
          }
        }
      }
      if (res_e) {  // r_e = y - A x_e with x_e rounded as stored
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          A blk[36];
          CloverBlkF<S>::template load<A>((const char*)op.A[sel][po] + b * CloverBlkF<S>::bytes(hv), hv, site, blk);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (!on[r]) continue;
            cx<A> i6[6], o6[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
              const cx<A> xs = acc[r].v[b * 6 + k];
              i6[k] = mk((A)Conv<S>::template to<A>(Conv<S>::from(xs.re)), (A)Conv<S>::template to<A>(Conv<S>::from(xs.im)));
            }
            clover_apply_block(blk, i6, o6);
#pragma unroll
            for (int k = 0; k < 6; ++k) resid[r].v[b * 6 + k] = resid[r].v[b * 6 + k] - o6[k];
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (on[r]) vstore<S, A, NTX>(w[r], a.vout, site, acc[r]);
  }

  // ---- reductions over the values as stored: one block partial per slot of the group
  if (a.red == RED_NONE) return;
  double v[R * RED_NV];
#pragma unroll
  for (int k = 0; k < R * RED_NV; ++k) v[k] = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!valid || !on[r]) continue;
    Spinor<A> o;
    if (NTX)
      o = acc[r];
    else
      vload<S, A>(w[r], a.vout, site, o);
    if (a.red == RED_ALPHA) {  // (rhat, o)
      Spinor<A> rh;
      vload<S, A>(w[r], a.vrhat, site, rh);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        v[r * 3 + 0] += (double)rh.v[k].re * o.v[k].re + (double)rh.v[k].im * o.v[k].im;
        v[r * 3 + 1] += (double)rh.v[k].re * o.v[k].im - (double)rh.v[k].im * o.v[k].re;
      }
    } else if (a.red == RED_OMEGA) {  // (o, aux2), |o|^2
      Spinor<A> x2;
      vload<S, A>(w[r], a.vaux2, site, x2);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        v[r * 3 + 0] += (double)o.v[k].re * x2.v[k].re + (double)o.v[k].im * x2.v[k].im;
        v[r * 3 + 1] += (double)o.v[k].re * x2.v[k].im - (double)o.v[k].im * x2.v[k].re;
        v[r * 3 + 2] += (double)o.v[k].re * o.v[k].re + (double)o.v[k].im * o.v[k].im;
      }
    } else if (EPI == EPI_INV && std::is_same<S, double>::value && a.red == RED_RES_E) {  // |r_e|^2
#pragma unroll
      for (int k = 0; k < 12; ++k)
        v[r * 3] += (double)resid[r].v[k].re * resid[r].v[k].re + (double)resid[r].v[k].im * resid[r].v[k].im;
    } else {  // |o|^2
#pragma unroll
      for (int k = 0; k < 12; ++k) v[r * 3] += (double)o.v[k].re * o.v[k].re + (double)o.v[k].im * o.v[k].im;
    }
  }
  block_sum_n<R * RED_NV, BS>(v);
  if ((int)threadIdx.x < R * RED_NV) {
    const int r = threadIdx.x / RED_NV, k = threadIdx.x % RED_NV;
    if (grp[r] >= 0) {
      double val = 0.0;
#pragma unroll
      for (int q = 0; q < R * RED_NV; ++q)
        if (q == (int)threadIdx.x) val = v[q];
      store_partial(a.rb, a.slots[grp[r]].sid, tile.y, k, val);
    }
  }
}

template <class P, int R>
static void launch_hop_r(const HopArgs& a, int ntiles, hipStream_t s) {
  const bool clov = (a.vaux2 >= 0 && a.cb != 0.0);
  if (a.inv == 2)
    hipLaunchKernelGGL((k_hop<P, R, EPI_INVA>), dim3(ntiles), dim3(BS), 0, s, a);
  else if (a.inv)
    hipLaunchKernelGGL((k_hop<P, R, EPI_INV>), dim3(ntiles), dim3(BS), 0, s, a);
  else if (clov)
    hipLaunchKernelGGL((k_hop<P, R, EPI_CLOV>), dim3(ntiles), dim3(BS), 0, s, a);
  else
    hipLaunchKernelGGL((k_hop<P, R, EPI_PLAIN>), dim3(ntiles), dim3(BS), 0, s, a);
}

template <class P>
static void launch_hop_p(int R, const HopArgs& a, int ntiles, hipStream_t s) {
  switch (R) {
    case 1: launch_hop_r<P, 1>(a, ntiles, s); break;
    case 2: launch_hop_r<P, 2>(a, ntiles, s); break;
    case 4: launch_hop_r<P, 4>(a, ntiles, s); break;
    default: break;
  }
}

// FP64 stencils of the correction-form reliable update: inputs from the inner arena
template <int R, int LOM, typename SI>
static void launch_hop_lo_r(const HopArgs& a, int ntiles, hipStream_t s) {
  if (LOM == 1)
    hipLaunchKernelGGL((k_hop<PrecF64, R, EPI_INV, 1, SI>), dim3(ntiles), dim3(BS), 0, s, a);
  else
    hipLaunchKernelGGL((k_hop<PrecF64, R, EPI_CLOV, 2, SI>), dim3(ntiles), dim3(BS), 0, s, a);
}

template <typename SI>
static void launch_hop_lo_s(int R, const HopArgs& a, int ntiles, hipStream_t s) {
  const bool first = a.lo_mask == 1;
  if (R == 1) {
    if (first)
      launch_hop_lo_r<1, 1, SI>(a, ntiles, s);
    else
      launch_hop_lo_r<1, 2, SI>(a, ntiles, s);
  } else {
    if (first)
      launch_hop_lo_r<2, 1, SI>(a, ntiles, s);
    else
      launch_hop_lo_r<2, 2, SI>(a, ntiles, s);
  }
}

bool hop_lo_supports(int R, int lo_mask, int lo_prec, int inv, bool clov) {
  if (R != 1 && R != 2) return false;
  if (lo_prec < 1 || lo_prec > 3) return false;
  return (lo_mask == 1 && inv && !clov) || (lo_mask == 2 && !inv && clov);
}

void launch_hop(int prec, int R, const HopArgs& a, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return;
  if (a.lo_mask) {  // FP64 arithmetic, inner-arena inputs (checked by the caller with hop_lo_supports)
    if (prec != 0) return;
    switch (a.lo_prec) {
      case 1: launch_hop_lo_s<float>(R, a, ntiles, s); break;
      case 2: launch_hop_lo_s<_Float16>(R, a, ntiles, s); break;
      case 3: launch_hop_lo_s<bf16_t>(R, a, ntiles, s); break;
      default: break;
    }
    return;
  }
  switch (prec) {
    case 0: launch_hop_p<PrecF64>(R, a, ntiles, s); break;
    case 1: launch_hop_p<PrecF32>(R, a, ntiles, s); break;
    case 2: launch_hop_p<PrecF16>(R, a, ntiles, s); break;
    case 3: launch_hop_p<PrecB16>(R, a, ntiles, s); break;
    default: break;
  }
}

}  // namespace a2a
