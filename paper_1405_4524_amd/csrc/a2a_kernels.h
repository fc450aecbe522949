// a2a_kernels.h -- host-side declarations of the kernel launchers (internal to liba2a).
#pragma once

#include <hip/hip_runtime.h>

#include "a2a_device.h"
#include "a2a_reduce.h"

namespace a2a {

constexpr int BS = 256;  // threads per block; one site per thread

// Fused stencil kernel (Sec. 7 "inversion"): for every output site of parity out_par and
// every slot of a group
//   o = gam * (H in) + ca * aux1 + cb * (A_out aux2);  if inv: o = A_out^{-1} o
// with gam = gsign * kappa^gpow, then an optional reduction over o.
struct HopArgs {
  const OpDev* ops;
  const SlotDev* slots;
  const int* groups;  // [ngroups][R] slot ids, -1 = padding
  const int2* tiles;  // {group, site block}
  int out_par;
  int psel;           // 0: inner precision fields/arena, 1: FP64
  int vin, vout, vaux1, vaux2;
  int vrhat;          // for RED_ALPHA: the shadow vector (inner arena)
  double ca, cb, gsign;
  int gpow;
  int inv;
  int red;
  int brick;          // site blocks are 4D bricks (several RHS groups per block), else linear
  int by, bz, bt;     // brick extents of this launch (0: the operator's; ignored unless they tile it)
  // FP64 stencils only: 1 = vin, 2 = vaux2 is the slot's inner (low-precision) vector, in the
  // inner storage lo_prec (1 FP32, 2 FP16, 3 BF16), times the slot's scale sigma
  int lo_mask, lo_prec;
  RedBuf rb;
};

// Matrix-core stencil for lane-interleaved groups (FP16 / BF16 inner vectors).
constexpr int IL_LANES = 48;  // RHS per interleaved group (three tiles of 16 lanes)

struct ILGroupDev {
  int op;
  int nt;                  // lane tiles in use
  char* base;             // arena: [vector][site][tile][3 chunks][16 lanes] of 16-byte chunks
  long long vs;           // bytes per vector
  int slot[IL_LANES];     // slot-table index of each lane, -1 = idle
};

struct HopMArgs {
  const OpDev* ops;
  const SlotDev* slots;
  const ILGroupDev* groups;
  const int2* tiles;  // {group, site block of BS sites}
  int out_par;
  int vin, vout, vaux1, vaux2, vrhat;
  double ca, cb, gsign;
  int gpow;
  int red;
  int nt3;  // every group of the launch has three lane tiles (48-lane groups)
  RedBuf rb;
};

// Site-local / vector kernels over per-slot tiles {slot, site block}.
enum VecKind {
  VK_BICG_S = 0,    // s = r - alpha v
  VK_BICG_XR,       // x += alpha p + omega s; r = s - omega t; (rhat, r), |r|^2 -> RED_RHO
  VK_BICG_P,        // p = r + beta (p - omega v)
  VK_RU_ACCUM,      // x64 += sigma x_lo; x_lo = 0
  VK_RU_RESCALE,    // r_lo = r64/sigma'; p, v *= sigma/sigma'; (rhat, r_lo) -> RED_RU
  VK_INIT,          // r_lo = r64/sigma; rhat = p = r_lo; v = x_lo = 0 -> RED_INIT
  VK_CLOVER,        // out = C in  (FP64 arena, C = A or A^{-1} of a parity)
  VK_ZERO_HI,       // hi[vout] = 0
  VK_ZERO_LO,       // lo[vout] = 0
  VK_FILL_LO,       // lo[vout] = deterministic pseudo-random values (benchmarks)
  VK_ZERO_X,        // inner x = 0
  // CG on the normal equations, iterating r' = gamma5 r (so that M^dag r = gamma5 M r')
  VK_CG_XR,         // x += alpha p; r' -= alpha gamma5 q; |r'|^2 -> RED_CG_R
  VK_CG_P,          // p = gamma5 u + beta p  (u = M r')
  VK_CG_INIT,       // r' = gamma5 r64/sigma; p = x_lo = 0 -> RED_CG_INIT
  VK_CG_RESCALE,    // r' = gamma5 r64/sigma'; p *= sigma/sigma' -> RED_CG_RU
  VK_COPY_HI,       // hi[vout] = hi[vin]
};

struct VecArgs {
  const OpDev* ops;
  const SlotDev* slots;
  const int2* tiles;     // per-slot mapping: {slot, site block}; interleaved: {lane tile, site block}
  const int* ilslots;    // interleaved mapping: 16 slot indices per lane tile (-1 = idle lane)
  int kind;
  int par;        // parity for VK_CLOVER
  int use_inv;    // VK_CLOVER: 1 -> A^{-1}
  int vin, vout;  // VK_CLOVER / VK_ZERO_HI / VK_COPY_HI; vin >= 0: FP64 residual source of the INIT / RESCALE kinds
  RedBuf rb;
};

// canonical complex128 [site][spin][colour] <-> even-odd chunked vectors
struct LayoutArgs {
  const OpDev* ops;
  const SlotDev* slots;
  const int2* tiles;
  int which_in;    // layout_in: 0 reads the slot's source, 1 its initial guess
  int psel;        // arena / precision of the eo vectors
  int v_even, v_odd;
  int gamma5;      // multiply by gamma_5 on the way
  int red;         // RED_ETA or RED_NONE (|in|^2 over both parities)
  RedBuf rb;
};

// Sum the block partials of `kind` for n slots (slot table indices from `list`, or 0..n-1
// when list is null) in block order and apply the scalar update.  Must follow the reducing
// launch on the same stream.
void launch_finalize(int kind, const OpDev* ops, const SlotDev* slots, const int* list, int n, RedBuf rb,
                     hipStream_t s);

void launch_hop(int prec, int R, const HopArgs& a, int ntiles, hipStream_t s);
// the FP64 correction-form variants (HopArgs::lo_mask): first stencil EPI_INV with the hopping
// input from the inner arena, second EPI_CLOV with the clover input from it; R = 1 or 2
bool hop_lo_supports(int R, int lo_mask, int lo_prec, int inv, bool clov);
// o = gam H in (+ cb A aux2) (then A^{-1} .) for every lane of the groups, on the matrix
// cores; reduction kinds NONE, ALPHA and OMEGA (with the clover term); no axpy term
bool hop_mfma_supports(int prec, int inv, bool clov, int red, bool aux1);
void launch_hop_mfma(int prec, const HopMArgs& a, int ntiles, int inv, bool clov, hipStream_t s);
void launch_vec(int prec, const VecArgs& a, int ntiles, hipStream_t s);
// the lane-interleaved variant (FP16 / BF16 inner vectors in interleaved groups); kinds that
// touch inner vectors only
void launch_vec_il(int prec, const VecArgs& a, int ntiles, hipStream_t s);
bool vec_kind_il(int kind);
void launch_layout_in(int prec, const LayoutArgs& a, int ntiles, hipStream_t s);
void launch_layout_out(int prec, const LayoutArgs& a, int ntiles, hipStream_t s);

// gauge field: canonical complex128 [site][mu][3][3] -> per-parity link fields
void launch_gauge_to_eo(int prec, const Geo& g, const double* canon, void* const dst[2], hipStream_t s);
// kappa-independent clover field G (FP64 packed, per parity) from canonical links
void launch_clover_field(const Geo& g, const double* canon_links, double* G[2], hipStream_t s);
// A = 1 + kappa c_sw G per parity in FP64, plus its per-block inverse (FP64)
void launch_clover_make(const Geo& g, const double* G, double kcsw, double* A, double* Ainv, hipStream_t s);
// per-site hop links (both directions, boundary sign folded in) of one parity, 16-bit formats
void launch_hop_links(int prec, const Geo& g, const double* canon, int par, void* dst, hipStream_t s);
// packed FP64 clover blocks -> full 6x6 blocks in a 16-bit format
void launch_clover_full(int prec, long hv, const double* packed, void* dst, hipStream_t s);
// precision conversion of a packed clover field
void launch_clover_convert(int prec, long hv, const double* src, void* dst, hipStream_t s);

// counter-hash complex Z2 noise into canonical layout
void launch_z2_noise(long V, int nsrc, unsigned long long seed, long long src_offset, double* out, hipStream_t s);

}  // namespace a2a
