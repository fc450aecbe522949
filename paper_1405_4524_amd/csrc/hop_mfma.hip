// hop_mfma.hip -- the Wilson-clover hopping stencil on the matrix cores for lane-interleaved
// groups of right-hand sides (FP16 or BF16 storage, FP32 accumulation).
//
// At one output site x the hopping term H (the sum over the eight neighbours in the
// hopping-parameter form of the Wilson-clover operator, Sec. 7) is a real 24 x 192 matrix
// acting on the eight neighbour spinors stacked as 8 x 24 reals: block d = 2 mu + f of the
// matrix is the real form of (1 -+ gamma_mu) (x) V_d with V_d the site's hop link of
// direction d (the link, or the daggered backward link, with the fermion boundary sign).
// Every RHS of a group sees the same matrix, so one wavefront takes one site at a time and
// multiplies the matrix with the 192 x 16 block of neighbour data of each 16-lane tile on the
// matrix cores: v_mfma_f32_16x16x32 over 2 row tiles (24 rows + 8 unused) x 6 K steps.  The
// clover term A_x psi(x) is one more K step (24 columns + 8 zero columns).  The inverse-clover
// epilogue is a second product after a register -> LDS -> register transpose of the hop result
// (which rounds that intermediate to the storage format).  Calls with an axpy term (aux1) use
// the per-thread stencil.
//
// The matrix is rebuilt per site in LDS by the 64 lanes of the wave: lane (d, s, c') writes
// the three row blocks (colour a = 0..2) of its direction d for output spin s and real /
// imaginary part c'.  Each entry is the real or imaginary part of a link element, possibly
// swapped and negated; which one is fixed per lane and selected once before the site loop.
// Half of the entries are zero (the spin projector has two non-zero entries per row) and are
// written once; the per-site build writes only the other half (7% faster Schur operator).
//
// Layout of one wavefront's LDS matrix: 24 rows of 464 bytes = 232 halves: columns 0..191
// the hopping blocks (d, spin s', colour b, re/im), 192..215 the clover block, 216..231 zero.
// Rows are 464 B apart so that the 16-byte fragment reads of 16 consecutive rows fall on
// distinct banks.
#include <type_traits>

#include "a2a_kernels.h"

namespace a2a {

namespace {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename S>
struct MM;

template <>
struct MM<_Float16> {
  static __device__ __forceinline__ f4v mma(const uint4& a, const uint4& b, const f4v& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0, 0,
                                                  0);
  }
  static __device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    const _Float16 a = (_Float16)lo, b = (_Float16)hi;
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
  }
  static __device__ __forceinline__ float lo(uint32_t u) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(u & 0xffffu));
  }
  static __device__ __forceinline__ float hi(uint32_t u) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(u >> 16)); }
};

template <>
struct MM<bf16_t> {
  static __device__ __forceinline__ f4v mma(const uint4& a, const uint4& b, const f4v& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8v, a), __builtin_bit_cast(b8v, b), c, 0, 0,
                                                   0);
  }
  static __device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    return (uint32_t)float_to_bf16(lo).v | ((uint32_t)float_to_bf16(hi).v << 16);
  }
  static __device__ __forceinline__ float lo(uint32_t u) { return bf16_to_float(bf16_t{(uint16_t)(u & 0xffffu)}); }
  static __device__ __forceinline__ float hi(uint32_t u) { return bf16_to_float(bf16_t{(uint16_t)(u >> 16)}); }
};

constexpr int WAVES = BS / 64;
constexpr int SITES_PER_WAVE = BS / WAVES;  // a block covers BS sites, like every reducing kernel
constexpr int TROW = 29;                    // uint4 per matrix row (464 B)
constexpr int TCLO = 24;                    // uint4 column of the clover K step (half 192)
constexpr int TRW = 5;                      // uint4 per transpose row (80 B)
constexpr int NTMAX = IL_LANES / 16;        // lane tiles per group

__device__ __forceinline__ uint32_t rot16(uint32_t v) { return (v >> 16) | (v << 16); }

// Pointers read from the group and operator tables are generic; accesses through them would be
// FLAT instructions, which count against the LDS counter too and so make every LDS wait also
// wait for outstanding HBM traffic.  All of these fields point to device global memory.
typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) uint32_t* gptr1;
typedef const __attribute__((address_space(1))) v2u* gptr2;
typedef const __attribute__((address_space(1))) v4u* gptr4;
__device__ __forceinline__ uint32_t gld1(const void* p) { return *(gptr1)p; }
__device__ __forceinline__ uint2 gld2(const void* p) {
  const v2u v = *(gptr2)p;
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint4 gld4(const void* p) {
  const v4u v = *(gptr4)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
// single-use operands (the site's own aux / shadow chunks, the output): streaming access
__device__ __forceinline__ uint4 gld4nt(const void* p) {
  const v4u v = __builtin_nontemporal_load((gptr4)p);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gst4nt(void* p, const uint4& v) {
  v4u w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  __builtin_nontemporal_store(w, (__attribute__((address_space(1))) v4u*)p);
}
__device__ __forceinline__ void gst4(void* p, const uint4& v) {
  v4u w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  *(__attribute__((address_space(1))) v4u*)p = w;
}
__device__ __forceinline__ void gst2(void* p, const uint2& v) {
  v2u w;
  w.x = v.x;
  w.y = v.y;
  *(__attribute__((address_space(1))) v2u*)p = w;
}

// (1 + sg gamma_mu)[s][t] in the chiral basis as a unit complex (re, im), entries in {-1, 0, 1}.
// gamma_mu = [[0, a_mu], [a_mu^dag, 0]] with a_k = -i sigma_k (mu = 0, 1, 2) and a_4 = 1.
__device__ __forceinline__ void proj_entry(int mu, int sg, int s, int t, int& re, int& im) {
  re = 0;
  im = 0;
  if (s == t) {
    re = 1;
    return;
  }
  if ((s < 2) == (t < 2)) return;
  const int u = s < 2 ? s : t, v = s < 2 ? t - 2 : s - 2;  // entry a[u][v] (conjugated below the diagonal)
  int ar = 0, ai = 0;
  if (mu == 0) {
    if (u != v) ai = -1;  // -i sigma_1
  } else if (mu == 1) {
    if (u == 0 && v == 1) ar = -1;  // -i sigma_2
    if (u == 1 && v == 0) ar = 1;
  } else if (mu == 2) {
    if (u == v) ai = u == 0 ? -1 : 1;  // -i sigma_3
  } else {
    if (u == v) ar = 1;
  }
  if (s >= 2) ai = -ai;
  re = sg * ar;
  im = sg * ai;
}

// Real-form row c' of (P v) for a unit complex P and a link element v = (vr, vi) packed as two
// 16-bit halves: c' = 0 gives (Re Pv, -Im Pv), c' = 1 gives (Im Pv, Re Pv).  All eight cases
// are one of (vr,-vi), (vi,vr), (-vr,vi), (-vi,-vr): a byte permutation (identity, half swap,
// or all-zero for a vanishing projector entry) and a sign mask.
struct Variant {
  uint32_t sel, xm;
};
__device__ __forceinline__ Variant variant(int re, int im, int cp) {
  int T = -1;
  if (re == 1) T = cp ? 1 : 0;
  if (re == -1) T = cp ? 3 : 2;
  if (im == 1) T = cp ? 0 : 3;
  if (im == -1) T = cp ? 2 : 1;
  Variant r;
  r.sel = T < 0 ? 0x0c0c0c0cu : (T == 1 || T == 3) ? 0x01000302u : 0x03020100u;
  r.xm = T == 0 ? 0x80000000u : T == 2 ? 0x00008000u : T == 3 ? 0x80008000u : 0u;
  return r;
}
__device__ __forceinline__ uint32_t apply(const Variant& V, uint32_t v) {
  return __builtin_amdgcn_perm(v, v, V.sel) ^ V.xm;
}

// LDS traffic of one wavefront is executed in issue order, so lanes of the same wave see each
// other's LDS writes without waiting on any counter; only the compiler must keep the order.
__device__ __forceinline__ void wave_lds_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

}  // namespace

// Data one 16-lane tile (nt) of one site needs, each as the lane's 16 bytes in the B-fragment layout
// (chunk gq of its RHS; lanes gq = 3 repeat chunk 0): the six K steps of neighbour data, the
// clover input (EPI_CLOV) and the other operand of the ALPHA reduction (OMEGA's is the clover
// input).  One 16-byte load per lane and operand keeps the count of memory instructions, which
// is what the address units spend their cycles on, low.
struct TileIn {
  int nt;
  uint4 SD;  // this lane's 16 bytes of the site's links (lanes 0..17) and clover (18..35)
  uint4 B[6];
  uint4 Bc;
  uint4 Bx;
  int site;
};

template <int EPI, int RED>
__device__ __forceinline__ void load_tile(TileIn& d, const char* vin, const char* vaux2, const char* vrh,
                                          const int (&nbs)[6], const int (&hoff)[6], int site, int NT, int nt,
                                          int n, int gq) {
#pragma unroll
  for (int kt = 0; kt < 6; ++kt) d.B[kt] = gld4(vin + ((long long)nbs[kt] * NT + nt) * 768 + hoff[kt]);
  const long long own = ((long long)site * NT + nt) * 768 + (gq < 3 ? gq : 0) * 256 + n * 16;
  if (EPI == 1 || EPI == 3) d.Bc = gld4nt(vaux2 + own);
  if (RED == RED_ALPHA) d.Bx = gld4nt(vrh + own);
}

// cb indices of the neighbour site each lane's chunk of K step kt comes from: chunk 4 kt + gq
// belongs to direction d = (4 kt + gq) / 3, d = 2 mu + f (f = 0 forward, 1 backward)
__device__ __forceinline__ void site_neighbours(const Geo& g, int site, int po, int gq, int (&nbs)[6]) {
  int c[4];
  cb_coords(g, site, po, c);
  const int xh = c[0] >> 1, x = c[0], y = c[1], z = c[2], t = c[3];
  const int sy = g.Xh, sz = g.Xh * g.Y, st = g.Xh * g.Y * g.Z;
  const int row = site - xh;
  int nb[8];
  nb[0] = row + ((x + 1 == g.X ? 0 : x + 1) >> 1);
  nb[1] = row + ((x == 0 ? g.X - 1 : x - 1) >> 1);
  nb[2] = site + (y == g.Y - 1 ? -(g.Y - 1) * sy : sy);
  nb[3] = site + (y == 0 ? (g.Y - 1) * sy : -sy);
  nb[4] = site + (z == g.Z - 1 ? -(g.Z - 1) * sz : sz);
  nb[5] = site + (z == 0 ? (g.Z - 1) * sz : -sz);
  nb[6] = site + (t == g.T - 1 ? -(g.T - 1) * st : st);
  nb[7] = site + (t == 0 ? (g.T - 1) * st : -st);
  nbs[0] = gq >= 3 ? nb[1] : nb[0];
  nbs[1] = gq >= 2 ? nb[2] : nb[1];
  nbs[2] = gq >= 1 ? nb[3] : nb[2];
  nbs[3] = gq >= 3 ? nb[5] : nb[4];
  nbs[4] = gq >= 2 ? nb[6] : nb[5];
  nbs[5] = gq >= 1 ? nb[7] : nb[6];
}

// A block takes all lane tiles of a group over BS sites (64 per wave) of a 4D brick of the
// lattice (the whole x row, then y, z, t extents), so that most neighbours of a block's sites
// are sites of the same block; bricks follow in lexicographic order.  A wave's items are
// (site, lane tile) pairs, tiles inner: the site's matrix is built once and applied to every
// tile of the group (one build per site instead of one per site and tile: 10% faster Schur
// operator at 48 RHS, results bitwise unchanged).  Inside a brick the sweep runs y fastest,
// then x, then z and t: the waves of a block take (z, t) planes of the brick at the same
// (x, y) positions, so that a neighbour spinor is used by the z and t neighbours of other
// waves at about the same time, by its y neighbours two positions apart and by its x
// neighbours a few positions apart, while it is still in the L2 (x fastest put the y uses a
// whole row apart and cost a quarter more L2 misses).  Blocks are not grouped by XCD.  The
// links, clover and neighbour data of item i + 2 are requested while item i is computed (a ring
// of three register buffers), and the matrix fragments are read from LDS right before their
// products.

template <class P, int EPI, int RED, bool NT3>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_hop_mfma(HopMArgs a) {
  using S = typename P::S;
  using M = MM<S>;
  __shared__ uint4 tbl[WAVES][24][TROW];  // the site's matrix
  __shared__ uint4 stg[WAVES][64];        // the site's links (chunks 0..17) and clover (18..35)
  __shared__ uint4 trb[WAVES][16][TRW];   // register-layout transposes, one row per RHS lane

  const int2 tile = a.tiles[blockIdx.x];  // {group, site block}
  const ILGroupDev& grp = a.groups[tile.x];
  const OpDev& op = a.ops[grp.op];
  const Geo g = op.g;
  const int hv = g.hv;
  const int NT = grp.nt;
  const int po = a.out_par;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = lane & 15, gq = lane >> 4;
  uint4(*T)[TROW] = tbl[w];
  uint2* tr2 = (uint2*)&trb[w][n][0];  // this lane's transpose row as 8-byte pieces

  // ---- lane constants: matrix-building role (d, s, c') and the four spin-column variants
  const int bd = lane & 7, bs = (lane >> 3) & 3, bc = lane >> 5;
  Variant var[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    int re, im;
    proj_entry(bd >> 1, (bd & 1) ? 1 : -1, bs, t, re, im);
    var[t] = variant(re, im, bc);
  }
  // Each row of (1 -+ gamma_mu) has two non-zero entries: the diagonal (spin s' = s) and one
  // partner spin p2 in the other chiral block.  Only those two column triplets of a row block
  // are ever written; the other entries keep the zeros written once below.
  int p2 = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    int re, im;
    proj_entry(bd >> 1, (bd & 1) ? 1 : -1, bs, t, re, im);
    if (t != bs && (re != 0 || im != 0)) p2 = t;
  }
  Variant var_d = var[0], var_p = var[0];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t == bs) var_d = var[t];
    if (t == p2) var_p = var[t];
  }
  // clover-building role: row o, column half h (lanes 48..63 repeat lanes 0..15: same values)
  const int co = (lane >> 1) % 24, ch = lane & 1;
  const int cs = co / 6, ca_ = (co % 6) >> 1, ccp = co & 1;
  const int cblk = cs >> 1, ci = 3 * cs + ca_ - 6 * cblk;
  const int cdw = 72 + (cblk * 6 + ci) * 6;  // staged dword of the row's six block entries
  // fragment rows (rows 24..31 of the second row tile read valid rows; their outputs are unused)
  const int frow0 = n, frow1 = n + 16 < 24 ? n + 16 : n + 8;
  int hoff[6];
#pragma unroll
  for (int t = 0; t < 6; ++t) hoff[t] = ((4 * t + gq) % 3) * 256 + n * 16;
  const int ochunk = gq < 3 ? gq : 0;  // the chunk this lane loads / stores (gq = 3 repeats 0)

  double kp = 1.0;
  for (int i = 0; i < a.gpow; ++i) kp *= op.kappa;
  const float gam = (float)(a.gsign * kp);
  const float cbv = (float)a.cb;

  const char* hl = (const char*)op.HL[po];
  const char* cf = (const char*)(EPI >= 2 ? op.AIF[po] : op.AF[po]);
  const long long vs = grp.vs;
  const char* vin = grp.base + (long long)a.vin * vs;
  char* vout = grp.base + (long long)a.vout * vs;
  const char* vaux2 = a.vaux2 >= 0 ? grp.base + (long long)a.vaux2 * vs : nullptr;
  const char* vrh = a.vrhat >= 0 ? grp.base + (long long)a.vrhat * vs : nullptr;

  int myslot[NTMAX];
#pragma unroll
  for (int t = 0; t < NTMAX; ++t) myslot[t] = (int)gld1(&grp.slot[t * 16 + n]);
  float red[NTMAX][3];
#pragma unroll
  for (int t = 0; t < NTMAX; ++t) red[t][0] = red[t][1] = red[t][2] = 0.f;

  // zero the matrix once: the padding columns stay zero
  for (int e = lane; e < 24 * TROW; e += 64) (&T[0][0])[e] = make_uint4(0, 0, 0, 0);
  wave_lds_sync();

  const int s0 = tile.y * BS + w * SITES_PER_WAVE;
  const int cnt = s0 < hv ? (hv - s0 < SITES_PER_WAVE ? hv - s0 : SITES_PER_WAVE) : 0;
  const int items = cnt * NT;  // items (site, lane tile), tiles inner

  // a site's links and clover: 36 chunks of 16 bytes, one per lane (lanes 36.. repeat)
  const int sdl = lane < 36 ? lane : lane - 36;
  const bool sd_clover = EPI != 0 && sdl >= 18;
  const char* sd_base = sd_clover ? cf + (sdl - 18) * 16 : hl + (sdl % 18) * 16;
  auto build = [&](const uint4& SD) {
    stg[w][lane] = SD;
    wave_lds_sync();
    const uint32_t* st32 = (const uint32_t*)&stg[w][0];
    uint32_t L[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) L[j] = st32[bd * 9 + j];
#pragma unroll
    for (int ca = 0; ca < 3; ++ca) {  // the non-zero triplets (s' = s and s' = p2) of the row block
      uint32_t* row = (uint32_t*)&T[6 * bs + 2 * ca + bc][bd * 3];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        row[3 * bs + b] = apply(var_d, L[ca * 3 + b]);
        row[3 * p2 + b] = apply(var_p, L[ca * 3 + b]);
      }
    }
    if (EPI != 0) {
      uint32_t o[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const uint32_t c = st32[cdw + j];
        o[j] = ccp ? rot16(c) : (c ^ 0x80000000u);
      }
      uint2* dst = (uint2*)((char*)&T[co][TCLO] + 24 * ch);
      if (ch == cblk) {  // the other chiral block's half stays zero
        dst[0] = make_uint2(o[0], o[1]);
        dst[1] = make_uint2(o[2], o[3]);
        dst[2] = make_uint2(o[4], o[5]);
      }
    }
  };

  // prefetch cursor: site pk
  int pk = 0;
  auto site_at = [&](int p) { return __builtin_amdgcn_readfirstlane(brick_site<true>(g, p)); };
  // Loads and stores in the sweep are unconditional (positions past the wave's range are clamped
  // to its last site, whose values are then recomputed and rewritten unchanged), so the number
  // of memory operations in flight is the same on every path and the waits on them stay exact.
  // With three tiles per group the ring buffer of an item is its tile (items are (site, tile)
  // pairs, tiles inner, three buffers), so only buffer 0 takes the site's links and clover:
  // one load per site instead of one per item.
  auto prefetch = [&](TileIn& dst, auto with_sd) {
    const int p = pk < items ? pk : items - 1;
    const int ntp = __builtin_amdgcn_readfirstlane(p % NT);
    const int site = site_at(s0 + p / NT);
    dst.site = site;
    dst.nt = ntp;
    if (decltype(with_sd)::value) dst.SD = gld4(sd_base + (size_t)site * 288);
    int nbs_p[6];
    site_neighbours(g, site, po, gq, nbs_p);
    load_tile<EPI, RED>(dst, vin, vaux2, vrh, nbs_p, hoff, site, NT, ntp, n, gq);
    ++pk;
  };
  // compute cursor: site ck
  int ck = 0;
  auto step = [&](TileIn& cur, TileIn& pf, auto may_build, auto pf_sd) {
    const int site = cur.site;
    const int nt = cur.nt;
    const bool live = ck < items;
    if (decltype(may_build)::value && nt == 0) build(cur.SD);  // this site's matrix, once for all its tiles
    prefetch(pf, pf_sd);
    __builtin_amdgcn_sched_barrier(0);  // keep the requests ahead of this item's work
    wave_lds_sync();
    f4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 6; ++kt) {
      acc0 = M::mma(T[frow0][4 * kt + gq], cur.B[kt], acc0);
      acc1 = M::mma(T[frow1][4 * kt + gq], cur.B[kt], acc1);
    }
    float v0[4], v1[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v0[r] = gam * acc0[r];
      v1[r] = gam * acc1[r];
    }
    if (EPI == 1) {
      const f4v zero = {0.f, 0.f, 0.f, 0.f};
      const f4v c0 = M::mma(T[frow0][TCLO + gq], cur.Bc, zero), c1 = M::mma(T[frow1][TCLO + gq], cur.Bc, zero);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v0[r] += cbv * c0[r];
        v1[r] += cbv * c1[r];
      }
    }
    if (EPI == 2 || EPI == 3) {  // o = A^{-1} (.): transpose the rounded result through LDS, second product
      tr2[gq] = make_uint2(M::pack2(v0[0], v0[1]), M::pack2(v0[2], v0[3]));
      tr2[4 + gq] = gq < 2 ? make_uint2(M::pack2(v1[0], v1[1]), M::pack2(v1[2], v1[3])) : make_uint2(0, 0);
      wave_lds_sync();
      const uint4 B2 = trb[w][n][gq];
      wave_lds_sync();
      const f4v zero = {0.f, 0.f, 0.f, 0.f};
      const f4v c0 = M::mma(T[frow0][TCLO + gq], B2, zero), c1 = M::mma(T[frow1][TCLO + gq], B2, zero);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v0[r] = c0[r];
        v1[r] = c1[r];
      }
    }
    if (EPI == 3) {  // o = aux2 + A^{-1} (.): the site's aux2 chunk to output rows through LDS
      trb[w][n][gq] = cur.Bc;
      wave_lds_sync();
      const uint2 a0 = tr2[gq], a1 = tr2[4 + gq];
      wave_lds_sync();
      v0[0] += M::lo(a0.x);
      v0[1] += M::hi(a0.x);
      v0[2] += M::lo(a0.y);
      v0[3] += M::hi(a0.y);
      v1[0] += M::lo(a1.x);
      v1[1] += M::hi(a1.x);
      v1[2] += M::lo(a1.y);
      v1[3] += M::hi(a1.y);
    }
    // rows 16 m + 4 gq .. +3 of row tile m, rounded to the storage format
    const uint2 q0 = make_uint2(M::pack2(v0[0], v0[1]), M::pack2(v0[2], v0[3]));
    const uint2 q1 = make_uint2(M::pack2(v1[0], v1[1]), M::pack2(v1[2], v1[3]));
    if (RED == RED_ALPHA || RED == RED_OMEGA) {  // over the values as stored
      trb[w][n][gq] = RED == RED_ALPHA ? cur.Bx : cur.Bc;  // the partner, to output rows
      wave_lds_sync();
      const uint2 xr0 = tr2[gq], xr1 = tr2[4 + gq];
      wave_lds_sync();
      float r0 = 0.f, r1 = 0.f, r2 = 0.f;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        if (m == 1 && gq >= 2) continue;
        const uint2 q = m ? q1 : q0;
        const uint2 x = m ? xr1 : xr0;
        const float o0 = M::lo(q.x), o1 = M::hi(q.x), o2 = M::lo(q.y), o3 = M::hi(q.y);
        const float x0 = M::lo(x.x), x1 = M::hi(x.x), x2 = M::lo(x.y), x3 = M::hi(x.y);
        if (RED == RED_ALPHA) {  // (rhat, o)
          r0 += x0 * o0 + x1 * o1 + x2 * o2 + x3 * o3;
          r1 += x0 * o1 - x1 * o0 + x2 * o3 - x3 * o2;
        } else {  // (o, aux2), |o|^2
          r0 += o0 * x0 + o1 * x1 + o2 * x2 + o3 * x3;
          r1 += o0 * x1 - o1 * x0 + o2 * x3 - o3 * x2;
          r2 += o0 * o0 + o1 * o1 + o2 * o2 + o3 * o3;
        }
      }
      // a select, not a product with 0 or 1: an idle lane's column holds whatever its memory
      // held, and 0 * NaN would reach the partial sums of the same lane in the other tiles
#pragma unroll
      for (int t = 0; t < NTMAX; ++t) {
        const bool keep = live && t == nt && myslot[t] >= 0;
        red[t][0] += keep ? r0 : 0.f;
        red[t][1] += keep ? r1 : 0.f;
        red[t][2] += keep ? r2 : 0.f;
      }
    }
    // to the storage layout through LDS: one 16-byte store per lane (idle lanes write their own
    // unread lane slots; lanes gq = 3 repeat the chunk-0 store of lane gq = 0)
    tr2[gq] = q0;
    tr2[4 + gq] = q1;
    wave_lds_sync();
    const uint4 ob = trb[w][n][ochunk];
    wave_lds_sync();
    gst4nt(vout + ((long long)site * NT + nt) * 768 + ochunk * 256 + n * 16, ob);
    ++ck;
  };

  if (items > 0) {
    TileIn R0, R1, R2;
    using yes = std::true_type;
    using tile0 = std::integral_constant<bool, !NT3>;  // buffers 1 and 2 hold tiles 1 and 2
    prefetch(R0, yes{});
    prefetch(R1, tile0{});
    for (int i = 0; i < items; i += 3) {
      step(R0, R2, yes{}, tile0{});
      step(R1, R0, tile0{}, yes{});
      step(R2, R1, tile0{}, tile0{});
    }
  }

  if (RED == RED_ALPHA || RED == RED_OMEGA) {
    __syncthreads();  // every wave is done with its matrix: reuse the LDS as scratch
    double* scr = (double*)&tbl[0][0][0];  // [tile][wave][lane][3]
#pragma unroll
    for (int t = 0; t < NTMAX; ++t)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        double x = (double)red[t][q];
        x += __shfl_xor(x, 16, 64);
        x += __shfl_xor(x, 32, 64);
        if (lane < 16) scr[((t * WAVES + w) * 16 + lane) * 3 + q] = x;
      }
    __syncthreads();
    if (threadIdx.x < 48 * NTMAX) {
      const int t = threadIdx.x / 48, m = (threadIdx.x / 3) % 16, q = threadIdx.x % 3;
      const int sl = t < NT ? grp.slot[t * 16 + m] : -1;
      if (sl >= 0) {
        double sum = 0.0;
#pragma unroll
        for (int j = 0; j < WAVES; ++j) sum += scr[((t * WAVES + j) * 16 + m) * 3 + q];
        store_partial(a.rb, a.slots[sl].sid, tile.y, q, sum);
      }
    }
  }
}

template <class P, bool NT3>
static void launch_mfma_nt(const HopMArgs& a, int ntiles, int epi, hipStream_t s) {
  const dim3 g(ntiles), b(BS);
  if (epi == 3) {
    if (a.red == RED_ALPHA)
      hipLaunchKernelGGL((k_hop_mfma<P, 3, RED_ALPHA, NT3>), g, b, 0, s, a);
    else if (a.red == RED_OMEGA)
      hipLaunchKernelGGL((k_hop_mfma<P, 3, RED_OMEGA, NT3>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((k_hop_mfma<P, 3, RED_NONE, NT3>), g, b, 0, s, a);
  } else if (epi == 2) {
    hipLaunchKernelGGL((k_hop_mfma<P, 2, RED_NONE, NT3>), g, b, 0, s, a);
  } else if (epi == 1) {
    if (a.red == RED_ALPHA)
      hipLaunchKernelGGL((k_hop_mfma<P, 1, RED_ALPHA, NT3>), g, b, 0, s, a);
    else if (a.red == RED_OMEGA)
      hipLaunchKernelGGL((k_hop_mfma<P, 1, RED_OMEGA, NT3>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((k_hop_mfma<P, 1, RED_NONE, NT3>), g, b, 0, s, a);
  } else {
    hipLaunchKernelGGL((k_hop_mfma<P, 0, RED_NONE, NT3>), g, b, 0, s, a);
  }
}

template <class P>
static void launch_mfma_p(const HopMArgs& a, int ntiles, int epi, hipStream_t s) {
  if (a.nt3)
    launch_mfma_nt<P, true>(a, ntiles, epi, s);
  else
    launch_mfma_nt<P, false>(a, ntiles, epi, s);
}

bool hop_mfma_supports(int prec, int inv, bool clov, int red, bool aux1) {
  if ((prec != 2 && prec != 3) || aux1) return false;
  if (inv == 2) return red == RED_NONE || red == RED_ALPHA || red == RED_OMEGA;
  if (inv) return red == RED_NONE;
  if (clov) return red == RED_NONE || red == RED_ALPHA || red == RED_OMEGA;
  return red == RED_NONE;
}

void launch_hop_mfma(int prec, const HopMArgs& a, int ntiles, int inv, bool clov, hipStream_t s) {
  if (ntiles <= 0) return;
  const int epi = inv == 2 ? 3 : inv ? 2 : clov ? 1 : 0;
  if (prec == 2) launch_mfma_p<PrecF16>(a, ntiles, epi, s);
  if (prec == 3) launch_mfma_p<PrecB16>(a, ntiles, epi, s);
}

}  // namespace a2a
