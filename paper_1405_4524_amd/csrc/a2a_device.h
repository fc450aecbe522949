// a2a_device.h -- device-side types for the even-odd clover-Wilson path on gfx950.
//
// Data layout in HBM (all per parity, "checkerboard" site index cb):
//   cb = ((t*Z + z)*Y + y)*(X/2) + x/2,   parity p = (x+y+z+t) & 1
//   a field with NR reals per site is stored as NCH planes of 16/8/4-byte chunks,
//   plane k holding chunk k of every site contiguously ([NCH][hv] chunks), so a
//   wavefront that reads one chunk of 64 consecutive sites issues one coalesced
//   512 B / 1 KiB transaction.
//     spinor  : 24 reals  (spin s, colour c -> complex index s*3+c)
//     link    : 18 reals  per direction mu; a parity's links are 4 such fields (mu = 0..3)
//     clover  : 72 reals  two Hermitian 6x6 blocks (chiral halves, spins {0,1} and {2,3}),
//               each packed as 6 real diagonals followed by the 15 complex entries of
//               the strictly lower triangle in row order (1,0),(2,0),(2,1),(3,0),...,(5,4)
//
// Operator (hopping-parameter form of the Wilson-clover "lattice fermion matrix", Sec. 7;
// c_SW of Sec. 8):  D = A - kappa H, with the chiral gamma basis
//   gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 = [[0, 1], [1, 0]], gamma_5 = diag(1,1,-1,-1)
//   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)
// and the fermion time-boundary sign on hops that wrap in t.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HD __host__ __device__ __forceinline__

namespace a2a {

// ------------------------------------------------------------------------------------
// storage precisions
// ------------------------------------------------------------------------------------
struct bf16_t {
  uint16_t v;
};

HD float bf16_to_float(bf16_t h) {
  uint32_t u = ((uint32_t)h.v) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

HD bf16_t float_to_bf16(float f) {  // round to nearest even (NaN kept quiet)
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  bf16_t r;
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    r.v = (uint16_t)((u >> 16) | 0x40);
    return r;
  }
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  r.v = (uint16_t)(u >> 16);
  return r;
}

template <typename S>
struct Conv;
template <>
struct Conv<double> {
  template <typename A>
  HD static A to(double x) { return (A)x; }
  template <typename A>
  HD static double from(A x) { return (double)x; }
};
template <>
struct Conv<float> {
  template <typename A>
  HD static A to(float x) { return (A)x; }
  template <typename A>
  HD static float from(A x) { return (float)x; }
};
template <>
struct Conv<_Float16> {
  template <typename A>
  HD static A to(_Float16 x) { return (A)(float)x; }
  template <typename A>
  HD static _Float16 from(A x) { return (_Float16)(float)x; }
};
template <>
struct Conv<bf16_t> {
  template <typename A>
  HD static A to(bf16_t x) { return (A)bf16_to_float(x); }
  template <typename A>
  HD static bf16_t from(A x) { return float_to_bf16((float)x); }
};

// precision modes: storage type S and arithmetic type A
// SX is the storage of the inner solution vector x, the storage format in every mode: x only
// holds the correction since the last reliable update (which adds it to the FP64 solution and
// zeroes it), of order |M^-1| times the unit-RMS residual, well inside the FP16 range; its
// rounding (2^-11 relative) is far below the reliable-update trigger (0.03).
struct PrecF64 { using S = double;   using SX = double; using A = double; static constexpr int id = 0; };
struct PrecF32 { using S = float;    using SX = float;  using A = float;  static constexpr int id = 1; };
struct PrecF16 { using S = _Float16; using SX = _Float16; using A = float; static constexpr int id = 2; };
struct PrecB16 { using S = bf16_t;   using SX = bf16_t; using A = float;  static constexpr int id = 3; };

// ------------------------------------------------------------------------------------
// chunked field access: NR reals per site, plane-major chunks
// ------------------------------------------------------------------------------------
template <int BYTES>
struct ChunkOf {
  static constexpr int CH = (BYTES % 16 == 0) ? 16 : ((BYTES % 8 == 0) ? 8 : 4);
};
template <int CH>
struct ChunkT;
template <> struct ChunkT<16> { using T = uint4; };
template <> struct ChunkT<8>  { using T = uint2; };
template <> struct ChunkT<4>  { using T = uint32_t; };

template <typename S, int NR>
struct Field {
  static constexpr int BYTES = NR * (int)sizeof(S);
  static constexpr int CH = ChunkOf<BYTES>::CH;
  static constexpr int NCH = BYTES / CH;
  using chunk_t = typename ChunkT<CH>::T;

  // bytes of one field with hv sites
  HD static size_t bytes(long hv) { return (size_t)BYTES * (size_t)hv; }

  template <typename A>
  HD static void load(const void* base, long hv, long site, A* r) {
    const chunk_t* p = (const chunk_t*)base;
    S tmp[NR];
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      chunk_t c = p[(size_t)k * hv + site];
      __builtin_memcpy((char*)tmp + k * CH, &c, CH);
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) r[i] = Conv<S>::template to<A>(tmp[i]);
  }

  template <typename A>
  HD static void store(void* base, long hv, long site, const A* r) {
    chunk_t* p = (chunk_t*)base;
    S tmp[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) tmp[i] = Conv<S>::from(r[i]);
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      chunk_t c;
      __builtin_memcpy(&c, (const char*)tmp + k * CH, CH);
      p[(size_t)k * hv + site] = c;
    }
  }
};

// a spinor of 16-byte chunks at p0 + site*ss + k*cs (any inner layout)
template <typename S>
struct StridedSpinor {
  static constexpr int NCH = 24 * (int)sizeof(S) / 16;
  // NT: non-temporal (streaming) loads and stores, for kernels that touch each value once
  template <typename A, bool NT = false>
  HD static void load(const char* p0, long long ss, long long cs, long site, A* r) {
    S tmp[24];
    const char* p = p0 + site * ss;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      uint4 c;
      if (NT) {
        typedef uint32_t u4v __attribute__((ext_vector_type(4)));
        const u4v v = __builtin_nontemporal_load((const u4v*)(p + k * cs));
        c = make_uint4(v.x, v.y, v.z, v.w);
      } else {
        c = *(const uint4*)(p + k * cs);
      }
      __builtin_memcpy((char*)tmp + k * 16, &c, 16);
    }
#pragma unroll
    for (int i = 0; i < 24; ++i) r[i] = Conv<S>::template to<A>(tmp[i]);
  }
  template <typename A, bool NT = false>
  HD static void store(char* p0, long long ss, long long cs, long site, const A* r) {
    S tmp[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) tmp[i] = Conv<S>::from(r[i]);
    char* p = p0 + site * ss;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      uint4 c;
      __builtin_memcpy(&c, (const char*)tmp + k * 16, 16);
      if (NT) {
        typedef uint32_t u4v __attribute__((ext_vector_type(4)));
        u4v v;
        v.x = c.x;
        v.y = c.y;
        v.z = c.z;
        v.w = c.w;
        __builtin_nontemporal_store(v, (u4v*)(p + k * cs));
      } else {
        *(uint4*)(p + k * cs) = c;
      }
    }
  }
};

template <typename S> using SpinorF = Field<S, 24>;
template <typename S> using LinkF = Field<S, 18>;
// a clover pair is two consecutive 36-real block fields (block 0 then block 1)
template <typename S> using CloverBlkF = Field<S, 36>;
template <typename S>
HD size_t clover_bytes(long hv) { return 2 * CloverBlkF<S>::bytes(hv); }

// ------------------------------------------------------------------------------------
// geometry
// ------------------------------------------------------------------------------------
struct Geo {
  int X, Y, Z, T;
  int Xh;   // X / 2
  int hv;   // sites per parity
  int tbc;  // +1 periodic, -1 antiperiodic fermions in time
  // 4D site bricks of the stencil sweeps (extents in xh, y, z, t dividing Xh, Y, Z, T)
  unsigned char bxh, by, bz, bt;
};

// cb index of position p of a stencil sweep: bricks in lexicographic order, inside a brick x
// fastest (YFAST = false) or y fastest (YFAST = true), then z and t.  A bijection of [0, hv).
template <bool YFAST>
HD int brick_site(const Geo& g, int p) {
  const int bxh = g.bxh, by = g.by, bz = g.bz, bt = g.bt;
  const int B = bxh * by * bz * bt;
  int br = p / B, r = p - br * B;
  int rx, ry;
  if (YFAST) {
    ry = r % by;
    r /= by;
    rx = r % bxh;
    r /= bxh;
  } else {
    rx = r % bxh;
    r /= bxh;
    ry = r % by;
    r /= by;
  }
  const int rz = r % bz, rt = r / bz;
  const int nbx = g.Xh / bxh, nby = g.Y / by, nbz = g.Z / bz;
  const int ix = br % nbx;
  br /= nbx;
  const int iy = br % nby;
  br /= nby;
  const int iz = br % nbz, it = br / nbz;
  return (((it * bt + rt) * g.Z + iz * bz + rz) * g.Y + iy * by + ry) * g.Xh + ix * bxh + rx;
}

HD void cb_coords(const Geo& g, int cb, int par, int c[4]) {
  int xh = cb % g.Xh;
  int r = cb / g.Xh;
  c[1] = r % g.Y;
  r /= g.Y;
  c[2] = r % g.Z;
  c[3] = r / g.Z;
  c[0] = 2 * xh + ((c[1] + c[2] + c[3] + par) & 1);
}

HD int cb_index(const Geo& g, const int c[4]) {
  return ((c[3] * g.Z + c[2]) * g.Y + c[1]) * g.Xh + (c[0] >> 1);
}

// lexicographic full-lattice index of cb-site (for the canonical layout)
HD long lex_index(const Geo& g, const int c[4]) {
  return (((long)c[3] * g.Z + c[2]) * g.Y + c[1]) * (long)g.X + c[0];
}

// neighbour cb index in direction mu (+1 or -1); the neighbour has the other parity
HD int neighbor(const Geo& g, const int c[4], int mu, int dir) {
  int d[4] = {c[0], c[1], c[2], c[3]};
  int L = (mu == 0) ? g.X : (mu == 1) ? g.Y : (mu == 2) ? g.Z : g.T;
  int v = d[mu] + dir;
  v = (v == L) ? 0 : ((v < 0) ? L - 1 : v);
  d[mu] = v;
  return cb_index(g, d);
}

// ------------------------------------------------------------------------------------
// complex helpers
// ------------------------------------------------------------------------------------
template <typename A>
struct cx {
  A re, im;
};

template <typename A> HD cx<A> mk(A r, A i) { cx<A> z; z.re = r; z.im = i; return z; }
template <typename A> HD cx<A> operator+(cx<A> a, cx<A> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename A> HD cx<A> operator-(cx<A> a, cx<A> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename A> HD cx<A> operator-(cx<A> a) { return mk(-a.re, -a.im); }
template <typename A> HD cx<A> operator*(cx<A> a, cx<A> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename A> HD cx<A> operator*(A s, cx<A> b) { return mk(s * b.re, s * b.im); }
template <typename A> HD cx<A> conj_mul(cx<A> a, cx<A> b) {  // conj(a) * b
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename A> HD cx<A> mul_i(cx<A> a) { return mk(-a.im, a.re); }     // i a
template <typename A> HD cx<A> mul_mi(cx<A> a) { return mk(a.im, -a.re); }   // -i a

// a spinor: 12 complex, index s*3 + c
template <typename A>
struct Spinor {
  cx<A> v[12];
};

template <typename S, typename A>
HD void load_spinor(const void* base, long hv, long site, Spinor<A>& s) {
  SpinorF<S>::template load<A>(base, hv, site, (A*)s.v);
}
template <typename S, typename A>
HD void store_spinor(void* base, long hv, long site, const Spinor<A>& s) {
  SpinorF<S>::template store<A>(base, hv, site, (const A*)s.v);
}

template <typename A>
struct Su3 {
  cx<A> m[9];  // row-major
};

// U h for the two spin components of a half spinor h[2][3]
template <typename A>
HD void su3_mul_half(const Su3<A>& U, const cx<A> h[6], cx<A> out[6]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<A> acc = U.m[a * 3 + 0] * h[s * 3 + 0];
      acc = acc + U.m[a * 3 + 1] * h[s * 3 + 1];
      acc = acc + U.m[a * 3 + 2] * h[s * 3 + 2];
      out[s * 3 + a] = acc;
    }
}

// U^dag h
template <typename A>
HD void su3_dag_mul_half(const Su3<A>& U, const cx<A> h[6], cx<A> out[6]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<A> acc = conj_mul(U.m[0 * 3 + a], h[s * 3 + 0]);
      acc = acc + conj_mul(U.m[1 * 3 + a], h[s * 3 + 1]);
      acc = acc + conj_mul(U.m[2 * 3 + a], h[s * 3 + 2]);
      out[s * 3 + a] = acc;
    }
}

// Spin projection for the forward hop (1 - gamma_mu) and the backward hop (1 + gamma_mu)
// in the chiral basis.  Writing psi = (u0, u1, l0, l1) with gamma_mu = [[0, a], [a^dag, 0]]
// (a_k = -i sigma_k, a_4 = 1), (1 -+ gamma_mu) psi = (h ; -+ a^dag h) with h = u -+ a l.
template <typename A>
HD void project(int mu, int fwd, const Spinor<A>& p, cx<A> h[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<A> u0 = p.v[0 * 3 + c], u1 = p.v[1 * 3 + c], l0 = p.v[2 * 3 + c], l1 = p.v[3 * 3 + c];
    cx<A> h0, h1;
    if (fwd) {  // h = u - a l
      switch (mu) {
        case 0: h0 = u0 + mul_i(l1); h1 = u1 + mul_i(l0); break;
        case 1: h0 = u0 + l1;        h1 = u1 - l0;        break;
        case 2: h0 = u0 + mul_i(l0); h1 = u1 - mul_i(l1); break;
        default: h0 = u0 - l0;       h1 = u1 - l1;        break;
      }
    } else {  // h = u + a l
      switch (mu) {
        case 0: h0 = u0 - mul_i(l1); h1 = u1 - mul_i(l0); break;
        case 1: h0 = u0 - l1;        h1 = u1 + l0;        break;
        case 2: h0 = u0 - mul_i(l0); h1 = u1 + mul_i(l1); break;
        default: h0 = u0 + l0;       h1 = u1 + l1;        break;
      }
    }
    h[0 * 3 + c] = h0;
    h[1 * 3 + c] = h1;
  }
}

// accumulate (h ; -+ a^dag h) into acc, with sign phase (+1/-1)
template <typename A>
HD void reconstruct_acc(int mu, int fwd, const cx<A> h[6], A phase, Spinor<A>& acc) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<A> h0 = phase * h[0 * 3 + c], h1 = phase * h[1 * 3 + c];
    cx<A> l0, l1;
    if (fwd) {  // -a^dag h
      switch (mu) {
        case 0: l0 = mul_mi(h1); l1 = mul_mi(h0); break;
        case 1: l0 = -h1;        l1 = h0;         break;
        case 2: l0 = mul_mi(h0); l1 = mul_i(h1);  break;
        default: l0 = -h0;       l1 = -h1;        break;
      }
    } else {  // +a^dag h
      switch (mu) {
        case 0: l0 = mul_i(h1);  l1 = mul_i(h0);  break;
        case 1: l0 = h1;         l1 = -h0;        break;
        case 2: l0 = mul_i(h0);  l1 = mul_mi(h1); break;
        default: l0 = h0;        l1 = h1;         break;
      }
    }
    acc.v[0 * 3 + c] = acc.v[0 * 3 + c] + h0;
    acc.v[1 * 3 + c] = acc.v[1 * 3 + c] + h1;
    acc.v[2 * 3 + c] = acc.v[2 * 3 + c] + l0;
    acc.v[3 * 3 + c] = acc.v[3 * 3 + c] + l1;
  }
}

// ------------------------------------------------------------------------------------
// packed Hermitian 6x6 blocks
// ------------------------------------------------------------------------------------
// offset of the complex lower-triangle entry (i > j) within a 36-real block
HD int tri_off(int i, int j) { return 6 + 2 * (i * (i - 1) / 2 + j); }

template <typename A>
HD void clover_apply_block(const A* blk, const cx<A> in[6], cx<A> out[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    cx<A> acc = blk[i] * in[i];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (j == i) continue;
      if (i > j) {
        cx<A> a = mk(blk[tri_off(i, j)], blk[tri_off(i, j) + 1]);
        acc = acc + a * in[j];
      } else {  // (i, j) = conj((j, i))
        cx<A> a = mk(blk[tri_off(j, i)], blk[tri_off(j, i) + 1]);
        acc = acc + conj_mul(a, in[j]);
      }
    }
    out[i] = acc;
  }
}

// out = C psi for the clover pair stored at `base` (two block fields), one block at a time
template <typename S, typename A>
HD void clover_apply_mem(const void* base, long hv, long site, const Spinor<A>& in, Spinor<A>& out) {
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    A blk[36];
    CloverBlkF<S>::template load<A>((const char*)base + b * CloverBlkF<S>::bytes(hv), hv, site, blk);
    cx<A> i6[6], o6[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) i6[k] = in.v[b * 6 + k];
    clover_apply_block(blk, i6, o6);
#pragma unroll
    for (int k = 0; k < 6; ++k) out.v[b * 6 + k] = o6[k];
  }
}

// ------------------------------------------------------------------------------------
// device descriptors shared by the solver kernels
// ------------------------------------------------------------------------------------
// An operator instance: geometry, links and clover for one (gauge field, c_sw, kappa).
// Index 0 of each [2] is the inner (working) precision, index 1 is FP64.
struct OpDev {
  Geo g;
  double kappa;
  const void* U[2][2];   // [prec][parity] -> 4 link fields (mu-major) of that parity's sites
  const void* A[2][2];   // [prec][parity] clover
  const void* Ai[2][2];  // [prec][parity] clover inverse
  // matrix-core stencil (16-bit inner precision, per output parity): hop links [site][8][3][3],
  // full clover and inverse-clover blocks [site][2][6][6], complex pairs of 16-bit reals
  const void* HL[2];
  const void* AF[2];
  const void* AIF[2];
};

// One right-hand side of a batch.
// Inner vectors are arrays of 16-byte chunks addressed by strides, so that one set of kernels
// serves both inner layouts:
//   per slot     chunk k of site i at arena + i*16 + k*hv*16   (plane-major, one slot)
//   interleaved  [site][tile][chunk][16 lanes] of 16-byte chunks shared by up to 64 slots of a
//                group; arena points at the slot's lane (tile*768 + lane*16 for 2-byte reals),
//                site stride = tiles*768, chunk stride = 256.  The inner x of FP16 mode (FP32,
//                six chunks) uses twice the site stride and an extra offset of tile*768.
struct SlotDev {
  int op;
  int nblk;              // site blocks of this slot's operator
  int sid;               // stable slot id: index of its reduction partials and counter
  int pad;
  char* arena[2];        // [prec] base of this slot's vectors
  long long vstride[2];  // [prec] bytes between consecutive vectors
  long long lss, lcs;    // inner vectors: bytes between sites, between chunks of a site
  long long lss_x, lxoff;  // inner x: site stride and extra offset
  double* scal;          // per-slot scalar block (NSCAL doubles)
  const double* src;     // canonical source (device)
  double* sol;           // canonical solution (device)
  const double* x0;      // canonical initial guess (device) or null
};

// a vector of one slot in one arena: base of vector 0, site and chunk strides
struct VView {
  char* base;
  long long vs, ss, cs;
};
HD VView lo_view(const SlotDev& sd) { return VView{sd.arena[0], sd.vstride[0], sd.lss, sd.lcs}; }
HD VView hi_view(const SlotDev& sd, long hv) { return VView{sd.arena[1], sd.vstride[1], 16, (long long)hv * 16}; }
HD VView view_of(const SlotDev& sd, int psel, long hv) { return psel ? hi_view(sd, hv) : lo_view(sd); }

template <typename S, typename A, bool NT = false>
HD void vload(const VView& w, int v, long site, Spinor<A>& s) {
  StridedSpinor<S>::template load<A, NT>(w.base + (long long)v * w.vs, w.ss, w.cs, site, (A*)s.v);
}
template <typename S, typename A, bool NT = false>
HD void vstore(const VView& w, int v, long site, const Spinor<A>& s) {
  StridedSpinor<S>::template store<A, NT>(w.base + (long long)v * w.vs, w.ss, w.cs, site, (const A*)s.v);
}
// the inner iterate x (storage SX) of a slot
template <typename SX, typename A, bool NT = false>
HD void xload(const SlotDev& sd, int v, long site, Spinor<A>& s) {
  StridedSpinor<SX>::template load<A, NT>(sd.arena[0] + (long long)v * sd.vstride[0] + sd.lxoff, sd.lss_x, sd.lcs,
                                          site, (A*)s.v);
}
template <typename SX, typename A, bool NT = false>
HD void xstore(const SlotDev& sd, int v, long site, const Spinor<A>& s) {
  StridedSpinor<SX>::template store<A, NT>(sd.arena[0] + (long long)v * sd.vstride[0] + sd.lxoff, sd.lss_x, sd.lcs,
                                           site, (const A*)s.v);
}

// slot scalar block layout (doubles)
enum {
  SC_RHO = 0,       // complex
  SC_ALPHA = 2,     // complex
  SC_OMEGA = 4,     // complex
  SC_BETA = 6,      // complex
  SC_RNORM2 = 8,    // iterated |r|^2 in inner units
  SC_SIGMA = 9,     // scale: inner vector = true vector / sigma
  SC_R64N2 = 10,    // |r|^2 from the last FP64 recomputation
  SC_ETAN2 = 11,    // |eta|^2 (both parities)
  SC_RHOPREV = 12,  // complex
  SC_FLAGS = 14,    // breakdown bits
  SC_RES_E = 15,    // full residual |r_e|^2
  SC_RES_O = 16,    // full residual |r_o|^2
  SC_TMP = 17,
  NSCAL = 32
};

// low-precision (inner) vectors of a slot, all half-lattice sized
enum { VL_R = 0, VL_RHAT, VL_P, VL_V, VL_S, VL_T, VL_TE, VL_X, NVEC_LO };
// FP64 vectors of a slot
enum { VH_ETA_E = 0, VH_ETA_O, VH_BHAT, VH_X, VH_R, VH_TE, NVEC_HI };

}  // namespace a2a
