// fields.hip -- gauge-field ingest, clover construction and inversion, noise generation.
//
// Clover term (c_SW of Sec. 8, tree-level value 1): per site the field strength
//   F_munu = (Q_munu - Q_munu^dag) / 8 from the four plaquette leaves around x, and
//   A = 1 + i kappa c_sw sum_{mu<nu} sigma_munu (x) F_munu.
// In the chiral basis every sigma_munu = i gamma_mu gamma_nu is block diagonal, so A is two
// Hermitian 6x6 blocks (spins {0,1} and {2,3}); the kappa-independent part
// G = i sum sigma (x) F is built once per (gauge field) and A, A^{-1} per kappa.
#include "a2a_contract.h"
#include "a2a_kernels.h"

namespace a2a {

// ------------------------------------------------------------------------------------
// gauge links: canonical [site][mu][3][3] complex128 -> per-parity, per-mu link fields
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BS) void k_gauge_to_eo(Geo g, const double* canon, void* d0, void* d1) {
  using S = typename P::S;
  const int site = blockIdx.x * BS + threadIdx.x;
  const int par = blockIdx.y;
  if (site >= g.hv) return;
  int c[4];
  cb_coords(g, site, par, c);
  const double* src = canon + lex_index(g, c) * 72;
  char* dst = (char*)(par ? d1 : d0);
  const size_t lb = LinkF<S>::bytes(g.hv);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    double u[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) u[k] = src[mu * 18 + k];
    LinkF<S>::template store<double>(dst + mu * lb, g.hv, site, u);
  }
}

void launch_gauge_to_eo(int prec, const Geo& g, const double* canon, void* const dst[2], hipStream_t s) {
  dim3 grid((g.hv + BS - 1) / BS, 2);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_gauge_to_eo<PrecF64>, grid, dim3(BS), 0, s, g, canon, dst[0], dst[1]); break;
    case 1: hipLaunchKernelGGL(k_gauge_to_eo<PrecF32>, grid, dim3(BS), 0, s, g, canon, dst[0], dst[1]); break;
    case 2: hipLaunchKernelGGL(k_gauge_to_eo<PrecF16>, grid, dim3(BS), 0, s, g, canon, dst[0], dst[1]); break;
    case 3: hipLaunchKernelGGL(k_gauge_to_eo<PrecB16>, grid, dim3(BS), 0, s, g, canon, dst[0], dst[1]); break;
    default: break;
  }
}

// ------------------------------------------------------------------------------------
// per-site hop links for the matrix-core stencil
// ------------------------------------------------------------------------------------
// For every site x of parity par, the eight 3x3 colour matrices that multiply the
// neighbour spinors of the hopping term, d = 2 mu + f:
//   f = 0:  U_mu(x)            times the boundary sign if x + mu wraps in t
//   f = 1:  U_mu(x - mu)^dag   times the boundary sign if x - mu wraps in t
// stored as [site][d][a][b] complex pairs of the storage format (288 B per site in 16 bits).
template <class P>
__global__ __launch_bounds__(BS) void k_hop_links(Geo g, const double* canon, int par, void* dst) {
  using S = typename P::S;
  const int site = blockIdx.x * BS + threadIdx.x;
  if (site >= g.hv) return;
  int c[4];
  cb_coords(g, site, par, c);
  S* out = (S*)dst + (size_t)site * 144;
  const long lx = lex_index(g, c);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const double* f = canon + (lx * 4 + mu) * 18;
    const double sf = (mu == 3 && c[3] == g.T - 1) ? (double)g.tbc : 1.0;
    int cb[4] = {c[0], c[1], c[2], c[3]};
    const int L = mu == 0 ? g.X : mu == 1 ? g.Y : mu == 2 ? g.Z : g.T;
    cb[mu] = c[mu] == 0 ? L - 1 : c[mu] - 1;
    const double* bk = canon + (lex_index(g, cb) * 4 + mu) * 18;
    const double sb = (mu == 3 && c[3] == 0) ? (double)g.tbc : 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        S* o0 = out + ((2 * mu) * 9 + a * 3 + b) * 2;
        o0[0] = Conv<S>::from(sf * f[(a * 3 + b) * 2]);
        o0[1] = Conv<S>::from(sf * f[(a * 3 + b) * 2 + 1]);
        S* o1 = out + ((2 * mu + 1) * 9 + a * 3 + b) * 2;  // (U^dag)_ab = conj(U_ba)
        o1[0] = Conv<S>::from(sb * bk[(b * 3 + a) * 2]);
        o1[1] = Conv<S>::from(-sb * bk[(b * 3 + a) * 2 + 1]);
      }
  }
}

void launch_hop_links(int prec, const Geo& g, const double* canon, int par, void* dst, hipStream_t s) {
  dim3 grid((g.hv + BS - 1) / BS);
  if (prec == 2) hipLaunchKernelGGL(k_hop_links<PrecF16>, grid, dim3(BS), 0, s, g, canon, par, dst);
  if (prec == 3) hipLaunchKernelGGL(k_hop_links<PrecB16>, grid, dim3(BS), 0, s, g, canon, par, dst);
}

// packed FP64 clover blocks -> full 6x6 complex blocks [site][block][i][j] in the storage format
template <class P>
__global__ __launch_bounds__(BS) void k_clover_full(long hv, const double* packed, void* dst) {
  using S = typename P::S;
  const long site = (long)blockIdx.x * BS + threadIdx.x;
  if (site >= hv) return;
  S* out = (S*)dst + site * 144;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    double blk[36];
    CloverBlkF<double>::template load<double>((const char*)packed + b * CloverBlkF<double>::bytes(hv), hv, site, blk);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        double re, im;
        if (i == j) {
          re = blk[i];
          im = 0.0;
        } else if (i > j) {
          re = blk[tri_off(i, j)];
          im = blk[tri_off(i, j) + 1];
        } else {
          re = blk[tri_off(j, i)];
          im = -blk[tri_off(j, i) + 1];
        }
        S* o = out + ((b * 6 + i) * 6 + j) * 2;
        o[0] = Conv<S>::from(re);
        o[1] = Conv<S>::from(im);
      }
  }
}

void launch_clover_full(int prec, long hv, const double* packed, void* dst, hipStream_t s) {
  dim3 grid((unsigned)((hv + BS - 1) / BS));
  if (prec == 2) hipLaunchKernelGGL(k_clover_full<PrecF16>, grid, dim3(BS), 0, s, hv, packed, dst);
  if (prec == 3) hipLaunchKernelGGL(k_clover_full<PrecB16>, grid, dim3(BS), 0, s, hv, packed, dst);
}

// ------------------------------------------------------------------------------------
// clover field
// ------------------------------------------------------------------------------------
struct M3 {
  cx<double> m[9];
};

HD M3 m3_load(const double* canon, long lex, int mu) {
  M3 r;
  const double* p = canon + (lex * 4 + mu) * 18;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.m[k] = mk(p[2 * k], p[2 * k + 1]);
  return r;
}
HD M3 m3_mul(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> acc = a.m[i * 3] * b.m[j];
      acc = acc + a.m[i * 3 + 1] * b.m[3 + j];
      acc = acc + a.m[i * 3 + 2] * b.m[6 + j];
      r.m[i * 3 + j] = acc;
    }
  return r;
}
HD M3 m3_dag(const M3& a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.m[i * 3 + j] = mk(a.m[j * 3 + i].re, -a.m[j * 3 + i].im);
  return r;
}

HD long lex_shift(const Geo& g, const int c[4], int mu, int dm, int nu, int dn) {
  int d[4] = {c[0], c[1], c[2], c[3]};
  const int L[4] = {g.X, g.Y, g.Z, g.T};
  d[mu] = (d[mu] + dm + L[mu]) % L[mu];
  d[nu] = (d[nu] + dn + L[nu]) % L[nu];
  return lex_index(g, d);
}

// F_munu at the site with coordinates c (four counter-clockwise leaves)
HD M3 field_strength(const Geo& g, const double* U, const int c[4], int mu, int nu) {
  const long x = lex_index(g, c);
  const long xpm = lex_shift(g, c, mu, 1, nu, 0), xpn = lex_shift(g, c, mu, 0, nu, 1);
  const long xmm = lex_shift(g, c, mu, -1, nu, 0), xmn = lex_shift(g, c, mu, 0, nu, -1);
  const long xmm_pn = lex_shift(g, c, mu, -1, nu, 1), xmm_mn = lex_shift(g, c, mu, -1, nu, -1);
  const long xmn_pm = lex_shift(g, c, mu, 1, nu, -1);
  M3 q;
  {
    M3 l = m3_mul(m3_mul(m3_load(U, x, mu), m3_load(U, xpm, nu)),
                  m3_mul(m3_dag(m3_load(U, xpn, mu)), m3_dag(m3_load(U, x, nu))));
    q = l;
  }
  {
    M3 l = m3_mul(m3_mul(m3_load(U, x, nu), m3_dag(m3_load(U, xmm_pn, mu))),
                  m3_mul(m3_dag(m3_load(U, xmm, nu)), m3_load(U, xmm, mu)));
#pragma unroll
    for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + l.m[k];
  }
  {
    M3 l = m3_mul(m3_mul(m3_dag(m3_load(U, xmm, mu)), m3_dag(m3_load(U, xmm_mn, nu))),
                  m3_mul(m3_load(U, xmm_mn, mu), m3_load(U, xmn, nu)));
#pragma unroll
    for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + l.m[k];
  }
  {
    M3 l = m3_mul(m3_mul(m3_dag(m3_load(U, xmn, nu)), m3_load(U, xmn, mu)),
                  m3_mul(m3_load(U, xmn_pm, nu), m3_dag(m3_load(U, x, mu))));
#pragma unroll
    for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + l.m[k];
  }
  M3 f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> a = q.m[i * 3 + j], b = q.m[j * 3 + i];
      f.m[i * 3 + j] = mk((a.re - b.re) / 8.0, (a.im + b.im) / 8.0);  // (q - q^dag)/8
    }
  return f;
}

// Pauli coefficients (c1, c2, c3) of the 2x2 block of sigma_munu in chiral block b, planes
// ordered (01, 02, 03, 12, 13, 23); sigma_munu = i gamma_mu gamma_nu = i diag(a_mu a_nu^dag,
// a_mu^dag a_nu) with a_k = -i sigma_k, a_4 = 1.
HD void sigma_block(int plane, int b, int cf[3]) {
  const int up[6][3] = {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  const int dn[6][3] = {{0, 0, -1}, {0, 1, 0}, {-1, 0, 0}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}};
#pragma unroll
  for (int k = 0; k < 3; ++k) cf[k] = b ? dn[plane][k] : up[plane][k];
}

// packed G = i sum_{mu<nu} sigma_munu^(b) (x) F_munu for chiral block b at site c
HD void clover_G_block(const Geo& g, const double* U, const int c[4], int b, double out[36]) {
  // every loop unrolled: plane, sigma coefficients and matrix indices are compile-time
  // constants (a run-time index into the coefficient tables would place them in scratch memory)
  cx<double> G[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) G[k] = mk(0.0, 0.0);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu)
#pragma unroll
    for (int nu = mu + 1; nu < 4; ++nu) {
      const int plane = mu == 0 ? nu - 1 : mu == 1 ? nu + 1 : 5;  // (01, 02, 03, 12, 13, 23)
      M3 F = field_strength(g, U, c, mu, nu);
      int cf[3];
      sigma_block(plane, b, cf);
      // M = c1 s1 + c2 s2 + c3 s3 = [[c3, c1 - i c2], [c1 + i c2, -c3]]
      cx<double> M[4] = {mk((double)cf[2], 0.0), mk((double)cf[0], -(double)cf[1]),
                         mk((double)cf[0], (double)cf[1]), mk(-(double)cf[2], 0.0)};
#pragma unroll
      for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          cx<double> im = mul_i(M[s1 * 2 + s2]);  // i M
          if (im.re == 0.0 && im.im == 0.0) continue;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
              G[(s1 * 3 + a) * 6 + s2 * 3 + bb] = G[(s1 * 3 + a) * 6 + s2 * 3 + bb] + im * F.m[a * 3 + bb];
        }
    }
  for (int i = 0; i < 6; ++i) out[i] = G[i * 6 + i].re;
  for (int i = 1; i < 6; ++i)
    for (int j = 0; j < i; ++j) {
      out[tri_off(i, j)] = G[i * 6 + j].re;
      out[tri_off(i, j) + 1] = G[i * 6 + j].im;
    }
}

__global__ __launch_bounds__(BS) void k_clover_field(Geo g, const double* U, double* G0, double* G1) {
  const int site = blockIdx.x * BS + threadIdx.x;
  const int par = blockIdx.y;
  const int b = blockIdx.z;
  if (site >= g.hv) return;
  int c[4];
  cb_coords(g, site, par, c);
  double blk[36];
  clover_G_block(g, U, c, b, blk);
  double* dst = (par ? G1 : G0);
  CloverBlkF<double>::store<double>((char*)dst + b * CloverBlkF<double>::bytes(g.hv), g.hv, site, blk);
}

void launch_clover_field(const Geo& g, const double* canon_links, double* G[2], hipStream_t s) {
  dim3 grid((g.hv + BS - 1) / BS, 2, 2);
  hipLaunchKernelGGL(k_clover_field, grid, dim3(BS), 0, s, g, canon_links, G[0], G[1]);
}

// ------------------------------------------------------------------------------------
// A = 1 + kcsw G and A^{-1} (FP64, Gauss-Jordan with partial pivoting per 6x6 block)
// ------------------------------------------------------------------------------------
HD void unpack6(const double* p, cx<double> M[36]) {
  for (int i = 0; i < 6; ++i) M[i * 6 + i] = mk(p[i], 0.0);
  for (int i = 1; i < 6; ++i)
    for (int j = 0; j < i; ++j) {
      cx<double> a = mk(p[tri_off(i, j)], p[tri_off(i, j) + 1]);
      M[i * 6 + j] = a;
      M[j * 6 + i] = mk(a.re, -a.im);
    }
}

HD void pack6(const cx<double> M[36], double* p) {
  // Hermitian part of M
  for (int i = 0; i < 6; ++i) p[i] = M[i * 6 + i].re;
  for (int i = 1; i < 6; ++i)
    for (int j = 0; j < i; ++j) {
      p[tri_off(i, j)] = 0.5 * (M[i * 6 + j].re + M[j * 6 + i].re);
      p[tri_off(i, j) + 1] = 0.5 * (M[i * 6 + j].im - M[j * 6 + i].im);
    }
}

HD double cabs2(cx<double> a) { return a.re * a.re + a.im * a.im; }

// Gauss-Jordan with partial pivoting.  Every loop is unrolled and the pivot row is swapped in
// by a comparison with each candidate row, so all indices are compile-time constants and the
// augmented matrix stays in registers (a run-time row index would place it in scratch memory,
// which the runtime must allocate at dispatch).
HD int invert6(const cx<double> M[36], cx<double> R[36]) {
  cx<double> a[6][12];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      a[i][j] = M[i * 6 + j];
      a[i][6 + j] = mk(i == j ? 1.0 : 0.0, 0.0);
    }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    double best = cabs2(a[c][c]);
#pragma unroll
    for (int r = c + 1; r < 6; ++r)
      if (cabs2(a[r][c]) > best) {
        best = cabs2(a[r][c]);
        piv = r;
      }
    if (best == 0.0) return 1;
#pragma unroll
    for (int r = c + 1; r < 6; ++r)
      if (r == piv)
#pragma unroll
        for (int j = 0; j < 12; ++j) {
          cx<double> t = a[c][j];
          a[c][j] = a[r][j];
          a[r][j] = t;
        }
    cx<double> d = a[c][c];
    double dn = cabs2(d);
    cx<double> di = mk(d.re / dn, -d.im / dn);
#pragma unroll
    for (int j = 0; j < 12; ++j) a[c][j] = di * a[c][j];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      cx<double> f = a[r][c];
#pragma unroll
      for (int j = 0; j < 12; ++j) a[r][j] = a[r][j] - f * a[c][j];
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) R[i * 6 + j] = a[i][6 + j];
  return 0;
}

// G, A, Ainv: one parity, packed FP64 pair fields
__global__ __launch_bounds__(128) void k_clover_make(long hv, const double* G, double kcsw, double* A, double* Ai) {
  const long site = (long)blockIdx.x * 128 + threadIdx.x;
  const int b = blockIdx.y;
  if (site >= hv) return;
  const size_t bb = CloverBlkF<double>::bytes(hv);
  double g[36], p[36];
  CloverBlkF<double>::load<double>((const char*)G + b * bb, hv, site, g);
  for (int k = 0; k < 36; ++k) p[k] = kcsw * g[k];
  for (int i = 0; i < 6; ++i) p[i] += 1.0;
  if (A) CloverBlkF<double>::store<double>((char*)A + b * bb, hv, site, p);
  if (Ai) {
    cx<double> M[36], R[36];
    unpack6(p, M);
    if (invert6(M, R)) {
      for (int k = 0; k < 36; ++k) p[k] = __builtin_nan("");
    } else {
      pack6(R, p);
    }
    CloverBlkF<double>::store<double>((char*)Ai + b * bb, hv, site, p);
  }
}

void launch_clover_make(const Geo& g, const double* G, double kcsw, double* A, double* Ainv, hipStream_t s) {
  dim3 grid((g.hv + 127) / 128, 2);
  hipLaunchKernelGGL(k_clover_make, grid, dim3(128), 0, s, (long)g.hv, G, kcsw, A, Ainv);
}

template <class P>
__global__ __launch_bounds__(BS) void k_clover_convert(long hv, const double* src, void* dst) {
  using S = typename P::S;
  const long site = (long)blockIdx.x * BS + threadIdx.x;
  const int b = blockIdx.y;
  if (site >= hv) return;
  double p[36];
  CloverBlkF<double>::load<double>((const char*)src + b * CloverBlkF<double>::bytes(hv), hv, site, p);
  CloverBlkF<S>::template store<double>((char*)dst + b * CloverBlkF<S>::bytes(hv), hv, site, p);
}

void launch_clover_convert(int prec, long hv, const double* src, void* dst, hipStream_t s) {
  dim3 grid((unsigned)((hv + BS - 1) / BS), 2);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_clover_convert<PrecF64>, grid, dim3(BS), 0, s, hv, src, dst); break;
    case 1: hipLaunchKernelGGL(k_clover_convert<PrecF32>, grid, dim3(BS), 0, s, hv, src, dst); break;
    case 2: hipLaunchKernelGGL(k_clover_convert<PrecF16>, grid, dim3(BS), 0, s, hv, src, dst); break;
    case 3: hipLaunchKernelGGL(k_clover_convert<PrecB16>, grid, dim3(BS), 0, s, hv, src, dst); break;
    default: break;
  }
}

// ------------------------------------------------------------------------------------
// complex Z2 noise from a counter hash (splitmix64 of Steele, Lea and Flood, 2014):
//   component k of the global flattened source array gets h = splitmix64(seed*2^48 + k),
//   real sign from bit 0, imaginary sign from bit 1 (set = minus), modulus 1.
// ------------------------------------------------------------------------------------
HD uint64_t splitmix64_first(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(BS) void k_z2_noise(long n, unsigned long long seed, long long first, double* out) {
  const long i = (long)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const uint64_t h = splitmix64_first((seed << 48) + (uint64_t)(first + i));
  const double r = 0.70710678118654752440;
  out[2 * i] = (h & 1ull) ? -r : r;
  out[2 * i + 1] = (h & 2ull) ? -r : r;
}

void launch_z2_noise(long V, int nsrc, unsigned long long seed, long long src_offset, double* out, hipStream_t s) {
  const long n = (long)nsrc * 12 * V;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_z2_noise, dim3((unsigned)((n + BS - 1) / BS)), dim3(BS), 0, s, n, seed,
                     (long long)(src_offset * 12 * V), out);
}

// Dilution (Sec. 7, "time-spin-colour dilution"): output source i D + d is noise vector i
// restricted to piece d -- one timeslice (scheme 1, d = t), one spin-colour component (scheme 2,
// d = 3 spin + colour) or both (scheme 3, d = 12 t + 3 spin + colour); zero elsewhere.
// Scheme 0 copies.  One thread per complex output element.
__global__ __launch_bounds__(BS) void k_dilute(long total, long V3, int T, int D, int scheme, const double* noise,
                                               double* out) {
  const long e = (long)blockIdx.x * BS + threadIdx.x;
  if (e >= total) return;
  const long per = 12L * V3 * T;  // complex per source
  const long src = e / per, k = e % per;
  const long i = src / D;
  const int d = (int)(src % D);
  const int sc = (int)(k % 12), t = (int)(k / (12L * V3));
  const bool on = scheme == 0 || (scheme == 1 && t == d) || (scheme == 2 && sc == d) || (scheme == 3 && 12 * t + sc == d);
  const double* in = noise + 2 * (i * per + k);
  out[2 * e] = on ? in[0] : 0.0;
  out[2 * e + 1] = on ? in[1] : 0.0;
}

void launch_dilute(const Geo& g, int nnoise, int scheme, int D, const double* noise, double* out, hipStream_t s) {
  const long V3 = (long)g.X * g.Y * g.Z;
  const long total = (long)nnoise * D * 12 * V3 * g.T;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_dilute, dim3((unsigned)((total + BS - 1) / BS)), dim3(BS), 0, s, total, V3, g.T, D, scheme,
                     noise, out);
}

// Point sources (Sec. 8: propagators from a point at the origin): the 12 unit vectors at one
// site, source k = 3 spin + colour; one thread per complex output element.
__global__ __launch_bounds__(BS) void k_point_sources(long per, long site, double* out) {
  const long e = (long)blockIdx.x * BS + threadIdx.x;
  if (e >= 12 * per) return;
  const long k = e / per, r = e % per;  // source k, complex element r = 12 site + spin-colour
  out[2 * e] = r == 12 * site + k ? 1.0 : 0.0;
  out[2 * e + 1] = 0.0;
}

void launch_point_sources(const Geo& g, long site, double* out, hipStream_t s) {
  const long per = 12L * g.X * g.Y * g.Z * g.T;
  hipLaunchKernelGGL(k_point_sources, dim3((unsigned)((12 * per + BS - 1) / BS)), dim3(BS), 0, s, per, site, out);
}

}  // namespace a2a
