// fill.hip -- the outer-product fill of the all-to-all propagator (Sec. 7, eq. Sfill) on the
// FP64 matrix cores, and the contraction sum_{z,x} tr[S1 S2^dag] built on it (the "S_s fill",
// "S_s^dag fill" and "sum_x sum_z tr S_s S_s^dag" operations of the paper's timing study).
//
//   S(t, z; t_src, x)_{ab} = (1/N) sum_i X_i(t, z)_a conj(eta_i(t_src, x)_b)
//
// is, for one sink timeslice t, the complex matrix product C = P Q^H of the (12 L^3) x N block
// P of solutions at t and the (12 L^3) x N block Q of sources at t_src; in the canonical
// [src][t][z][y][x][spin][colour] arrays each (source, timeslice) column is contiguous.  The
// kernel is generic in the strides: C(m, n) = scale sum_k P(m, k) conj(Q(n, k)) with
// P(m, k) = P[m pm + k pk], Q(n, k) = Q[n qm + k qk] (complex elements), one product per
// grid.y index z (operand offsets pz, qz per z).
//
// A block of four waves owns a 64 x 64 tile of C; each wave a 32 x 32 quadrant as 2 x 2 tiles
// of 16 x 16 on v_mfma_f64_16x16x4_f64, four real products per complex tile and K step of 4
// (Re += Pr Qr + Pi Qi, Im += Pi Qr - Pr Qi).  Each lane loads its operands straight from
// memory (one 16-byte complex per operand tile and K step; 16 lanes read 256 contiguous bytes
// of a column); at 16 flop per byte of operand traffic per tile the kernel is bound by the
// FP64 matrix rate, not by memory.  Operands past M, N or K read a clamped in-range element
// and are zeroed, so every load is unconditional.
//
// Fill mode stores C (or the spin-colour dagger of its 12 x 12 blocks) to memory.  Contract
// mode multiplies two products (S1 from the first operand pair, S2 from the second) tile by
// tile and accumulates sum C1 conj(C2) without storing either: per-block FP64 partials,
// summed in block order by a second launch.
#include "a2a_contract.h"
#include "a2a_kernels.h"

namespace a2a {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
constexpr int FT = 64;  // output tile edge

// global loads / stores through address-space-1 pointers (the arrays are device memory)
__device__ __forceinline__ double2 ldc(const double* base, long long idx) {
  const d2v v = *(const __attribute__((address_space(1))) d2v*)(base + 2 * idx);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void stc(double* p, double re, double im) {
  d2v v;
  v.x = re;
  v.y = im;
  *(__attribute__((address_space(1))) d2v*)p = v;
}

__device__ __forceinline__ d4v mfma(double a, double b, const d4v& c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace

template <int MODE>  // 0: store the product, 1: contract two products
__global__ __launch_bounds__(256) void k_fill(FillArgs a) {
  constexpr int NP = MODE == 1 ? 2 : 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int idx = lane & 15, kr = lane >> 4;
  const int tiles_n = (a.N + FT - 1) / FT;
  const int m0 = (int)(blockIdx.x / tiles_n) * FT + 32 * (w >> 1);
  const int n0 = (int)(blockIdx.x % tiles_n) * FT + 32 * (w & 1);
  const long long z = blockIdx.y;

  int mr[2], nc[2];
  bool mok[2], nok[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    mr[i] = m0 + 16 * i + idx;
    mok[i] = mr[i] < a.M;
    if (!mok[i]) mr[i] = a.M - 1;
    nc[i] = n0 + 16 * i + idx;
    nok[i] = nc[i] < a.N;
    if (!nok[i]) nc[i] = a.N - 1;
  }
  const double* P[NP];
  const double* Q[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    P[p] = a.P[p] + 2 * z * a.pz;
    Q[p] = a.Q[p] + 2 * z * a.qz;
  }

  d4v cr[NP][2][2], ci[NP][2][2];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) cr[p][i][j] = ci[p][i][j] = d4v{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < a.K; k0 += 4) {
    const int k = k0 + kr;
    const bool kok = k < a.K;
    const long long kc = kok ? k : a.K - 1;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      double2 A[2], B[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        A[i] = ldc(P[p], mr[i] * a.pm + kc * a.pk);
        if (!(mok[i] && kok)) A[i] = make_double2(0.0, 0.0);
        B[i] = ldc(Q[p], nc[i] * a.qm + kc * a.qk);
        if (!(nok[i] && kok)) B[i] = make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[p][i][j] = mfma(A[i].x, B[j].x, cr[p][i][j]);
          cr[p][i][j] = mfma(A[i].y, B[j].y, cr[p][i][j]);
          ci[p][i][j] = mfma(A[i].y, B[j].x, ci[p][i][j]);
          ci[p][i][j] = mfma(-A[i].x, B[j].y, ci[p][i][j]);
        }
    }
  }

  // element q of a 16 x 16 accumulator tile is row 4 q + lane / 16, column lane % 16
  if constexpr (MODE == 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int m = m0 + 16 * i + 4 * q + kr, n = n0 + 16 * j + idx;
          if (m >= a.M || n >= a.N) continue;
          double re = a.scale * cr[0][i][j][q], im = a.scale * ci[0][i][j][q];
          if (a.dagger) {  // (12 u + s, 12 v + s') -> (12 u + s', 12 v + s), conjugated
            const int s = m % 12, s2 = n % 12;
            m += s2 - s;
            n += s - s2;
            im = -im;
          }
          stc(a.out + 2 * (z * a.oz + m * a.om + n * a.on), re, im);
        }
  } else {
    double vr = 0.0, vi = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {  // C1 conj(C2); tiles past M, N are zero
          const double r1 = cr[0][i][j][q], i1 = ci[0][i][j][q], r2 = cr[NP - 1][i][j][q], i2 = ci[NP - 1][i][j][q];
          vr += r1 * r2 + i1 * i2;
          vi += i1 * r2 - r1 * i2;
        }
    double v[2] = {vr * a.scale * a.scale, vi * a.scale * a.scale};
    block_sum_n<2, 256>(v);
    if (threadIdx.x < 2)
      a.partial[2 * (z * gridDim.x + blockIdx.x) + threadIdx.x] = threadIdx.x == 0 ? v[0] : v[1];
  }
}

// corr[z] = sum of the block partials of z, in block order
__global__ __launch_bounds__(64) void k_fill_sum(int nblk, const double* partial, double* corr) {
  const long long z = blockIdx.x;
  double r = 0.0, im = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) {
    r += partial[2 * (z * nblk + b)];
    im += partial[2 * (z * nblk + b) + 1];
  }
  r = wave_sum(r);
  im = wave_sum(im);
  if (threadIdx.x == 0) {
    corr[2 * z] = r;
    corr[2 * z + 1] = im;
  }
}

long long fill_blocks(int M, int N) { return (long long)((M + FT - 1) / FT) * ((N + FT - 1) / FT); }

void launch_fill(const FillArgs& a, int nz, hipStream_t s) {
  const dim3 g((unsigned)fill_blocks(a.M, a.N), (unsigned)nz);
  hipLaunchKernelGGL(k_fill<0>, g, dim3(256), 0, s, a);
}

void launch_fill_contract(const FillArgs& a, int nz, double* corr, hipStream_t s) {
  const int nb = (int)fill_blocks(a.M, a.N);
  hipLaunchKernelGGL(k_fill<1>, dim3((unsigned)nb, (unsigned)nz), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_fill_sum, dim3((unsigned)nz), dim3(64), 0, s, nb, a.partial, corr);
}

}  // namespace a2a
