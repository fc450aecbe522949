// contract.hip -- the stochastic-operator contraction (Sec. 7, eq. stoop) and the
// zero-momentum pion / pi-pi correlators built from it (Sec. 7; Sec. 5 and 8 diagrams).
//
//   O_ab(t) = sum_{y in timeslice t} eta_a(y)^dag gamma_5 X_b(y)
//
// is, per timeslice, a complex matrix product E_t^dag (gamma_5 X_t) with inner dimension
// K = 12 L^3 taken straight from the canonical [src][t][z][y][x][spin][colour] arrays, where
// each (source, timeslice) column is contiguous.  Blocks own a K-chunk of one timeslice and
// a 64x64 tile of (a, b); operand tiles are staged through LDS (coalesced along K) and the
// products run on the FP64 matrix cores, each wave a 16 x 64 strip of the tile.  Chunk partials
// are summed in fixed order.
#include "a2a_contract.h"
#include "a2a_kernels.h"

namespace a2a {

constexpr int CT = 64;   // output tile edge
constexpr int KC = 16;   // complex elements per K step

// rows (optional, [T][na]): row r of timeslice t is source rows[t na + r] (sources supported on
// that timeslice only, e.g. after time dilution); without it na = n and row r is source r.
typedef double d4v __attribute__((ext_vector_type(4)));

// NC: 16-column tiles per wave (1..4, from n); columns past n are staged as zeros
template <int NC>
__global__ __launch_bounds__(256) void k_stoch_partial(int n, int na, long V, int V3, int nchunk, int kchunk,
                                                        int g5, int t_first, const double* __restrict__ eta,
                                                        const double* __restrict__ X,
                                                        const double* __restrict__ phase,
                                                        const int* __restrict__ rows, double* partial) {
  __shared__ double2 Es[CT][KC + 1];
  __shared__ double2 Xs[CT][KC + 1];
  // grid: x = output tile (row tile x column tile), y = timeslice, z = K chunk (<= 4096)
  const int chunk = blockIdx.z, tl = blockIdx.y, t = t_first + tl;
  const int ntb = (n + CT - 1) / CT;
  const int ta = blockIdx.x / ntb, tb = blockIdx.x % ntb;
  const int a0 = ta * CT, b0 = tb * CT;
  const long K = 12L * V3;
  const long k_begin = (long)chunk * kchunk;
  const long k_end = min(K, k_begin + kchunk);
  // wave w owns output rows a0 + 16 w .. + 15 and NC 16-column tiles of the block; a wave whose
  // rows are all past na issues no products (wave-uniform)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const bool row_on = a0 + 16 * w < na;
  d4v cr[NC], ci[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) cr[c] = ci[c] = d4v{0.0, 0.0, 0.0, 0.0};
  const size_t src_stride = (size_t)12 * V;  // complex per source
  const size_t tbase = (size_t)t * V3 * 12;
  // operand loads of the stage at k0 (64 rows x 16 complex of each operand, 4 per thread):
  // every load is unconditional, from a clamped in-range element, and out-of-range elements
  // are zeroed afterwards.  (Loading the next stage during the products cost occupancy and
  // gained nothing.)
  double2 pe[4], px[4];
  auto load = [&](long k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * 256;
      const int row = e / KC, kk = e % KC;
      const long k = k0 + kk;
      const long kc = min(k, k_end - 1);
      const int ra = min(a0 + row, na - 1), rb = min(b0 + row, n - 1);
      const int ar = rows ? rows[(size_t)t * na + ra] : ra;
      double2 ev = *(const double2*)(eta + 2 * ((size_t)ar * src_stride + tbase + kc));
      double2 xv = *(const double2*)(X + 2 * ((size_t)rb * src_stride + tbase + kc));
      if (phase) {  // eta conj(f) with f = exp(-i p.y): the product below takes conj(eta) f
        const double fr = phase[2 * (kc / 12)], fi = phase[2 * (kc / 12) + 1];
        ev = make_double2(ev.x * fr + ev.y * fi, ev.y * fr - ev.x * fi);
      }
      const double sg = (g5 && (kc % 12) >= 6) ? -1.0 : 1.0;  // gamma_5 = diag(1,1,-1,-1)
      const bool kin = k < k_end;
      pe[q] = kin && a0 + row < na ? ev : make_double2(0.0, 0.0);
      px[q] = kin && b0 + row < n ? make_double2(sg * xv.x, sg * xv.y) : make_double2(0.0, 0.0);
    }
  };
  for (long k0 = k_begin; k0 < k_end; k0 += KC) {
    load(k0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * 256;
      Es[e / KC][e % KC] = pe[q];
      Xs[e / KC][e % KC] = px[q];
    }
    __syncthreads();
    if (row_on) {
      // v_mfma_f64_16x16x4: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; four real
      // products per complex K step: Re += er xr + ei xi, Im += er xi - ei xr, issued tile-
      // interleaved so that consecutive products accumulate into different registers
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        const double2 e = Es[16 * w + li][4 * ks + lk];
        double2 x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = Xs[16 * c + li][4 * ks + lk];
#pragma unroll
        for (int c = 0; c < NC; ++c) cr[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(e.x, x[c].x, cr[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < NC; ++c) ci[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(e.x, x[c].y, ci[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < NC; ++c) cr[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(e.y, x[c].y, cr[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < NC; ++c) ci[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(-e.y, x[c].x, ci[c], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // element q of a 16 x 16 accumulator tile is row 4 q + lane / 16, column lane % 16
  double* out = partial + (((size_t)tl * nchunk + chunk) * na) * n * 2;
  if (row_on)
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = a0 + 16 * w + 4 * q + lk, b = b0 + 16 * c + li;
        if (a < na && b < n) {
          out[2 * ((size_t)a * n + b)] = cr[c][q];
          out[2 * ((size_t)a * n + b) + 1] = ci[c][q];
        }
      }
}

__global__ void k_stoch_sum(int n, int na, int T, int nchunk, const double* partial, double* O) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;  // over T*na*n complex
  const long per = (long)na * n;
  if (i >= (long)T * per) return;
  const long t = i / per, ab = i % per;
  double sr = 0.0, si = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    const double* p = partial + (((size_t)t * nchunk + c) * per + ab) * 2;
    sr += p[0];
    si += p[1];
  }
  O[2 * i] = sr;
  O[2 * i + 1] = si;
}

void launch_stoch_ops(const Geo& g, int n, const double* eta, const double* X, double* partial, int nchunk,
                      double* O, hipStream_t s, int g5, int t_first, int nt, const double* phase, const int* rows,
                      int na) {
  const int V3 = g.X * g.Y * g.Z;
  const long V = (long)V3 * g.T;
  const long K = 12L * V3;
  if (nt < 0) nt = g.T;
  long kchunk = (K + nchunk - 1) / nchunk;
  kchunk = ((kchunk + KC - 1) / KC) * KC;
  if (na <= 0) na = n;  // rows == null: eta rows 0 .. na - 1
  const int ntb = (n + CT - 1) / CT, nta = (na + CT - 1) / CT;
  dim3 grid((unsigned)(nta * ntb), nt, nchunk);
  // column tiles per wave: enough for n (a single column block), else all four
  const int nc = ntb > 1 ? 4 : (n + 15) / 16;
  auto kern = nc == 1 ? k_stoch_partial<1> : nc == 2 ? k_stoch_partial<2> : nc == 3 ? k_stoch_partial<3>
                                                                                       : k_stoch_partial<4>;
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, n, na, V, V3, nchunk, (int)kchunk, g5, t_first, eta, X, phase, rows,
                     partial);
  const long tot = (long)nt * na * n;
  hipLaunchKernelGGL(k_stoch_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, na, nt, nchunk, partial,
                     O);
}

// Gram form of sum_{z,x} tr[S1 S2^dag]: corr[t] = (1/n^2) sum_ij E[i][j] F[t][j][i] with
// E = <eta1_i, eta2_j> on the source timeslice and F[t] = <X2_j, X1_i> on timeslice t.
__global__ __launch_bounds__(256) void k_gram_corr(int n, const double* E, const double* F, double* corr) {
  const int t = blockIdx.x;
  const long per = (long)n * n;
  const double* Ft = F + 2 * (size_t)t * per;
  double v[2] = {0.0, 0.0};
  for (long e = threadIdx.x; e < per; e += 256) {
    const long i = e / n, j = e % n;
    const double er = E[2 * (i * n + j)], ei = E[2 * (i * n + j) + 1];
    const double fr = Ft[2 * (j * n + i)], fi = Ft[2 * (j * n + i) + 1];
    v[0] += er * fr - ei * fi;
    v[1] += er * fi + ei * fr;
  }
  block_sum_n<2, 256>(v);
  const double inv = 1.0 / ((double)n * n);
  if (threadIdx.x < 2) corr[2 * t + threadIdx.x] = (threadIdx.x == 0 ? v[0] : v[1]) * inv;
}

void launch_gram_corr(int T, int n, const double* E, const double* F, double* corr, hipStream_t s) {
  hipLaunchKernelGGL(k_gram_corr, dim3((unsigned)T), dim3(256), 0, s, n, E, F, corr);
}

// pi-pi diagrams from point propagators S_p (the 12 solutions of the point sources at
// (t0, x0)) and stochastic propagators of two noise sets (Sec. 8), in factorised form, from the
// timeslice Gram matrices
//   G[t][i][j] = <eta1_i, eta2_j>_t   Fp[t][i][j] = <X1_i, X2_j>_t   Pn[t][k][l] = <Sp_k, Sp_l>_t
//   A[k][i] = <Sp_k, X1_i>_t0          B[t][j][k] = <X2_j, Sp_k>_t
// with, for t = t0 + dt:
//   Cs(dt) = sum_ij G[t0]_ij conj(Fp[t]_ij) / (n1 n2)       L(dt) = sum_ij G[t]_ij conj(Fp[t]_ij) / (n1 n2)
//   D2(dt) = sum_ij G[t]_ij sum_k B[t]_jk A_ki / (n1 n2)    Cp(dt) = sum_k Pn[t]_kk
// The partial kernel sums a chunk of rows i per block (grid: chunks x T); the final kernel sums
// the chunks in order and forms D0 = Cp Cs, D1 = L Cp(0), D2, D3 = conj(D2).
__global__ __launch_bounds__(256) void k_pipi_mixed_partial(int T, int t0, int n1, int n2, int rows,
                                                            const double* G, const double* Fp, const double* A,
                                                            const double* B, double* partial) {
  const int c = blockIdx.x, dt = blockIdx.y, t = (t0 + dt) % T;
  const int i0 = c * rows, i1 = min(n1, i0 + rows);
  const size_t per = (size_t)n1 * n2;
  const double* G0 = G + 2 * (size_t)t0 * per;
  const double* Gt = G + 2 * (size_t)t * per;
  const double* Ft = Fp + 2 * (size_t)t * per;
  const double* Bt = B + 2 * (size_t)t * n2 * 12;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // Cs, L, D2 (re, im)
  const long cnt = (long)(i1 - i0) * n2;
  for (long e = threadIdx.x; e < cnt; e += 256) {
    const int i = i0 + (int)(e / n2), j = (int)(e % n2);
    const size_t ij = 2 * ((size_t)i * n2 + j);
    const double fr = Ft[ij], fi = -Ft[ij + 1];  // F_ji = conj(Fp_ij)
    const double g0r = G0[ij], g0i = G0[ij + 1], gr = Gt[ij], gi = Gt[ij + 1];
    v[0] += g0r * fr - g0i * fi;
    v[1] += g0r * fi + g0i * fr;
    v[2] += gr * fr - gi * fi;
    v[3] += gr * fi + gi * fr;
    double br = 0.0, bi = 0.0;  // (B A)_ji
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double* b = Bt + 2 * ((size_t)j * 12 + k);
      const double* a = A + 2 * ((size_t)k * n1 + i);
      br += b[0] * a[0] - b[1] * a[1];
      bi += b[0] * a[1] + b[1] * a[0];
    }
    v[4] += gr * br - gi * bi;
    v[5] += gr * bi + gi * br;
  }
  block_sum_n<6, 256>(v);
  if (threadIdx.x < 6) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
      if (q == (int)threadIdx.x) r = v[q];
    partial[((size_t)dt * gridDim.x + c) * 6 + threadIdx.x] = r;
  }
}

__global__ __launch_bounds__(64) void k_pipi_mixed_final(int T, int t0, int nchunk, double norm, const double* Pn,
                                                         const double* partial, double* diag, double* pieces) {
  const int dt = blockIdx.x, t = (t0 + dt) % T;
  double v[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double s = 0.0;
    for (int c = threadIdx.x; c < nchunk; c += 64) s += partial[((size_t)dt * nchunk + c) * 6 + q];
    v[q] = wave_sum(s) * norm;
  }
  if (threadIdx.x != 0) return;
  double cpr = 0.0, cpi = 0.0, c0r = 0.0, c0i = 0.0;  // traces of the point Gram matrices at t, t0
  for (int k = 0; k < 12; ++k) {
    cpr += Pn[2 * (((size_t)t * 12 + k) * 12 + k)];
    cpi += Pn[2 * (((size_t)t * 12 + k) * 12 + k) + 1];
    c0r += Pn[2 * (((size_t)t0 * 12 + k) * 12 + k)];
    c0i += Pn[2 * (((size_t)t0 * 12 + k) * 12 + k) + 1];
  }
  double* d = diag + 2 * dt;
  d[0] = cpr * v[0] - cpi * v[1];  // D0 = Cp Cs
  d[1] = cpr * v[1] + cpi * v[0];
  d[2 * T] = v[2] * c0r - v[3] * c0i;  // D1 = L Cp(0)
  d[2 * T + 1] = v[2] * c0i + v[3] * c0r;
  d[4 * T] = v[4];  // D2
  d[4 * T + 1] = v[5];
  d[6 * T] = v[4];  // D3 = conj(D2)
  d[6 * T + 1] = -v[5];
  if (pieces) {
    double* p = pieces + 2 * dt;
    p[0] = cpr;
    p[1] = cpi;
    p[2 * T] = v[0];
    p[2 * T + 1] = v[1];
    p[4 * T] = v[2];
    p[4 * T + 1] = v[3];
  }
}

int pipi_mixed_chunks(int n1) { return std::max(1, std::min(n1, 64)); }

void launch_pipi_mixed(int T, int t0, int n1, int n2, const double* Pn, const double* G, const double* Fp,
                       const double* A, const double* B, double* partial, double* diag, double* pieces,
                       hipStream_t s) {
  const int nchunk = pipi_mixed_chunks(n1), rows = (n1 + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(k_pipi_mixed_partial, dim3((unsigned)nchunk, (unsigned)T), dim3(256), 0, s, T, t0, n1, n2, rows,
                     G, Fp, A, B, partial);
  hipLaunchKernelGGL(k_pipi_mixed_final, dim3((unsigned)T), dim3(64), 0, s, T, t0, nchunk,
                     1.0 / ((double)n1 * (double)n2), Pn, partial, diag, pieces);
}

// Momentum-projected pion from O(t, p) and O(t, -p): corr[dt] = sum_t0 sum_{a, b}
// Op[t0 + dt][a][b] Om[t0][b][a] over pairs of sources from different noise vectors (a / group
// != b / group), normalised by 1 / (T n (n - 1)) with n = N / group noise vectors (mode 0), or
// over all pairs without normalisation (mode 3).
__global__ __launch_bounds__(256) void k_pion_mom(int T, int N, int group, int mode, const double* Op,
                                                  const double* Om, double* corr) {
  const int dt = blockIdx.x;
  const long per = (long)N * N;
  double v[2] = {0.0, 0.0};
  for (long e = threadIdx.x; e < (long)T * per; e += 256) {
    const int t0 = (int)(e / per);
    const int a = (int)((e % per) / N), b = (int)(e % N);
    if (mode == 0 && a / group == b / group) continue;
    const int t1 = (t0 + dt) % T;
    const double* x = Op + 2 * ((size_t)t1 * per + (size_t)a * N + b);
    const double* y = Om + 2 * ((size_t)t0 * per + (size_t)b * N + a);
    v[0] += x[0] * y[0] - x[1] * y[1];
    v[1] += x[0] * y[1] + x[1] * y[0];
  }
  block_sum_n<2, 256>(v);
  const double nv = (double)(N / group);
  const double norm = mode == 0 ? 1.0 / ((double)T * nv * (nv - 1.0)) : 1.0;
  if (threadIdx.x < 2) corr[2 * dt + threadIdx.x] = (threadIdx.x == 0 ? v[0] : v[1]) * norm;
}

void launch_pion_mom(int T, int N, int group, int mode, const double* Op, const double* Om, double* corr,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_pion_mom, dim3((unsigned)T), dim3(256), 0, s, T, N, group, mode, Op, Om, corr);
}

// The same for time-diluted sources, from the compact operators Op[t][r][b] of the na sources
// rows[t][r] supported on timeslice t: a source a contributes to O(t) only at its own timeslice.
__global__ __launch_bounds__(256) void k_pion_mom_rows(int T, int N, int na, const int* rows, int group, int mode,
                                                       const double* Op, const double* Om, double* corr) {
  const int dt = blockIdx.x;
  const long per = (long)na * na;
  double v[2] = {0.0, 0.0};
  for (long e = threadIdx.x; e < (long)T * per; e += 256) {
    const int t0 = (int)(e / per);
    const int r1 = (int)((e % per) / na), r0 = (int)(e % na);
    const int t1 = (t0 + dt) % T;
    const int a = rows[(size_t)t1 * na + r1], b = rows[(size_t)t0 * na + r0];
    if (mode == 0 && a / group == b / group) continue;
    const double* x = Op + 2 * (((size_t)t1 * na + r1) * N + b);
    const double* y = Om + 2 * (((size_t)t0 * na + r0) * N + a);
    v[0] += x[0] * y[0] - x[1] * y[1];
    v[1] += x[0] * y[1] + x[1] * y[0];
  }
  block_sum_n<2, 256>(v);
  const double nv = (double)(N / group);
  const double norm = mode == 0 ? 1.0 / ((double)T * nv * (nv - 1.0)) : 1.0;
  if (threadIdx.x < 2) corr[2 * dt + threadIdx.x] = (threadIdx.x == 0 ? v[0] : v[1]) * norm;
}

void launch_pion_mom_rows(int T, int N, int na, const int* rows, int group, int mode, const double* Op,
                          const double* Om, double* corr, hipStream_t s) {
  hipLaunchKernelGGL(k_pion_mom_rows, dim3((unsigned)T), dim3(256), 0, s, T, N, na, rows, group, mode, Op, Om, corr);
}

// ------------------------------------------------------------------------------------
// pion correlator from O.  mode 0: unbiased a != b, 1/(T N (N-1)); 1: all pairs 1/(T N^2)
// (the form printed with eq. stoop); 2, 3: the same two sums without normalisation.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pion(int T, int n, const double* O, int mode, double* corr) {
  const int dt = blockIdx.x;
  double sr = 0.0, si = 0.0;
  const long per = (long)n * n;
  for (long e = threadIdx.x; e < (long)T * per; e += 256) {
    const int t0 = (int)(e / per);
    const int a = (int)((e % per) / n), b = (int)(e % n);
    if ((mode == 0 || mode == 2) && a == b) continue;
    const int t1 = (t0 + dt) % T;
    const double* x = O + 2 * ((size_t)t1 * per + (size_t)a * n + b);
    const double* y = O + 2 * ((size_t)t0 * per + (size_t)b * n + a);
    sr += x[0] * y[0] - x[1] * y[1];
    si += x[0] * y[1] + x[1] * y[0];
  }
  double v[2] = {sr, si};
  block_sum_all<2, 256>(v);
  if (threadIdx.x == 0) {
    double norm = 1.0;
    if (mode == 0) norm = (double)T * n * (n - 1);
    if (mode == 1) norm = (double)T * n * n;
    corr[2 * dt] = v[0] / norm;
    corr[2 * dt + 1] = v[1] / norm;
  }
}

void launch_pion_corr(int T, int n, const double* O, int mode, double* corr, hipStream_t s) {
  hipLaunchKernelGGL(k_pion, dim3(T), dim3(256), 0, s, T, n, O, mode, corr);
}

// ------------------------------------------------------------------------------------
// pi-pi zero-momentum pieces from four disjoint noise groups of m = N/4 sources
// (Sec. 7: independent noise for each propagator of a diagram).  B^{gh}(t) is the m x m
// block of O(t) with rows in group g and columns in group h.
//   L^{gh}(t1,t2) = tr[B^{gh}(t1) B^{hg}(t2)] / m^2
//   D0(dt) = 1/T sum_t0 L^{12}(t1,t0) L^{34}(t1,t0)          t1 = t0 + dt
//   D1(dt) = 1/T sum_t0 L^{12}(t1,t1) L^{34}(t0,t0)          (no vacuum subtraction)
//   D2(dt) = 1/T sum_t0 tr[B^{12}(t0) B^{23}(t1) B^{34}(t1) B^{41}(t0)] / m^4
//   D3(dt) = 1/T sum_t0 tr[B^{12}(t1) B^{23}(t1) B^{34}(t0) B^{41}(t0)] / m^4
//   vac(t) = L^{12}(t,t)
// One block per dt; the 4-fold traces use two m x m products staged in LDS (m <= 32).
// ------------------------------------------------------------------------------------
constexpr int PIPI_MMAX = 32;

__device__ __forceinline__ cx<double> oblk(const double* O, int N, int m, int t, int g, int h, int i, int j) {
  const double* p = O + 2 * (((size_t)t * N + g * m + i) * N + h * m + j);
  return mk(p[0], p[1]);
}

__device__ cx<double> loop2_block(const double* O, int N, int m, int g, int h, int t1, int t2, double* lds) {
  double sr = 0.0, si = 0.0;
  for (int e = threadIdx.x; e < m * m; e += 256) {
    const int i = e / m, j = e % m;
    cx<double> p = oblk(O, N, m, t1, g, h, i, j) * oblk(O, N, m, t2, h, g, j, i);
    sr += p.re;
    si += p.im;
  }
  double v[2] = {sr, si};
  block_sum_all<2, 256>(v);
  __shared__ cx<double> res;
  if (threadIdx.x == 0) res = mk(v[0], v[1]);
  __syncthreads();
  cx<double> r = res;
  __syncthreads();
  return r;
}

__device__ cx<double> loop4_block(const double* O, int N, int m, int ta, int tb, int tc, int td, cx<double>* M1,
                                  cx<double>* M2, double* lds) {
  for (int e = threadIdx.x; e < m * m; e += 256) {  // M1 = B12(ta) B23(tb)
    const int i = e / m, k = e % m;
    cx<double> acc = mk(0.0, 0.0);
    for (int j = 0; j < m; ++j) acc = acc + oblk(O, N, m, ta, 0, 1, i, j) * oblk(O, N, m, tb, 1, 2, j, k);
    M1[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * m; e += 256) {  // M2 = M1 B34(tc)
    const int i = e / m, l = e % m;
    cx<double> acc = mk(0.0, 0.0);
    for (int k = 0; k < m; ++k) acc = acc + M1[i * m + k] * oblk(O, N, m, tc, 2, 3, k, l);
    M2[e] = acc;
  }
  __syncthreads();
  double sr = 0.0, si = 0.0;
  for (int e = threadIdx.x; e < m * m; e += 256) {  // tr(M2 B41(td))
    const int i = e / m, l = e % m;
    cx<double> p = M2[i * m + l] * oblk(O, N, m, td, 3, 0, l, i);
    sr += p.re;
    si += p.im;
  }
  double v[2] = {sr, si};
  block_sum_all<2, 256>(v);
  __shared__ cx<double> res;
  if (threadIdx.x == 0) res = mk(v[0], v[1]);
  __syncthreads();
  cx<double> r = res;
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_pipi(int T, int N, const double* O, double* diag, double* vac) {
  __shared__ cx<double> M1[PIPI_MMAX * PIPI_MMAX];
  __shared__ cx<double> M2[PIPI_MMAX * PIPI_MMAX];
  __shared__ double lds[8];
  const int dt = blockIdx.x;
  const int m = N / 4;
  const double m2 = (double)m * m, m4 = m2 * m2;
  cx<double> d0 = mk(0.0, 0.0), d1 = d0, d2 = d0, d3 = d0;
  for (int t0 = 0; t0 < T; ++t0) {
    const int t1 = (t0 + dt) % T;
    cx<double> l12 = loop2_block(O, N, m, 0, 1, t1, t0, lds);
    cx<double> l34 = loop2_block(O, N, m, 2, 3, t1, t0, lds);
    d0 = d0 + (1.0 / (m2 * m2)) * (l12 * l34);
    cx<double> v12 = loop2_block(O, N, m, 0, 1, t1, t1, lds);
    cx<double> v34 = loop2_block(O, N, m, 2, 3, t0, t0, lds);
    d1 = d1 + (1.0 / (m2 * m2)) * (v12 * v34);
    d2 = d2 + (1.0 / m4) * loop4_block(O, N, m, t0, t1, t1, t0, M1, M2, lds);
    d3 = d3 + (1.0 / m4) * loop4_block(O, N, m, t1, t1, t0, t0, M1, M2, lds);
  }
  if (threadIdx.x == 0) {
    const double it = 1.0 / T;
    diag[2 * (0 * T + dt)] = it * d0.re;
    diag[2 * (0 * T + dt) + 1] = it * d0.im;
    diag[2 * (1 * T + dt)] = it * d1.re;
    diag[2 * (1 * T + dt) + 1] = it * d1.im;
    diag[2 * (2 * T + dt)] = it * d2.re;
    diag[2 * (2 * T + dt) + 1] = it * d2.im;
    diag[2 * (3 * T + dt)] = it * d3.re;
    diag[2 * (3 * T + dt) + 1] = it * d3.im;
  }
  if (vac) {
    cx<double> v = loop2_block(O, N, m, 0, 1, dt, dt, lds);
    if (threadIdx.x == 0) {
      vac[2 * dt] = v.re / m2;
      vac[2 * dt + 1] = v.im / m2;
    }
  }
}

void launch_pipi(int T, int n, const double* O, double* diag, double* vac, hipStream_t s) {
  hipLaunchKernelGGL(k_pipi, dim3(T), dim3(256), 0, s, T, n, O, diag, vac);
}

}  // namespace a2a
