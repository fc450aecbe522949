// a2a_contract.h -- host-side declarations of the contraction, fill, dilution and point-source
// launchers (internal to liba2a).
#pragma once

#include <hip/hip_runtime.h>

#include "a2a_device.h"

namespace a2a {

// stochastic operators O[t][a][b] (Sec. 7, eq. stoop) and the correlators built from them
// (g5 = 0: without gamma_5, the Gram matrices <eta_a, X_b>_t; timeslices t_first .. + nt)
// phase (complex per spatial site, or null): momentum projection O = sum_y phase(y) eta^dag g5 X
// rows (or null), [T][na]: row r of O(t) is source rows[t na + r] (time-diluted sources);
// without rows, na > 0 takes rows 0 .. na - 1 of eta (O is na x n), na <= 0 means na = n
void launch_stoch_ops(const Geo& g, int n, const double* eta, const double* X, double* partial, int nchunk,
                      double* O, hipStream_t s, int g5 = 1, int t_first = 0, int nt = -1,
                      const double* phase = nullptr, const int* rows = nullptr, int na = 0);
void launch_pion_mom_rows(int T, int N, int na, const int* rows, int group, int mode, const double* Op,
                          const double* Om, double* corr, hipStream_t s);
void launch_pion_mom(int T, int N, int group, int mode, const double* Op, const double* Om, double* corr,
                     hipStream_t s);
// the 12 unit sources at one site (canonical complex128 [12][V][12])
void launch_point_sources(const Geo& g, long site, double* out, hipStream_t s);
// pi-pi diagrams from point and stochastic propagators, from the timeslice Gram matrices
// Pn [T][12][12], G and Fp [T][n1][n2], A [12][n1] (at t0), B [T][n2][12]; partial holds
// pipi_mixed_chunks(n1) x T x 6 doubles; diag [4][T] and pieces [3][T] complex (device)
int pipi_mixed_chunks(int n1);
void launch_pipi_mixed(int T, int t0, int n1, int n2, const double* Pn, const double* G, const double* Fp,
                       const double* A, const double* B, double* partial, double* diag, double* pieces,
                       hipStream_t s);
void launch_dilute(const Geo& g, int nnoise, int scheme, int D, const double* noise, double* out, hipStream_t s);
void launch_gram_corr(int T, int n, const double* E, const double* F, double* corr, hipStream_t s);

// outer-product fill (Sec. 7, eq. Sfill) on the FP64 matrix cores:
// C(m, n) = scale sum_k P(m, k) conj(Q(n, k)), complex operands with element strides
struct FillArgs {
  const double* P[2];  // operand pairs: [0] the product to store or S1, [1] S2 (contract mode)
  const double* Q[2];
  long long pm, pk, qm, qk;  // P(m, k) = P[m pm + k pk], Q(n, k) = Q[n qm + k qk] (complex elements)
  long long pz, qz;          // operand offsets per grid.y index (sink timeslice)
  int M, N, K;
  double scale;
  double* out;               // fill mode: C(m, n) at out[z oz + m om + n on]
  long long om, on, oz;
  int dagger;                // store the spin-colour dagger of every 12 x 12 block
  double* partial;           // contract mode: [z][block] complex partials of sum C1 conj(C2)
};
long long fill_blocks(int M, int N);
void launch_fill(const FillArgs& a, int nz, hipStream_t s);
void launch_fill_contract(const FillArgs& a, int nz, double* corr, hipStream_t s);
void launch_pion_corr(int T, int n, const double* O, int mode, double* corr, hipStream_t s);
void launch_pipi(int T, int n, const double* O, double* diag, double* vac, hipStream_t s);

}  // namespace a2a
