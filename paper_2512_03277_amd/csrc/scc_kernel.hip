// Batched SCC-DFTB unit evaluation on CDNA4 (gfx950).
//
// One workgroup evaluates one unit geometry ("job") at a time and loops over
// jobs persistently (job = blockIdx.x + k * gridDim.x), so per-workgroup
// scratch can be preallocated and the job order is fixed (deterministic).
//
// Per job (second-order SCC-DFTB, Elstner et al. 1998, which the paper uses
// for every cell - Computational details):
//   H0, S from the Slater-Koster rules (Slater & Koster 1954, Table I) with the
//   exponential radial tables; gamma from Elstner's kernel (tau = 16U/5).
//   An S-orthonormal basis X (X^T S X = I) is built by Cholesky
//   orthonormalisation of the identity (cold) or of the stored MO basis of the
//   unit (warm).  Each SCC iteration forms H = H0 + 1/2 S o (V_a + V_b),
//   A = X^T H X, and diagonalises A by cyclic parallel Jacobi whose rotations
//   are applied straight to X, so X becomes the MO coefficient matrix C and
//   stays the (near-diagonalising) basis of the next iteration.  Aufbau
//   occupation of the n_occ lowest levels, P = 2 C_occ C_occ^T, Mulliken
//   charges, Johnson's modified Broyden mixing.  After convergence:
//   W = 2 C_occ eps C_occ^T, E = Tr(P H0) + 1/2 Dq gamma Dq + E_rep and the
//   pair-wise force contraction, all with fixed-order reductions.
//
// LDS holds the three n x n working matrices (X, A, T) with padded rows; H0,
// S and gamma live in per-workgroup global scratch (L2 resident) and are read
// with coalesced (row or, by symmetry, column) walks.
#include <math.h>

#include "internal.h"

namespace cavdftb {
namespace {

constexpr int kMaxSweeps = 30;
constexpr double kJacobiThr = 1.0e-14;  // off-diagonal threshold (hartree)
constexpr double kGapMin = 1.0e-6;
constexpr int kStagnation = 20;  // iterations without a new smallest residual before giving up
constexpr int kStagnationFailed = 5;  // the same for a unit whose last undisplaced SCC did not converge
// warm orthonormalisation: Newton-Schulz from max|C0^T S C0 - I| <= kNsStart
constexpr double kNsStart = 0.1;
constexpr double kNsTol = 1.0e-15;
constexpr int kNsMaxSteps = 8;
// occupied-virtual step: used while the occupied columns of X stay separated
// from the virtual ones (diagonal gap > kOvGap), the coupling is small
// (max |A_ov| < kOvAngle gap) and the within-block couplings are small
// (max |A_oo|, |A_vv| off the diagonal < kOvOff gap); else full Jacobi
constexpr double kOvGap = 0.02;
constexpr double kOvAngle = 0.1;
constexpr double kOvOff = 0.2;
constexpr double kOvNorm = 1.0e-2;  // bound on ||L||_F^2 for the Neumann series of (I + L^T L)^{-1}
constexpr int kSylvester = 2;       // Jacobi sweeps on the Sylvester equation
constexpr bool kMatrixCores = true; // dense products on the FP64 matrix cores (NMAX % 16 == 0)

// ---------------------------------------------------------------- SK rules
__device__ __forceinline__ void radial(const DevParams& P, int t, double r, double& h, double& s, double& hp,
                                       double& sp) {
  h = P.sk[t][0] * exp(-P.sk[t][1] * r);
  s = P.sk[t][2] * exp(-P.sk[t][3] * r);
  hp = -P.sk[t][1] * h;
  sp = -P.sk[t][3] * s;
}

// Two-centre block <i on A | . | j on B> for d = R_B - R_A (nA x nB, row-major
// with leading dimension 4).
__device__ void sk_block(const DevParams& P, int spA, int spB, const double d[3], double H[16], double S[16]) {
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double ir = 1.0 / r;
  const double u[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
  int t_ss, t_sp, t_ps;
  if (spA == 0 && spB == 0) {
    t_ss = 0; t_sp = 1; t_ps = 1;
  } else if (spA == 0) {  // O-H
    t_ss = 4; t_sp = -1; t_ps = 5;
  } else if (spB == 0) {  // H-O
    t_ss = 4; t_sp = 5; t_ps = -1;
  } else {
    t_ss = 6; t_sp = -1; t_ps = -1;
  }
  const int nA = spA == 0 ? 4 : 1, nB = spB == 0 ? 4 : 1;
  double h, s, hp, spr;
  radial(P, t_ss, r, h, s, hp, spr);
  H[0] = h;
  S[0] = s;
  if (nB == 4) {  // s on A, p on B:  u_b V
    radial(P, t_sp, r, h, s, hp, spr);
    for (int b = 0; b < 3; ++b) {
      H[1 + b] = u[b] * h;
      S[1 + b] = u[b] * s;
    }
  }
  if (nA == 4) {  // p on A, s on B:  -u_a V
    radial(P, t_ps, r, h, s, hp, spr);
    for (int a = 0; a < 3; ++a) {
      H[(1 + a) * 4] = -u[a] * h;
      S[(1 + a) * 4] = -u[a] * s;
    }
  }
  if (nA == 4 && nB == 4) {  // p-p
    double hs, ss, hsp, ssp, hpi, spi, hpip, spip;
    radial(P, 2, r, hs, ss, hsp, ssp);
    radial(P, 3, r, hpi, spi, hpip, spip);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const double dl = a == b ? 1.0 : 0.0;
        const int e = (1 + a) * 4 + 1 + b;
        H[e] = u[a] * u[b] * (hs - hpi) + dl * hpi;
        S[e] = u[a] * u[b] * (ss - spi) + dl * spi;
      }
  }
}

// Gradient contribution of the pair (A, B) with respect to d = R_B - R_A:
// g += sum_ij [ 2 P_ij dH0_ij - 2 (W_ij - 1/2 P_ij (V_A + V_B)) dS_ij ].
// With u = d / r and du_a / dd_k = (delta_ak - u_a u_k) / r each block reduces
// to contractions of its weights c (the H and S weights folded together) with u:
//   s-p, value u_b f:  sum_b c_b d(u_b f) = (f c + u (c.u)(r f' - f)) / r
//   p-p, value u_a u_b (f_sig - f_pi) + delta_ab f_pi:
//     sum_ab c_ab d(.) = (f_sig - f_pi) [(c + c^T) u - 2 (u^T c u) u] / r
//                        + u [(f_sig' - f_pi') u^T c u + f_pi' tr c]
// so a block costs one batch of weight loads per row and O(16) products.
__device__ void pair_band_grad(const DevParams& P, int spA, int spB, const double d[3], const double* Pm,
                               const double* Wm, int ld, int oA, int oB, double vab, double g[3]) {
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double ir = 1.0 / r;
  const double u[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
  const bool pA = spA == 0, pB = spB == 0;  // oxygen carries the p shell
  const int t_ss = pA ? (pB ? 0 : 4) : (pB ? 4 : 6);
  const int t_sp = pA && pB ? 1 : 5;
  // weights of element (i, j): H 2 P_ij, S -2 W_ij + P_ij (V_A + V_B)
  auto wt = [&](int i, int j, double& ch, double& cs) {
    const double pij = Pm[i * ld + j];
    ch = 2.0 * pij;
    cs = pij * vab - 2.0 * Wm[i * ld + j];
  };
  double rad = 0.0;                // coefficient of u
  double gv[3] = {0.0, 0.0, 0.0};  // remaining terms, times 1 / r
  double h, s, hp, sp;
  {
    double ch, cs;
    wt(oA, oB, ch, cs);
    radial(P, t_ss, r, h, s, hp, sp);
    rad += ch * hp + cs * sp;
  }
  if (pA || pB) {
    radial(P, t_sp, r, h, s, hp, sp);
    const double fh = hp - h * ir, fs = sp - s * ir;
    if (pB) {  // <s_A | p_B,b> = u_b V
      double ch[3], cs[3];
#pragma unroll
      for (int b = 0; b < 3; ++b) wt(oA, oB + 1 + b, ch[b], cs[b]);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        gv[b] += ch[b] * h + cs[b] * s;
        rad += u[b] * (ch[b] * fh + cs[b] * fs);
      }
    }
    if (pA) {  // <p_A,a | s_B> = -u_a V
      double ch[3], cs[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) wt(oA + 1 + a, oB, ch[a], cs[a]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        gv[a] -= ch[a] * h + cs[a] * s;
        rad -= u[a] * (ch[a] * fh + cs[a] * fs);
      }
    }
  }
  if (pA && pB) {
    double hs, ss, hsp, ssp, hpi, spi, hpip, spip;
    radial(P, 2, r, hs, ss, hsp, ssp);
    radial(P, 3, r, hpi, spi, hpip, spip);
    const double dh = hs - hpi, ds = ss - spi, dhp = hsp - hpip, dsp = ssp - spip;
    double mu[3] = {0.0, 0.0, 0.0}, mtu[3] = {0.0, 0.0, 0.0};
    double unu = 0.0, tr = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double ch[3], cs[3];
#pragma unroll
      for (int b = 0; b < 3; ++b) wt(oA + 1 + a, oB + 1 + b, ch[b], cs[b]);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double m = dh * ch[b] + ds * cs[b];
        mu[a] += m * u[b];
        mtu[b] += m * u[a];
        unu += u[a] * u[b] * (dhp * ch[b] + dsp * cs[b]);
        if (a == b) tr += hpip * ch[b] + spip * cs[b];
      }
    }
    const double umu = u[0] * mu[0] + u[1] * mu[1] + u[2] * mu[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) gv[k] += mu[k] + mtu[k];
    rad += unu + tr - 2.0 * umu * ir;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) g[k] += rad * u[k] + gv[k] * ir;
}

// Elstner gamma and d gamma / dR for distinct sites: gamma = 1/R - S with
// S(ta, tb, R) from the Coulomb integral of two exponential densities
// (tau = 16 U / 5).  The closed form for ta != tb is a removable singularity
// at ta = tb whose two terms cancel like 1/(ta - tb)^3, so near-equal
// exponents use its expansion about t = (ta + tb)/2 instead: with
// y = t R, x = (ta - tb)/(ta + tb),
//   S     = t   e^{-y} sum_k c_k(y) x^k,     k = 0, 2, ..., 14,
//   dS/dR = t^2 e^{-y} sum_k (c_k' - c_k)(y) x^k,
// c_0 = (y^3 + 9y^2 + 33y + 48)/(48y) being the equal-exponent form.  The
// c_k are polynomials in y (numerators below, ascending powers, over the
// denominators kGsDen), derived by expanding the closed form in
// delta = (ta - tb)/2.  For x < 0.1 the truncation error is below 1e-15 of
// 1/R; above it the closed form loses less than 1e-14 of 1/R.
__constant__ double kGsNum[7][17] = {
    {180, 180, 75, 15, 1},
    {-840, -840, 0, 280, 133, 21, 1},
    {0, 0, -7560, -7560, -2268, 252, 207, 27, 1},
    {0, 0, 0, 0, -33264, -33264, -9504, 0, 297, 33, 1},
    {0, 0, 0, 0, 0, 0, -102960, -102960, -25740, -572, 403, 39, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, -257400, -257400, -56160, -1560, 525, 45, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, -556920, -556920, -107100, -3060, 663, 51, 1}};
__constant__ double kGdNum[7][17] = {
    {0, -30, -30, -11, -1},
    {0, 840, 840, 252, -28, -15, -1},
    {0, -15120, -15120, -1512, 3528, 990, -18, -19, -1},
    {0, 0, 0, -133056, -133056, -23760, 9504, 2376, 0, -23, -1},
    {0, 0, 0, 0, 0, -617760, -617760, -102960, 20592, 4602, 26, -27, -1},
    {0, 0, 0, 0, 0, 0, 0, -2059200, -2059200, -304200, 39000, 7860, 60, -31, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, -5569200, -5569200, -728280, 67320, 12342, 102, -35, -1}};
__constant__ double kGsDen[7] = {480.0, 13440.0, 725760.0, 63866880.0, 8302694400.0, 1494484992000.0,
                                 355687428096000.0};
constexpr double kGammaSeriesX = 0.1;

__device__ void gamma_pair(double ua, double ub, double r, double& g, double& dg) {
  const double ta = 3.2 * ua, tb = 3.2 * ub;  // 16 U / 5
  const double x = (ta - tb) / (ta + tb);
  double s, ds;
  if (fabs(x) < kGammaSeriesX) {
    const double t = 0.5 * (ta + tb), y = t * r, e = exp(-y), x2 = x * x;
    double ss = 0.0, sd = 0.0;  // sum over k >= 2, Horner in x^2 from the top
    for (int k = 6; k >= 0; --k) {
      double ps = 0.0, pd = 0.0;
      for (int j = 16; j >= 0; --j) {
        ps = fma(ps, y, kGsNum[k][j]);
        pd = fma(pd, y, kGdNum[k][j]);
      }
      ss = fma(ss, x2, ps / kGsDen[k]);
      sd = fma(sd, x2, pd / kGsDen[k]);
    }
    ss *= x2;
    sd *= x2;
    // k = 0 in the equal-exponent form
    const double poly = 1.0 / r + 11.0 * t / 16.0 + 3.0 * t * t * r / 16.0 + t * t * t * r * r / 48.0;
    const double dpoly = -1.0 / (r * r) - t / r - 0.5 * t * t - 7.0 * t * t * t * r / 48.0 -
                         t * t * t * t * r * r / 48.0;
    s = e * (poly + t * ss);
    ds = e * (dpoly + t * t * sd);
  } else {
    s = 0.0;
    ds = 0.0;
    for (int k = 0; k < 2; ++k) {
      const double a = k == 0 ? ta : tb, b = k == 0 ? tb : ta;
      const double d2 = a * a - b * b;
      const double k1 = b * b * b * b * a / (2.0 * d2 * d2);
      const double k2 = (b * b * b * b * b * b - 3.0 * a * a * b * b * b * b) / (d2 * d2 * d2);
      const double e = exp(-a * r);
      const double v = e * (k1 - k2 / r);
      s += v;
      ds += -a * v + e * (k2 / (r * r));
    }
  }
  g = 1.0 / r - s;
  dg = -1.0 / (r * r) - ds;
}

// ---------------------------------------------------------------- block helpers
// Reductions: butterfly within each 64-lane wave (cross-lane shuffles, fixed
// order), then the per-wave partials through LDS in wave order.  Every thread
// gets the result; the trailing barrier lets red be reused at once.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int NT>
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

template <int NT>
__device__ double block_max(double v, double* red) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// value of v held by lane k of the wave (k uniform)
__device__ __forceinline__ double lane_bcast(double v, int k) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// orders the LDS accesses of one wave across this point (no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// v[0] <- block max, v[1] <- block sum (nw = waves per block)
__device__ __forceinline__ void block_max_sum(double (&v)[2], double* red, int nw) {
  v[0] = wave_max(v[0]);
  v[1] = wave_sum(v[1]);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = v[0];
    red[nw + (threadIdx.x >> 6)] = v[1];
  }
  __syncthreads();
  double mx = red[0], sm = red[nw];
  for (int w = 1; w < nw; ++w) {
    mx = fmax(mx, red[w]);
    sm += red[nw + w];
  }
  v[0] = mx;
  v[1] = sm;
  __syncthreads();
}

// K maxima at once (v updated in place)
template <int NT, int K>
__device__ void block_max_n(double (&v)[K], double* red) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_max(v[k]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * (NT / 64) + (threadIdx.x >> 6)] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double r = red[k * (NT / 64)];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) r = fmax(r, red[k * (NT / 64) + w]);
    v[k] = r;
  }
  __syncthreads();
}

// Working-matrix layout: NMAX x LD doubles, LD = NMAX + 1 so that a column
// walk (consecutive rows, one column) spreads over the LDS banks.  For
// NMAX <= 64 the three working matrices live in LDS; larger buckets keep them
// in per-workgroup global scratch (L2 / Infinity-Cache resident).  Elementwise
// loops use lane = column (tid & 63, in chunks of 64) and row groups tid >> 6,
// so no integer division appears in the hot loops.
template <int NMAX, int NT>
struct Cfg {
  static constexpr int LD = NMAX + 1;
  static constexpr int G = (NT == 256) ? 16 : 8;
  static constexpr int TM = NMAX / G;
  static constexpr int TMB = TM < 4 ? TM : 4;  // rows/cols per thread and output block
  static constexpr int BLK = G * TMB;           // output block edge
  static constexpr int RG = NT / 64;            // row groups of 64 lanes
  static constexpr bool GM = NMAX > 64;         // working matrices in global scratch
  static_assert(TM * G == NMAX, "tile mismatch");
};

// Register-blocked product over the leading nr x nc block:
//   acc(r, c) = sum_{k < kd} opA(r, k) opB(k, c) + s2 sum_{k < kd2} A2[r][k] B2[k][c]
// with opA(r, k) = A[r][k] (TA: A[k][r]) and opB(k, c) = B[k][c] (TB: B[c][k]);
// epi(r, c, acc) consumes each element (the same thread owns (r, c) for equal nr,
// nc, so consecutive products can chain through it without a barrier).  The k
// loops are unrolled with all loads of a step issued before its multiply-adds
// (LDS latency is the bound at these sizes); the order over k is sequential.
template <int NMAX, int NT, bool TA, bool TB, class Epi>
__device__ __forceinline__ void gemm_v(const double* __restrict__ A, const double* __restrict__ B, int kd,
                       const double* __restrict__ A2, const double* __restrict__ B2, int kd2, double s2, int nr,
                       int nc, Epi epi) {
  constexpr int G = Cfg<NMAX, NT>::G, TMB = Cfg<NMAX, NT>::TMB, BLK = Cfg<NMAX, NT>::BLK, LD = Cfg<NMAX, NT>::LD;
  constexpr int UK = TMB >= 4 ? 2 : 4;  // k unroll within the register budget
  const int tx = threadIdx.x % G, ty = threadIdx.x / G;
  for (int bi = 0; bi < nr; bi += BLK)
    for (int bj = 0; bj < nc; bj += BLK) {
      // rows / columns past the logical nr x nc block are clamped onto its last row /
      // column: every read stays inside the operands, the extra results are not stored
      int row[TMB], col[TMB];
#pragma unroll
      for (int r = 0; r < TMB; ++r) {
        row[r] = min(bi + ty + G * r, nr - 1);
        col[r] = min(bj + tx + G * r, nc - 1);
      }
      double acc[TMB][TMB];
#pragma unroll
      for (int r = 0; r < TMB; ++r)
#pragma unroll
        for (int c = 0; c < TMB; ++c) acc[r][c] = 0.0;
      int k = 0;
      for (; k + UK <= kd; k += UK) {
        double av[UK][TMB], bv[UK][TMB];
#pragma unroll
        for (int u = 0; u < UK; ++u)
#pragma unroll
          for (int r = 0; r < TMB; ++r) {
            av[u][r] = TA ? A[(k + u) * LD + row[r]] : A[row[r] * LD + k + u];
            bv[u][r] = TB ? B[col[r] * LD + k + u] : B[(k + u) * LD + col[r]];
          }
#pragma unroll
        for (int u = 0; u < UK; ++u)
#pragma unroll
          for (int r = 0; r < TMB; ++r)
#pragma unroll
            for (int c = 0; c < TMB; ++c) acc[r][c] = fma(av[u][r], bv[u][c], acc[r][c]);
      }
      for (; k < kd; ++k) {
        double av[TMB], bv[TMB];
#pragma unroll
        for (int r = 0; r < TMB; ++r) {
          av[r] = TA ? A[k * LD + row[r]] : A[row[r] * LD + k];
          bv[r] = TB ? B[col[r] * LD + k] : B[k * LD + col[r]];
        }
#pragma unroll
        for (int r = 0; r < TMB; ++r)
#pragma unroll
          for (int c = 0; c < TMB; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
      }
      for (k = 0; k < kd2; ++k) {
        double av[TMB], bv[TMB];
#pragma unroll
        for (int r = 0; r < TMB; ++r) {
          av[r] = A2[row[r] * LD + k];
          bv[r] = s2 * B2[k * LD + col[r]];
        }
#pragma unroll
        for (int r = 0; r < TMB; ++r)
#pragma unroll
          for (int c = 0; c < TMB; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
      }
#pragma unroll
      for (int r = 0; r < TMB; ++r)
#pragma unroll
        for (int c = 0; c < TMB; ++c) {
          const int rr = bi + ty + G * r, cc = bj + tx + G * c;
          if (rr < nr && cc < nc) epi(rr, cc, acc[r][c]);
        }
    }
}

typedef double mfma_acc4 __attribute__((ext_vector_type(4)));
// The same product on the FP64 matrix cores (v_mfma_f64_16x16x4), in blocks of
// TI x TJ output tiles of 16 x 16 per wave: the TI A fragments and TJ B
// fragments of a k-step feed TI * TJ independent MFMAs, and the loads of UK
// k-steps are issued before their MFMAs (latency hiding for LDS and for
// matrices in global scratch).  Lane l feeds A[t_r + l % 16][k0 + l / 16] and
// B[k0 + l / 16][t_c + l % 16] and receives C[t_r + l / 16 + 4 i][t_c + l % 16]
// in accumulator i.  Rows, columns and k past the logical operands read as zero
// (no access outside them); the extra results are never passed to epi.
template <int NMAX, int NT, bool TA, bool TB, int TI, int TJ, int UK, class Epi>
__device__ __forceinline__ void gemm_mt(const double* __restrict__ A, const double* __restrict__ B, int kd,
                        const double* __restrict__ A2, const double* __restrict__ B2, int kd2, double s2, int nr,
                        int nc, Epi epi) {
  static_assert(NMAX % 16 == 0, "matrix-core tiles need NMAX % 16 == 0");
  constexpr int LD = Cfg<NMAX, NT>::LD;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tr = (nr + 16 * TI - 1) / (16 * TI), tcn = (nc + 16 * TJ - 1) / (16 * TJ);
  for (int t = wave; t < tr * tcn; t += NT / 64) {
    const int r0 = (t / tcn) * 16 * TI, c0 = (t % tcn) * 16 * TJ;
    int ra[TI], cb[TJ];
    bool rin[TI], cin[TJ];
#pragma unroll
    for (int g = 0; g < TI; ++g) {
      ra[g] = r0 + 16 * g + li;
      rin[g] = ra[g] < nr;
    }
#pragma unroll
    for (int g = 0; g < TJ; ++g) {
      cb[g] = c0 + 16 * g + li;
      cin[g] = cb[g] < nc;
    }
    mfma_acc4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) acc[i][j] = (mfma_acc4){0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < kd; k0 += 4 * UK) {
      double av[UK][TI], bv[UK][TJ];
#pragma unroll
      for (int u = 0; u < UK; ++u) {
        const int k = k0 + 4 * u + lk;
        const bool kin = k < kd;
#pragma unroll
        for (int g = 0; g < TI; ++g) av[u][g] = (kin && rin[g]) ? (TA ? A[k * LD + ra[g]] : A[ra[g] * LD + k]) : 0.0;
#pragma unroll
        for (int g = 0; g < TJ; ++g) bv[u][g] = (kin && cin[g]) ? (TB ? B[cb[g] * LD + k] : B[k * LD + cb[g]]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UK; ++u)
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][i], bv[u][j], acc[i][j], 0, 0, 0);
    }
    for (int k0 = 0; k0 < kd2; k0 += 4) {
      const int k = k0 + lk;
      const bool kin = k < kd2;
      double av[TI], bv[TJ];
#pragma unroll
      for (int g = 0; g < TI; ++g) av[g] = (kin && rin[g]) ? A2[ra[g] * LD + k] : 0.0;
#pragma unroll
      for (int g = 0; g < TJ; ++g) bv[g] = (kin && cin[g]) ? s2 * B2[k * LD + cb[g]] : 0.0;
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = r0 + 16 * i + lk + 4 * q, cc = c0 + 16 * j + li;
          if (rr < nr && cc < nc) epi(rr, cc, acc[i][j][q]);
        }
  }
}

// matrices in global scratch (L2 / Infinity Cache latency): 2 x 2 tiles per wave,
// four k-steps of loads in flight
template <int NMAX, int NT, bool TA, bool TB, class Epi>
__device__ __forceinline__ void gemm_mg(const double* __restrict__ A, const double* __restrict__ B, int kd,
                        const double* __restrict__ A2, const double* __restrict__ B2, int kd2, double s2, int nr,
                        int nc, Epi epi) {
  gemm_mt<NMAX, NT, TA, TB, 2, 2, 4>(A, B, kd, A2, B2, kd2, s2, nr, nc, epi);
}

// small products (the occupied-virtual step) on the matrix cores where the tiles fit
// the buffers (one tile per wave, four k-steps of loads in flight), else on the
// vector units; the n x n products (gemm_g) stay on the
// vector units for LDS-resident matrices, which measured faster there, and use the
// matrix cores when the matrices live in global scratch
template <int NMAX, int NT, bool TA, bool TB, class Epi>
__device__ __forceinline__ void gemm_e(const double* __restrict__ A, const double* __restrict__ B, int kd,
                                       const double* __restrict__ A2, const double* __restrict__ B2, int kd2,
                                       double s2, int nr, int nc, Epi epi) {
  if constexpr (kMatrixCores && Cfg<NMAX, NT>::GM)
    gemm_mg<NMAX, NT, TA, TB>(A, B, kd, A2, B2, kd2, s2, nr, nc, epi);
  else if constexpr (kMatrixCores && NMAX % 16 == 0)
    gemm_mt<NMAX, NT, TA, TB, 1, 1, 4>(A, B, kd, A2, B2, kd2, s2, nr, nc, epi);
  else
    gemm_v<NMAX, NT, TA, TB>(A, B, kd, A2, B2, kd2, s2, nr, nc, epi);
}

// C[r][c] = scale sum_{k < kd} opA(r, k) opB(k, c) over the leading nr x nc block
template <int NMAX, int NT, bool TA, bool TB>
__device__ __forceinline__ void gemm_g(const double* __restrict__ A, const double* __restrict__ B,
                                       double* __restrict__ C, int nr, int nc, int kd, double scale) {
  constexpr int LD = Cfg<NMAX, NT>::LD;
  auto st = [=](int r, int c, double v) { C[r * LD + c] = scale * v; };
  if constexpr (kMatrixCores && Cfg<NMAX, NT>::GM)  // operands in L2: fewer loads per flop on the matrix cores
    gemm_mg<NMAX, NT, TA, TB>(A, B, kd, A, B, 0, 0.0, nr, nc, st);
  else
    gemm_v<NMAX, NT, TA, TB>(A, B, kd, A, B, 0, 0.0, nr, nc, st);
}

// C = op(A) B over the leading n x n block (op = transpose when TA)
template <int NMAX, int NT, bool TA>
__device__ __forceinline__ void gemm(const double* __restrict__ A, const double* __restrict__ B,
                                     double* __restrict__ C, int n) {
  gemm_g<NMAX, NT, TA, false>(A, B, C, n, n, n, 1.0);
}

// sum_{k < len} a[k sa] b[k sb], loads issued four at a time, sequential order
__device__ __forceinline__ double dotp(const double* __restrict__ a, int sa, const double* __restrict__ b, int sb,
                                       int len) {
  double s = 0.0;
  int k = 0;
  for (; k + 4 <= len; k += 4) {
    double x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = a[(k + u) * sa];
      y[u] = b[(k + u) * sb];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s = fma(x[u], y[u], s);
  }
  for (; k < len; ++k) s = fma(a[k * sa], b[k * sb], s);
  return s;
}

// Elementwise pass over the leading n x n block of two matrices in global
// scratch (leading dimension NMAX): f(i, j, g1[i][j], g2[i][j]) for every
// element, lane = column, rows dealt to the 64-lane row groups.  The loads of
// UR rows are issued before their uses, so a pass pays one memory latency per
// UR rows; indices are clamped into the block (no load leaves it) and clamped
// elements are not passed to f.
template <int NMAX, int NT, int UR = 4, class F>
__device__ __forceinline__ void ew_global(const double* __restrict__ g1, const double* __restrict__ g2, int n, F f) {
  constexpr int RG = NT / 64;
  const int lane = threadIdx.x & 63, rgrp = threadIdx.x >> 6;
  for (int j0 = 0; j0 < n; j0 += 64) {
    const int j = j0 + lane, jc = j < n ? j : n - 1;
    for (int i0 = rgrp; i0 < n; i0 += UR * RG) {
      double x[UR], y[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int i = min(i0 + u * RG, n - 1);
        x[u] = g1[i * NMAX + jc];
        y[u] = g2[i * NMAX + jc];
      }
#pragma unroll
      for (int u = 0; u < UR; ++u)
        if (i0 + u * RG < n && j < n) f(i0 + u * RG, j, x[u], y[u]);
    }
  }
}

// Site potential V_t = field . R_t + sum_s gamma_ts dq_s for t < na (gamma in
// global scratch, symmetric, leading dimension ld).  Eight lanes share a site:
// each sums every eighth term with its loads issued four at a time, then a
// butterfly over the eight lanes (fixed order); the group's first lane writes V.
template <int NT>
__device__ __forceinline__ void site_potential(const double* __restrict__ gG, int ld, const double* __restrict__ dq,
                                               const double* __restrict__ pos, const double* fld, int na,
                                               double* __restrict__ V) {
  constexpr int SP = 8, UK = 4;
  const int tid = threadIdx.x, part = tid & (SP - 1);
  for (int t0 = 0; t0 < na; t0 += NT / SP) {
    const int t = t0 + tid / SP;
    const int tc = t < na ? t : na - 1;
    double s = 0.0;
    for (int k0 = part; k0 < na; k0 += UK * SP) {
      double g[UK], q[UK];
#pragma unroll
      for (int u = 0; u < UK; ++u) {
        const int k = k0 + u * SP;
        const int kc = k < na ? k : na - 1;
        g[u] = gG[kc * ld + tc];
        q[u] = k < na ? dq[kc] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UK; ++u) s = fma(g[u], q[u], s);
    }
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 4);
    if (part == 0 && t < na) V[t] = fld[0] * pos[t * 3] + fld[1] * pos[t * 3 + 1] + fld[2] * pos[t * 3 + 2] + s;
  }
}

// e = q w + r (0 <= r < w) without an integer division: float reciprocal and one correction
__device__ __forceinline__ void split_idx(int e, int w, float inv_w, int& q, int& r) {
  q = (int)(((float)e + 0.5f) * inv_w);
  r = e - q * w;
  if (r < 0) {
    --q;
    r += w;
  } else if (r >= w) {
    ++q;
    r -= w;
  }
}

// index held by slot s in round r of the circle (round-robin) ordering of m indices
__device__ __forceinline__ int rr_index(int s, int r, int m) { return s == 0 ? 0 : 1 + (s - 1 + r) % (m - 1); }

// ---------------------------------------------------------------- full eigensolve, large buckets
// For units above 64 orbitals, whose working matrices live in global scratch,
// a full diagonalisation of A (cold start, or an SCC iteration where the
// occupied-virtual step is unsafe) runs as
//   1. Householder tridiagonalisation A = Q T Q^T (Golub & Van Loan, Alg.
//      8.3.1): reflector k from row k of the trailing matrix, p = tau A22 v,
//      w = p - (tau/2)(p.v) v, A22 -= v w^T + w v^T.  The update of step k is
//      fused with the matrix-vector product of step k + 1 (one pass over the
//      trailing matrix per step): row k + 1 is updated first, reflector k + 1
//      is formed from it, then the remaining rows are updated and multiplied
//      by it in the same walk.  Reflector k is kept in row k of A.
//   2. Eigenvalues of T by bisection on the Sturm count (one thread per
//      eigenvalue, so they come out sorted ascending).
//   3. Eigenvectors of T from the twisted factorisation at each eigenvalue
//      (Dhillon & Parlett): stationary and progressive pivots
//      d+_k = (d_k - l) - e_{k-1}^2 / d+_{k-1}, d-_k = (d_k - l) - e_k^2 / d-_{k+1},
//      twist r = argmin |d+_r + d-_r - (d_r - l)|, z_r = 1 and
//      z_k = -e_k z_{k+1} / d+_k above, z_{k+1} = -e_k z_k / d-_{k+1} below.
//      Vectors whose eigenvalues lie within kHhCluster max|l| of each other
//      are orthonormalised by two passes of modified Gram-Schmidt.
//   4. Y = Q Z by blocks of kHhNb reflectors in compact WY form
//      (Q_b = I - V T V^T, T from the recurrence of Schreiber & Van Loan),
//      every product on the FP64 matrix cores, then C = X Y.
//   5. The S-orthonormality of C is checked (C^T S C on the matrix cores); one
//      Newton-Schulz step C (3I - M)/2 cleans a small residue, a large one
//      (a failed solve) sends the iteration to cyclic Jacobi instead.
constexpr int kHhNb = 16;
constexpr int kBisect = 60;              // halvings of the Gershgorin interval (width / 2^60)
constexpr double kHhCluster = 1.0e-3;    // relative gap below which vectors are re-orthogonalised
constexpr double kHhPivmin = 1.0e-290;   // smallest pivot magnitude in the recurrences
constexpr double kHhMgsMin = 1.0e-2;     // a vector keeping less of its norm in Gram-Schmidt fails the solve
constexpr double kHhOrthoFail = 1.0e-3;  // max |C^T S C - I| above which the solve is discarded
constexpr double kHhOrthoClean = 1.0e-13;

template <int NMAX>
struct HhLds {
  double v0[NMAX], v1[NMAX], w[NMAX];
  double tt[kHhNb * kHhNb], gg[kHhNb * kHhNb];
  double sc[4];
  int fail;
};

__device__ __forceinline__ double hh_guard(double q) { return fabs(q) < kHhPivmin ? -kHhPivmin : q; }

// Full eigendecomposition of the symmetric n x n matrix A (sA) in the
// S-orthonormal basis X (sX): on success the eigenvectors C = X V, columns by
// ascending eigenvalue, are left in *out (one of sA, sT) and the eigenvalues in
// eig[0..n); false when the solve was discarded (A and the scratch buffers are
// then overwritten, X is intact).  hd/he/he2/htau: LDS vectors of NMAX doubles
// (the diagonal, off-diagonal, its square and the reflector scalars); cst: LDS
// ints of NMAX; part: LDS doubles of (NT / 64) NMAX; gS: the overlap matrix
// (row stride NMAX).
template <int NMAX, int NT>
__device__ bool eig_householder(double* __restrict__ sA, const double* __restrict__ sX, double* __restrict__ sT,
                                double* __restrict__ sD, const double* __restrict__ gS, int n, double* hd,
                                double* he, double* he2, double* htau, int* cst, double* part, HhLds<NMAX>& L,
                                double* red, double* eig, double** out) {
  constexpr int LD = Cfg<NMAX, NT>::LD;
  constexpr int RG = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* vcur = L.v0;
  double* vnext = L.v1;

  // ---- 1. tridiagonalisation.  form(k): reflector k from row k (columns > k)
  // into row k and vnext, tau_k, d_k, e_k.
  auto form = [&](int k, double* vout) {
    const double alpha = sA[k * LD + k + 1];  // read by every thread before the barrier below
    double sig = 0.0;
    for (int j = k + 2 + tid; j < n; j += NT) {
      const double x = sA[k * LD + j];
      sig = fma(x, x, sig);
    }
    sig = block_sum<NT>(sig, red);
    double beta, tau, scale;
    if (sig == 0.0) {
      beta = alpha;
      tau = 0.0;
      scale = 0.0;
    } else {
      const double nrm = sqrt(fma(alpha, alpha, sig));
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    for (int j = k + 1 + tid; j < n; j += NT) {
      const double v = j == k + 1 ? 1.0 : sA[k * LD + j] * scale;
      sA[k * LD + j] = v;
      vout[j] = v;
    }
    if (tid == 0) {
      hd[k] = sA[k * LD + k];
      he[k] = beta;
      htau[k] = tau;
    }
    __syncthreads();
  };
  // matrix-vector partials: part[w][i] = sum over rows j >= j0 with j = j0 + w (mod RG) of
  // A[j][i] v[j], for columns i in [i0, n) (A symmetric: column i read as row walks)
  auto matvec = [&](int j0, int i0, const double* v) {
    for (int c0 = i0; c0 < n; c0 += 64) {
      const int i = c0 + lane;
      double acc = 0.0;
      if (i < n)
        for (int j = j0 + wv; j < n; j += RG) acc = fma(sA[j * LD + i], v[j], acc);
      if (i < n) part[wv * NMAX + i] = acc;
    }
    __syncthreads();
  };

  form(0, vcur);
  matvec(1, 1, vcur);
  for (int k = 0; k + 2 < n; ++k) {
    // p = tau A22 v over columns [k+1, n); K = tau/2 p.v; w = p - K v
    const double tau = htau[k];
    double pv = 0.0;
    for (int i = k + 1 + tid; i < n; i += NT) {
      double p = 0.0;
#pragma unroll
      for (int g = 0; g < RG; ++g) p += part[g * NMAX + i];
      p *= tau;
      L.w[i] = p;
      pv = fma(p, vcur[i], pv);
    }
    const double kk = 0.5 * tau * block_sum<NT>(pv, red);
    for (int i = k + 1 + tid; i < n; i += NT) L.w[i] = fma(-kk, vcur[i], L.w[i]);
    __syncthreads();
    const double* v = vcur;
    const double* w = L.w;
    if (k + 3 == n) {  // last reflector: update the trailing 2 x 2 block and read off T's corner
      if (tid == 0) {
        const int a = n - 2, b = n - 1;
        const double aa = sA[a * LD + a] - 2.0 * v[a] * w[a];
        const double ab = sA[b * LD + a] - (v[b] * w[a] + w[b] * v[a]);
        const double bb = sA[b * LD + b] - 2.0 * v[b] * w[b];
        hd[a] = aa;
        hd[b] = bb;
        he[a] = ab;
        htau[a] = 0.0;
        htau[b] = 0.0;
        he[b] = 0.0;
      }
      __syncthreads();
      break;
    }
    // update row k + 1 (columns [k+1, n)), then reflector k + 1 from it
    const int r1 = k + 1;
    for (int i = r1 + tid; i < n; i += NT) sA[r1 * LD + i] -= v[r1] * w[i] + w[r1] * v[i];
    __syncthreads();
    form(r1, vnext);
    // rows [k+2, n): A[j][i] -= v_j w_i + w_j v_i for i in [k+2, n), and the
    // partial products with reflector k + 1 in the same walk
    for (int c0 = k + 2; c0 < n; c0 += 64) {
      const int i = c0 + lane;
      double acc = 0.0;
      if (i < n) {
        const double wi = w[i], vi = v[i];
        int j = k + 2 + wv;
        for (; j + RG < n; j += 2 * RG) {  // two rows of loads in flight
          const double x0 = sA[j * LD + i], x1 = sA[(j + RG) * LD + i];
          const double y0 = x0 - (v[j] * wi + w[j] * vi), y1 = x1 - (v[j + RG] * wi + w[j + RG] * vi);
          sA[j * LD + i] = y0;
          sA[(j + RG) * LD + i] = y1;
          acc = fma(y0, vnext[j], acc);
          acc = fma(y1, vnext[j + RG], acc);
        }
        for (; j < n; j += RG) {
          const double y = sA[j * LD + i] - (v[j] * wi + w[j] * vi);
          sA[j * LD + i] = y;
          acc = fma(y, vnext[j], acc);
        }
        part[wv * NMAX + i] = acc;
      }
    }
    __syncthreads();
    double* t = vcur;
    vcur = vnext;
    vnext = t;
  }
  // reflector rows hold zeros left of their first element (operands of the
  // blocked back-transform)
  for (int k = wv; k + 2 < n; k += RG)
    for (int j = lane; j <= k; j += 64) sA[k * LD + j] = 0.0;
  // T's off-diagonal squares, the Gershgorin interval and the cluster scale
  double glo = INFINITY, ghi = -INFINITY;
  for (int k = tid; k < n; k += NT) {
    const double ek = k + 1 < n ? he[k] : 0.0, ekm = k > 0 ? he[k - 1] : 0.0;
    he2[k] = ek * ek;
    const double rad = fabs(ek) + fabs(ekm);
    glo = fmin(glo, hd[k] - rad);
    ghi = fmax(ghi, hd[k] + rad);
  }
  {
    double gv[2] = {-glo, ghi};
    block_max_n<NT, 2>(gv, red);
    glo = -gv[0];
    ghi = gv[1];
  }
  if (!(glo <= ghi)) return false;  // non-finite tridiagonal matrix

  // ---- 2. eigenvalue i by bisection on the Sturm count (thread i)
  double lam = 0.0;
  if (tid < n) {
    double lo = glo, hi = ghi;
    for (int it = 0; it < kBisect; ++it) {
      const double x = 0.5 * (lo + hi);
      double q = hh_guard(hd[0] - x);
      int cnt = q < 0.0 ? 1 : 0;
      for (int k = 1; k < n; ++k) {
        q = hh_guard((hd[k] - x) - he2[k - 1] / q);
        cnt += q < 0.0 ? 1 : 0;
      }
      if (cnt > tid)
        hi = x;
      else
        lo = x;
    }
    lam = 0.5 * (lo + hi);
    eig[tid] = lam;
  }
  // ---- 3. eigenvector i of T by the twisted factorisation (thread i): d+ into
  // column i of sD, d- then the vector into column i of sT
  bool ok = true;
  if (tid < n) {
    const int i = tid;
    double dp = hh_guard(hd[0] - lam);
    sD[i] = dp;
    for (int k = 0; k + 1 < n; ++k) {
      dp = hh_guard((hd[k + 1] - lam) - he2[k] / dp);
      sD[(k + 1) * LD + i] = dp;
    }
    double dm = hh_guard(hd[n - 1] - lam);
    sT[(n - 1) * LD + i] = dm;
    double best = fabs(dp + dm - (hd[n - 1] - lam));
    int r = n - 1;
    for (int k = n - 2; k >= 0; --k) {
      dm = hh_guard((hd[k] - lam) - he2[k] / dm);
      const double g = fabs(sD[k * LD + i] + dm - (hd[k] - lam));
      if (g < best) {
        best = g;
        r = k;
      }
      sT[k * LD + i] = dm;
    }
    double z = 1.0, nrm2 = 1.0;
    sT[r * LD + i] = 1.0;
    for (int k = r - 1; k >= 0; --k) {
      z = -(he[k] / sD[k * LD + i]) * z;
      sT[k * LD + i] = z;
      nrm2 = fma(z, z, nrm2);
    }
    z = 1.0;
    for (int k = r; k + 1 < n; ++k) {
      z = -(he[k] / sT[(k + 1) * LD + i]) * z;
      sT[(k + 1) * LD + i] = z;
      nrm2 = fma(z, z, nrm2);
    }
    const double inv = 1.0 / sqrt(nrm2);
    ok = inv > 0.0 && inv < INFINITY;
    for (int k = 0; k < n; ++k) sT[k * LD + i] *= inv;
  }
  if (tid == 0) L.fail = 0;
  __syncthreads();
  if (!ok) L.fail = 1;
  // clusters of close eigenvalues: cst[i] = 1 where a new cluster starts
  const double ctol = kHhCluster * fmax(fabs(eig[0]), fabs(eig[n - 1]));
  for (int i = tid; i < n; i += NT) cst[i] = (i == 0 || eig[i] - eig[i - 1] > ctol) ? 1 : 0;
  __syncthreads();
  // modified Gram-Schmidt within each cluster, twice; wave w takes the clusters
  // whose index is w (mod RG), lanes over the vector elements
  {
    int ci = -1;
    for (int c0 = 0; c0 < n; ++c0) {
      if (!cst[c0]) continue;
      ++ci;
      int c1 = c0 + 1;
      while (c1 < n && !cst[c1]) ++c1;
      if (c1 - c0 < 2 || ci % RG != wv) continue;
      for (int rep = 0; rep < 2; ++rep)
        for (int j = c0 + 1; j < c1; ++j) {
          for (int q = c0; q < j; ++q) {
            double dt = 0.0;
            for (int k = lane; k < n; k += 64) dt = fma(sT[k * LD + q], sT[k * LD + j], dt);
            dt = wave_sum(dt);
            for (int k = lane; k < n; k += 64) sT[k * LD + j] = fma(-dt, sT[k * LD + q], sT[k * LD + j]);
          }
          double nn = 0.0;
          for (int k = lane; k < n; k += 64) nn = fma(sT[k * LD + j], sT[k * LD + j], nn);
          nn = wave_sum(nn);
          if (!(nn > kHhMgsMin * kHhMgsMin)) {
            if (lane == 0) L.fail = 1;
            nn = 1.0;
          }
          const double inv = 1.0 / sqrt(nn);
          for (int k = lane; k < n; k += 64) sT[k * LD + j] *= inv;
        }
    }
  }
  __syncthreads();
  if (L.fail) return false;

  // ---- 4. Y = Q Z in place on sT, blocks of reflectors from the last one
  const int nref = n - 2;
  for (int b = ((nref - 1) / kHhNb) * kHhNb; b >= 0; b -= kHhNb) {
    const int kb = min(kHhNb, nref - b);
    const double* V = sA + b * LD;  // row j: reflector b + j (zeros left of column b + j + 1)
    // Gram matrix G = V^T V (kb x kb)
    gemm_mt<NMAX, NT, false, true, 1, 1, 4>(V, V, n, V, V, 0, 0.0, kb, kb,
                                            [&](int r, int c, double x) { L.gg[r * kHhNb + c] = x; });
    __syncthreads();
    // T upper triangular: T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j]
    if (wv == 0) {
      if (lane < kHhNb * kHhNb) L.tt[lane] = 0.0;
      for (int l = 64 + lane; l < kHhNb * kHhNb; l += 64) L.tt[l] = 0.0;
      wave_sync();
      for (int j = 0; j < kb; ++j) {
        const double tj = htau[b + j];
        double s = 0.0;
        if (lane < j)
          for (int l = lane; l < j; ++l) s = fma(L.tt[lane * kHhNb + l], L.gg[l * kHhNb + j], s);
        wave_sync();
        if (lane < j) L.tt[lane * kHhNb + j] = -tj * s;
        if (lane == j) L.tt[j * kHhNb + j] = tj;
        wave_sync();
      }
    }
    // W1 = V Y (kb x n) into sD rows [0, kb)
    gemm_mt<NMAX, NT, false, false, 1, 2, 4>(V, sT, n, V, V, 0, 0.0, kb, n,
                                             [&](int r, int c, double x) { sD[r * LD + c] = x; });
    __syncthreads();
    // W2 = T W1 into sD rows [kHhNb, kHhNb + kb)
    for (int e = tid; e < kb * n; e += NT) {
      const int r = e / n, c = e - r * n;
      double s = 0.0;
      for (int l = r; l < kb; ++l) s = fma(L.tt[r * kHhNb + l], sD[l * LD + c], s);
      sD[(kHhNb + r) * LD + c] = s;
    }
    __syncthreads();
    // Y -= V^T-walk: Y[r][c] -= sum_j V[j][r] W2[j][c]
    gemm_mt<NMAX, NT, true, false, 2, 2, 1>(V, sD + kHhNb * LD, kb, V, V, 0, 0.0, n, n,
                                            [&](int r, int c, double x) { sT[r * LD + c] -= x; });
    __syncthreads();
  }
  // C = X Y into sA (the reflectors are no longer needed)
  gemm_mt<NMAX, NT, false, false, 2, 2, 4>(sX, sT, n, sX, sX, 0, 0.0, n, n,
                                           [&](int r, int c, double x) { sA[r * LD + c] = x; });
  __syncthreads();
  // ---- 5. M = C^T S C; clean with one Newton-Schulz step or discard
  for (int i = wv; i < n; i += RG)
    for (int j = lane; j < n; j += 64) sD[i * LD + j] = gS[i * NMAX + j];
  __syncthreads();
  gemm_mt<NMAX, NT, false, false, 2, 2, 4>(sD, sA, n, sD, sD, 0, 0.0, n, n,
                                           [&](int r, int c, double x) { sT[r * LD + c] = x; });
  __syncthreads();
  double e = 0.0;
  gemm_mt<NMAX, NT, true, false, 2, 2, 4>(sA, sT, n, sA, sA, 0, 0.0, n, n, [&](int r, int c, double x) {
    const double m = x - (r == c ? 1.0 : 0.0);
    e = fmax(e, m == m ? fabs(m) : INFINITY);
    sD[r * LD + c] = (r == c ? 1.0 : 0.0) - 0.5 * m;  // (3I - M)/2
  });
  e = block_max<NT>(e, red);
  if (!(e < kHhOrthoFail)) return false;
  if (e > kHhOrthoClean) {
    gemm_mt<NMAX, NT, false, false, 2, 2, 4>(sA, sD, n, sA, sA, 0, 0.0, n, n,
                                             [&](int r, int c, double x) { sT[r * LD + c] = x; });
    __syncthreads();
    *out = sT;
  } else {
    *out = sA;
  }
  return true;
}

struct Shared {
  int n, nocc, na, notpd;
  int bcount, bhead, sweeps, jac_iters;
  int next_job, hh_solves, hh_fails, pad2;
  double homo, lumo;
  double fld[3];  // uniform external field of the job (zero except for field jobs)
};


template <int NMAX, int NT>
// Four workgroups per CU for the 32-orbital bucket (its LDS allows it): the
// compiler then keeps 128 VGPRs and spills a few hundred bytes per lane, and
// the extra waves hide more latency than the spills cost (workload 5: 26.4 ->
// 24.6 ms per step).  The larger LDS buckets are held to two by their LDS.
__global__ __launch_bounds__(NT, NMAX == 32 ? 4 : 2) void scc_kernel(const SccArgs a) {
  constexpr int LD = Cfg<NMAX, NT>::LD;
  constexpr int RG = Cfg<NMAX, NT>::RG;
  constexpr int HALF = NMAX / 2;
  constexpr int KSTEP_A = NT / 32;  // row-of-blocks step in the Jacobi block update
  constexpr bool GM = Cfg<NMAX, NT>::GM;
  constexpr bool F_IN_X = !GM && NMAX * LD >= 3 * NT;
  __shared__ double lX[GM ? 1 : NMAX * LD];
  __shared__ double lA[GM ? 1 : NMAX * LD];
  __shared__ double lT[GM ? 1 : NMAX * LD];
  __shared__ double sFbuf[F_IN_X ? 1 : 3 * NT];
  __shared__ double sPos[NMAX * 3];
  __shared__ double sDqIn[NMAX], sDqOut[NMAX], sV[NMAX], sQ0[NMAX], sEig[NMAX], sQorb[NMAX];
  __shared__ int sOrbAtom[NMAX], sAtomOff[NMAX + 1], sSp[NMAX], sRank[NMAX];
  __shared__ double sRed[NT];
  __shared__ int sRp[2][HALF], sRq[2][HALF];
  __shared__ double sRc[2][HALF], sRs[2][HALF], sRt[2][HALF];
  __shared__ double lDF[kMaxHist * NMAX];  // Broyden dF history of the job (LDS copy)
  __shared__ double sBa[kMaxHist * kMaxHist], sBm[kMaxHist * (kMaxHist + 1)], sBc[kMaxHist], sBg[kMaxHist];
  __shared__ Shared sh;
  __shared__ HhLds<GM ? NMAX : 1> sHh;  // tridiagonal solve of the large buckets
  __shared__ DevParams sPrm;  // LDS copy: the SK helpers never take the address of the kernel arguments

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int rgrp = tid >> 6;
  if (tid == 0) sPrm = a.prm;
  const DevParams& P = sPrm;
  double* scr = a.scratch + (int64_t)blockIdx.x * a.scratch_per_wg;
  double* gH0 = scr;
  double* gS = scr + NMAX * NMAX;
  double* gG = scr + 2 * NMAX * NMAX;
  double* bXp = scr + 3 * NMAX * NMAX;
  double* bFp = bXp + NMAX;
  double* sDF = bFp + NMAX;           // per-workgroup history (displaced jobs)
  double* sU = sDF + kMaxHist * NMAX;
  double* sX = GM ? sU + kMaxHist * NMAX : lX;
  double* sA = GM ? sX + NMAX * LD : lA;
  double* sT = GM ? sA + NMAX * LD : lT;
  double* sD = GM ? sT + NMAX * LD : nullptr;  // fourth working matrix (large buckets only)

  const int n_jobs = a.n_jobs_dev ? *a.n_jobs_dev : a.n_jobs;
  // job queue: with a counter, each workgroup takes the next job when it is free
  // (the lists are ordered largest unit first), else a fixed stride over the list
  auto next_job = [&](int j) -> int {
    if (!a.job_counter) return j + gridDim.x;
    __syncthreads();  // every thread has read the previous job index
    if (tid == 0) sh.next_job = (int)atomicAdd(a.job_counter, 1u);
    __syncthreads();
    return sh.next_job;
  };
  for (int job = a.job_counter ? next_job(-1) : blockIdx.x; job < n_jobs; job = next_job(job)) {
    const int u = a.job_unit[job];
    if (a.unit_mask && !a.unit_mask[u]) {  // block-uniform skip (fallback launches)
      if (tid == 0) {
        if (a.job_status) a.job_status[job] = 0;
        if (a.job_iters) a.job_iters[job] = 0;
      }
      continue;
    }
    const int disp = a.job_disp ? a.job_disp[job] : -1;
    const int fcode = disp <= -2 ? -2 - disp : -1;  // field job: dir*2 + (field < 0)
    // sign and slot of a perturbed job of a central difference: the +h (+field)
    // job of slot (3 atom + dir) (dir) runs in pass 1, its -h partner in pass 2
    const int pm_sign = disp >= 0 ? (disp & 1) : (fcode >= 0 ? (fcode & 1) : -1);
    if (a.fd_pass && pm_sign >= 0 && pm_sign != (a.fd_pass == 2 ? 1 : 0)) continue;  // the other sign's pass
    const int a0 = a.unit_off[u];
    const int na = a.unit_off[u + 1] - a0;
    // slot of the job's charge response in fd_dq: 3 atom + dir (displaced), 3 n_a + dir (field)
    const int64_t fd_slot = disp >= 0 ? (disp >> 1) : 3LL * na + (fcode >> 1);
    const int d_atom = disp >= 0 ? (disp >> 1) / 3 : -1;
    const int d_dir = disp >= 0 ? (disp >> 1) % 3 : 0;
    const double d_step = disp >= 0 ? ((disp & 1) ? -a.fd_h : a.fd_h) : 0.0;
    // Broyden history: the unit's own store for undisplaced jobs (read-write),
    // a workgroup copy of it for displaced jobs (read-only use of the store)
    double* hst = a.hist ? a.hist + a.hist_off[u] : nullptr;  // [count, head, Gram H*H, dF H*NMAX, U H*NMAX]
    const bool own_hist = hst && disp == -1 && (a.flags & JF_STORE_HIST);
    // dF vectors in LDS (written through to the unit's store when it is owned), U
    // vectors in the store (owned) or in the workgroup copy
    double* bDF = lDF;
    double* gDF = own_hist ? hst + 2 + kMaxHist * kMaxHist : nullptr;
    double* bU = own_hist ? hst + 2 + kMaxHist * kMaxHist + kMaxHist * NMAX : sU;

    // ---- load atoms, clear the working matrices
    for (int t = tid; t < na; t += NT) {
      sSp[t] = a.species[a0 + t];
      for (int g = 0; g < 3; ++g) sPos[t * 3 + g] = a.pos[(int64_t)(a0 + t) * 3 + g];
      if (t == d_atom) sPos[t * 3 + d_dir] += d_step;
    }
    for (int e = tid; e < NMAX * LD; e += NT) {
      sX[e] = 0.0;
      sA[e] = 0.0;
      sT[e] = 0.0;
    }
    __syncthreads();
    if (tid == 0) {
      int o = 0;
      double nel = 0.0;
      bool bad = false;
      for (int t = 0; t < na; ++t) {
        sAtomOff[t] = o;
        o += sSp[t] == 0 ? 4 : 1;
        nel += P.q0[sSp[t]];
        for (int g = 0; g < 3; ++g) bad |= !isfinite(sPos[t * 3 + g]);
      }
      sAtomOff[na] = o;
      sh.n = o;
      sh.nocc = (int)(nel + 0.5) / 2;
      sh.na = na;
      sh.notpd = bad ? 2 : 0;  // 2 marks a non-finite position
      sh.bcount = 0;
      sh.bhead = 0;
      if (hst && (a.flags & JF_WARM_HIST)) {
        sh.bcount = (int)hst[0];
        sh.bhead = (int)hst[1];
      }
      sh.sweeps = 0;
      sh.jac_iters = 0;
      sh.hh_solves = 0;
      sh.hh_fails = 0;
      for (int g = 0; g < 3; ++g) sh.fld[g] = 0.0;
      if (fcode >= 0) sh.fld[fcode >> 1] = (fcode & 1) ? -a.fd_h : a.fd_h;
    }
    __syncthreads();
    const int n = sh.n, nocc = sh.nocc;
    for (int t = tid; t < na; t += NT) {
      for (int o = sAtomOff[t]; o < sAtomOff[t + 1]; ++o) sOrbAtom[o] = t;
      sQ0[t] = P.q0[sSp[t]];
      double dq0 = (a.flags & JF_WARM_DQ) ? a.ws_dq[a0 + t] : 0.0;
      if ((a.flags & JF_WARM_DQ) && a.n_extrap >= 2) {  // charges of earlier MD steps
        const double d1 = a.ws_dq_hist[a0 + t], d2 = a.ws_dq_hist[(int64_t)a.n_atoms + a0 + t];
        dq0 = a.n_extrap >= 3 ? 3.0 * dq0 - 3.0 * d1 + d2 : 2.0 * dq0 - d1;
      }
      if (a.fd_pass && pm_sign >= 0) {
        // charge response ddq of the + job of this slot: a -h job starts from the
        // +h charges of this pass reflected through the centre, dq_c - ddq; a +h
        // job from its response at the previous evaluation, dq_c + ddq (first
        // order in the change of the response between evaluations; zero before
        // the first).  Failed + jobs leave NaN: start from the centre.
        const double d = a.fd_dq[a.fd_dq_off[u] + fd_slot * na + t];
        if (isfinite(d)) dq0 += (pm_sign == 1) ? -d : d;
      }
      sDqIn[t] = dq0;
    }
    {
      const int m0 = sh.bcount;
      for (int e = tid; e < m0 * kMaxHist; e += NT) sBa[e] = hst[2 + e];
      for (int e = tid; e < m0 * NMAX; e += NT) {
        bDF[e] = hst[2 + kMaxHist * kMaxHist + e];
        if (!own_hist) bU[e] = hst[2 + kMaxHist * kMaxHist + kMaxHist * NMAX + e];
      }
    }

    // ---- H0, S (global scratch) and gamma
    for (int task = tid; task < na * na; task += NT) {
      const int A = task / na, B = task % na;
      if (B < A) continue;
      const int oA = sAtomOff[A], oB = sAtomOff[B];
      const int nA = sSp[A] == 0 ? 4 : 1, nB = sSp[B] == 0 ? 4 : 1;
      if (A == B) {
        for (int i = 0; i < nA; ++i)
          for (int j = 0; j < nA; ++j) {
            const double h = (i == j) ? P.onsite[sSp[A]][i == 0 ? 0 : 1] : 0.0;
            gH0[(oA + i) * NMAX + oA + j] = h;
            gS[(oA + i) * NMAX + oA + j] = (i == j) ? 1.0 : 0.0;
          }
        gG[A * NMAX + A] = P.U[sSp[A]];
      } else {
        double d[3], H[16], S[16];
        for (int g = 0; g < 3; ++g) d[g] = sPos[B * 3 + g] - sPos[A * 3 + g];
        sk_block(P, sSp[A], sSp[B], d, H, S);
        for (int i = 0; i < nA; ++i)
          for (int j = 0; j < nB; ++j) {
            gH0[(oA + i) * NMAX + oB + j] = H[i * 4 + j];
            gS[(oA + i) * NMAX + oB + j] = S[i * 4 + j];
            gH0[(oB + j) * NMAX + oA + i] = H[i * 4 + j];
            gS[(oB + j) * NMAX + oA + i] = S[i * 4 + j];
          }
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double g, dg;
        gamma_pair(P.U[sSp[A]], P.U[sSp[B]], r, g, dg);
        gG[A * NMAX + B] = g;
        gG[B * NMAX + A] = g;
      }
    }
    __syncthreads();

    // ---- S-orthonormal starting basis X.  Warm: M = C0^T S C0 of the stored
    // basis C0; when M is close to I, Newton-Schulz steps X <- X (3I - M)/2
    // (quadratic convergence to the symmetric orthonormalisation C0 M^{-1/2},
    // which keeps the column order and the near-eigenvector property);
    // otherwise, and for the cold start X = I, Cholesky M = R^T R and X = C0 R^{-1}.
    const bool warm = (a.flags & JF_WARM_C) != 0;
    bool use_chol = true;
    if (warm) {
      const double* wc = a.ws_C + a.ws_off[u];
      ew_global<NMAX, NT>(wc, gS, n, [&](int i, int j, double c, double sv) {
        sX[i * LD + j] = c;
        sA[i * LD + j] = sv;
      });
      __syncthreads();
      gemm<NMAX, NT, false>(sA, sX, sT, n);  // T = S C0
      __syncthreads();
      gemm<NMAX, NT, true>(sX, sT, sA, n);  // M = C0^T S C0
      __syncthreads();
      double e = 0.0;
      for (int i = rgrp; i < n; i += RG)
        for (int j = lane; j < n; j += 64) e = fmax(e, fabs(sA[i * LD + j] - (i == j ? 1.0 : 0.0)));
      e = block_max<NT>(e, sRed);
      if (e <= kNsStart) {  // false for a non-finite M
        use_chol = false;
        for (int k = 0; k < kNsMaxSteps && e > kNsTol; ++k) {
          for (int i = rgrp; i < n; i += RG)
            for (int j = lane; j < n; j += 64) sA[i * LD + j] = (i == j ? 1.5 : 0.0) - 0.5 * sA[i * LD + j];
          __syncthreads();
          gemm<NMAX, NT, false>(sX, sA, sT, n);  // X (3I - M) / 2
          __syncthreads();
          double* tmp = sX;
          sX = sT;
          sT = tmp;
          if (0.75 * e * e < kNsTol * 1e-2) break;  // the next M would be I to rounding
          ew_global<NMAX, NT>(gS, gS, n, [&](int i, int j, double sv, double) { sA[i * LD + j] = sv; });
          __syncthreads();
          gemm<NMAX, NT, false>(sA, sX, sT, n);  // S X
          __syncthreads();
          gemm<NMAX, NT, true>(sX, sT, sA, n);  // M = X^T S X
          __syncthreads();
          e = 0.0;
          for (int i = rgrp; i < n; i += RG)
            for (int j = lane; j < n; j += 64) e = fmax(e, fabs(sA[i * LD + j] - (i == j ? 1.0 : 0.0)));
          e = block_max<NT>(e, sRed);
        }
      }
    } else {
      ew_global<NMAX, NT>(gS, gS, n, [&](int i, int j, double sv, double) {
        sX[i * LD + j] = (i == j) ? 1.0 : 0.0;
        sA[i * LD + j] = sv;
      });
      __syncthreads();
    }
    // right-looking Cholesky of M fused with the solve X R = C0
    for (int k = 0; use_chol && k < n; ++k) {
      const double dkk = sA[k * LD + k];
      const double rkk = dkk > 0.0 ? sqrt(dkk) : 1.0;
      if (tid == 0 && !(dkk > 0.0)) sh.notpd |= 1;
      const double irkk = 1.0 / rkk;
      for (int t = tid; t < 2 * n; t += NT) {
        if (t < n) {
          if (t > k) sA[k * LD + t] *= irkk;  // row k of R
        } else {
          sX[(t - n) * LD + k] *= irkk;      // column k of X
        }
      }
      __syncthreads();
      for (int i = k + 1 + rgrp; i < n; i += RG)
        for (int j = lane; j < n; j += 64)
          if (j >= i) sA[i * LD + j] -= sA[k * LD + i] * sA[k * LD + j];
      for (int i = rgrp; i < n; i += RG)
        for (int j = lane; j < n; j += 64)
          if (j > k) sX[i * LD + j] -= sX[i * LD + k] * sA[k * LD + j];
      __syncthreads();
    }
    int status = 0;
    if (sh.notpd) status |= (sh.notpd & 2) ? CAVDFTB_ST_NAN : CAVDFTB_ST_NOT_PD;
    bool ordered = warm;  // stored bases keep the occupied orbitals first

    int it = 0;
    // a unit that failed its last undisplaced SCC (charge sloshing that does not
    // settle) gets a shorter stagnation window: it keeps iterating while it finds
    // new smallest residuals, but does not hold its launch for kStagnation idle
    // iterations every evaluation
    const int stag_window = (a.unit_fail && a.unit_fail[u]) ? kStagnationFailed : kStagnation;
    double res_prev = INFINITY;  // no charge residual known before the first iteration
    double res_best = INFINITY;  // smallest residual so far and its iteration (stagnation stop)
    int it_best = 0;
    if (status == 0) {
      for (it = 1; it <= a.max_iter; ++it) {
        // V = gamma Dq_in + field . R
        site_potential<NT>(gG, NMAX, sDqIn, sPos, sh.fld, na, sV);
        __syncthreads();
        // H = H0 + 1/2 S o (V_a + V_b) into sA
        ew_global<NMAX, NT>(gH0, gS, n, [&](int i, int j, double h, double sv) {
          sA[i * LD + j] = h + 0.5 * sv * (sV[sOrbAtom[i]] + sV[sOrbAtom[j]]);
        });
        __syncthreads();

        gemm<NMAX, NT, false>(sA, sX, sT, n);  // T = H X
        __syncthreads();
        gemm<NMAX, NT, true>(sX, sT, sA, n);  // A = X^T H X
        __syncthreads();
        // Symmetrise A.  With the occupied columns first the same pass takes the
        // block statistics of the occupied-virtual step below and its start
        // K0 = A_ov / (d_v - d_o), into a slot of sT (slots: columns [0, nv) and
        // [nv, 2 nv) of sT; the last Sylvester sweep writes the first).  Each
        // unordered pair is read and written by one thread; the diagonal is only read.
        const int nv = n - nocc;
        const bool ov_try = ordered && nocc > 0 && nv > 0 && 2 * nv <= n &&  // K ping-pong needs 2 n_v <= n
                            a.eig_mode != CAVDFTB_EIG_FULL;
        const int s0 = (kSylvester & 1) ? nv : 0;
        double st[4] = {0.0, 0.0, -INFINITY, -INFINITY};  // off-block, ov, max d_o, -min d_v
        {
          // rows in groups of SR per thread: all loads of a group (both triangles and
          // the diagonals) are issued before its stores, so a group pays one LDS
          // round trip; every index is clamped into the block, clamped work is skipped
          constexpr int SR = 4;
          for (int j0 = 0; j0 < n; j0 += 64) {
            const int j = j0 + lane, jc = j < n ? j : n - 1;
            const double djj = sA[jc * LD + jc];
            for (int i0 = rgrp; i0 < n; i0 += SR * RG) {
              double aij[SR], aji[SR], dii[SR];
#pragma unroll
              for (int g = 0; g < SR; ++g) {
                const int i = min(i0 + g * RG, n - 1);
                aij[g] = sA[i * LD + jc];
                aji[g] = sA[jc * LD + i];
                dii[g] = sA[i * LD + i];
              }
#pragma unroll
              for (int g = 0; g < SR; ++g) {
                const int i = i0 + g * RG;
                if (i >= n || j >= n) continue;
                if (j > i) {
                  const double v = 0.5 * (aij[g] + aji[g]);
                  sA[i * LD + j] = v;
                  sA[j * LD + i] = v;
                  if (i < nocc && j >= nocc) {
                    st[1] = fmax(st[1], fabs(v));
                    if (ov_try) sT[i * LD + s0 + j - nocc] = v / (djj - dii[g]);
                  } else {
                    st[0] = fmax(st[0], fabs(v));
                  }
                } else if (j == i) {
                  if (i < nocc)
                    st[2] = fmax(st[2], dii[g]);
                  else
                    st[3] = fmax(st[3], -dii[g]);
                }
              }
            }
          }
        }
        if (ov_try)
          block_max_n<NT, 4>(st, sRed);  // also orders the writes of A and K0
        else
          __syncthreads();

        // ---- occupied-virtual step.  With the occupied columns first, rotate X by
        // the exactly orthogonal Cayley transform U = (I + B)(I - B)^{-1},
        // B = [[0, L], [-L^T, 0]], L = K / 2, where K (n_occ x n_v) solves the
        // first-order decoupling condition K A_vv - A_oo K = A_ov (Jacobi sweeps
        // on the Sylvester equation from K = A_ov / (d_v - d_o)).  Then
        //   X_occ <- X_occ - Z K^T - 2 X_v Y^T,  X_v <- X_v + 2 Z + 2 X_v (G - I),
        // G = (I + L^T L)^{-1} (Neumann series), Y = L G, Z = X_occ Y.
        bool use_ov = false;
        double kmax = 0.0;
        if (ov_try) {
          const double gap = -st[3] - st[2];
          use_ov = gap > kOvGap && st[1] < kOvAngle * gap && st[0] < kOvOff * gap;
          double lf2 = 0.0;  // ||L||_F^2
          if (use_ov) {
            // Jacobi sweeps on K A_vv - A_oo K = A_ov:  K <- K + (A_ov - K A_vv + A_oo K) / D
            for (int sw = 0; sw < kSylvester; ++sw) {
              const int src = ((kSylvester - sw) & 1) ? nv : 0, dst = nv - src;
              double km = 0.0, k2 = 0.0;
              gemm_e<NMAX, NT, false, false>(
                  sA, sT + src, nocc, sT + src, sA + nocc * LD + nocc, nv, -1.0, nocc, nv,
                  [&](int i, int c, double r) {
                    const double kn = sT[i * LD + src + c] +
                                      (sA[i * LD + nocc + c] + r) / (sA[(nocc + c) * LD + nocc + c] - sA[i * LD + i]);
                    sT[i * LD + dst + c] = kn;
                    km = fmax(km, fabs(kn));
                    k2 = fma(kn, kn, k2);
                  });
              if (sw == kSylvester - 1) {
                double v2[2] = {km, k2};
                block_max_sum(v2, sRed, NT / 64);  // orders the writes of K as well
                kmax = v2[0];
                lf2 = 0.25 * v2[1];
                if (!(kmax < INFINITY)) lf2 = INFINITY;
              } else {
                __syncthreads();
              }
            }
            use_ov = lf2 <= kOvNorm;
          }
          if (use_ov) {
            // M = L^T L -> sA rows [0, nv); G_1 = I - M -> sT rows [nocc, n), columns [0, nv)
            gemm_e<NMAX, NT, true, false>(sT, sT, nocc, sT, sT, 0, 0.0, nv, nv, [&](int c, int b, double v) {
              const double mm = 0.25 * v;
              sA[c * LD + b] = mm;
              sT[(nocc + c) * LD + b] = (c == b ? 1.0 : 0.0) - mm;
            });
            __syncthreads();
            // Horner steps G_j = I - M G_{j-1} (column blocks 0 / nv of sT rows [nocc, n))
            // until the remainder ||M||^{j+1} <= ||L||_F^{2(j+1)} is below 1e-17
            int gsrc = 0;
            for (double bound = lf2 * lf2; bound > 1.0e-17; bound *= lf2) {
              const int gdst = nv - gsrc;
              gemm_e<NMAX, NT, false, false>(sA, sT + nocc * LD + gsrc, nv, sA, sA, 0, 0.0, nv, nv,
                                             [&](int c, int b, double v) {
                                               sT[(nocc + c) * LD + gdst + b] = (c == b ? 1.0 : 0.0) - v;
                                             });
              __syncthreads();
              gsrc = gdst;
            }
            const double* Gm = sT + nocc * LD + gsrc;
            // Y2 = K G -> sT rows [0, nocc), columns [nv, 2 nv)
            gemm_e<NMAX, NT, false, false>(sT, Gm, nv, sT, sT, 0, 0.0, nocc, nv,
                                           [&](int i, int c, double v) { sT[i * LD + nv + c] = v; });
            __syncthreads();
            // Z = X_occ Y2 / 2 -> sA columns [0, nv); copy of X_v -> sA columns [nv, 2 nv)
            gemm_e<NMAX, NT, false, false>(sX, sT + nv, nocc, sX, sX, 0, 0.0, n, nv,
                                           [&](int r, int c, double v) { sA[r * LD + c] = 0.5 * v; });
            for (int r = rgrp; r < n; r += RG)
              for (int c = lane; c < nv; c += 64) sA[r * LD + nv + c] = sX[r * LD + nocc + c];
            __syncthreads();
            // X_occ -= [Z | X_v] [K | Y2]^T ;  X_v <- 2 X_v G + 2 Z - X_v
            gemm_e<NMAX, NT, false, true>(sA, sT, 2 * nv, sA, sA, 0, 0.0, n, nocc,
                                          [&](int r, int c, double v) { sX[r * LD + c] -= v; });
            gemm_e<NMAX, NT, false, false>(sA + nv, Gm, nv, sA, sA, 0, 0.0, n, nv, [&](int r, int c, double v) {
              sX[r * LD + nocc + c] = 2.0 * v + 2.0 * sA[r * LD + c] - sA[r * LD + nv + c];
            });
            __syncthreads();
            if (tid == 0) {
              sh.homo = st[2];
              sh.lumo = -st[3];
            }
          }
        }

        // ---- cyclic parallel Jacobi on A, rotations accumulated into X; then
        // the columns of X are sorted by eigenvalue (occupied first)
        if (!use_ov) {
        kmax = 0.0;
        if (tid == 0) sh.jac_iters += 1;
        bool solved = false;
        if constexpr (GM) {
          if (a.eig_mode != CAVDFTB_EIG_JACOBI) {
            double* cbuf = nullptr;
            solved = eig_householder<NMAX, NT>(sA, sX, sT, sD, gS, n, sQorb, &sRc[0][0], &sRs[0][0], &sRt[0][0],
                                               &sRp[0][0], sFbuf, sHh, sRed, sEig, &cbuf);
            if (solved) {
              double* tmp = sX;
              if (cbuf == sA) {
                sX = sA;
                sA = tmp;
              } else {
                sX = sT;
                sT = tmp;
              }
              if (tid == 0) {
                sh.hh_solves += 1;
                sh.homo = sEig[nocc - 1];
                sh.lumo = nocc < n ? sEig[nocc] : sEig[n - 1];
              }
              __syncthreads();
            } else {
              // discarded: A = X^T H X again for the Jacobi solve below (X is intact)
              if (tid == 0) sh.hh_fails += 1;
              ew_global<NMAX, NT>(gH0, gS, n, [&](int i, int j, double h, double sv) {
                sA[i * LD + j] = h + 0.5 * sv * (sV[sOrbAtom[i]] + sV[sOrbAtom[j]]);
              });
              __syncthreads();
              gemm<NMAX, NT, false>(sA, sX, sT, n);
              __syncthreads();
              gemm<NMAX, NT, true>(sX, sT, sA, n);
              __syncthreads();
              for (int i = rgrp; i < n; i += RG)
                for (int j = lane; j < n; j += 64)
                  if (j > i) {
                    const double v = 0.5 * (sA[i * LD + j] + sA[j * LD + i]);
                    sA[i * LD + j] = v;
                    sA[j * LD + i] = v;
                  }
              __syncthreads();
            }
          }
        }
        if (!solved) {
        const int half = n / 2;
        double thr = kJacobiThr;
        for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
          double off = 0.0;
          for (int i = rgrp; i < n; i += RG)
            for (int j = lane; j < n; j += 64)
              if (j > i) off = fmax(off, fabs(sA[i * LD + j]));
          off = block_max<NT>(off, sRed);
          // target: a fraction of the previous charge residual, and never above
          // a fraction of the coupling this iteration starts from
          if (sweep == 0) thr = fmax(kJacobiThr, a.jac_factor * fmin(res_prev, off));
          if (off < thr) break;
          if (tid == 0) sh.sweeps += 1;
          // round r: rotations of round r (wave 0) overlap the X update of
          // round r-1 (other waves); then the A update of round r.
          for (int r = 0; r < n; ++r) {
            const int b = r & 1;
            for (int kr = tid; r < n - 1 && kr < half; kr += NT) {
              int p = rr_index(kr, r, n), q = rr_index(n - 1 - kr, r, n);
              if (p > q) {
                const int tmp = p;
                p = q;
                q = tmp;
              }
              const double app = sA[p * LD + p], aqq = sA[q * LD + q], apq = sA[p * LD + q];
              double c = 1.0, sn = 0.0, t = 0.0;
              if (fabs(apq) > 1.0e-300) {
                const double d = aqq - app, h2 = 2.0 * apq;
                const double rr = sqrt(fma(d, d, h2 * h2));
                t = (d >= 0.0 ? h2 : -h2) / (fabs(d) + rr);
                c = rsqrt(fma(t, t, 1.0));
                sn = t * c;
              }
              sRp[b][kr] = p;
              sRq[b][kr] = q;
              sRc[b][kr] = c;
              sRs[b][kr] = sn;
              sRt[b][kr] = t;
            }
            if (RG > 1 && r > 0 && rgrp > 0) {
              for (int k = rgrp - 1; k < half; k += RG - 1) {
                const int p = sRp[b ^ 1][k], q = sRq[b ^ 1][k];
                const double c = sRc[b ^ 1][k], sn = sRs[b ^ 1][k];
                for (int i = lane; i < n; i += 64) {
                  const double xp = sX[i * LD + p], xq = sX[i * LD + q];
                  sX[i * LD + p] = c * xp - sn * xq;
                  sX[i * LD + q] = sn * xp + c * xq;
                }
              }
            }
            __syncthreads();
            if (r == n - 1) break;
            for (int l = tid & 31; l < half; l += 32) {
              {
                const int pl = sRp[b][l], ql = sRq[b][l];
                const double cl = sRc[b][l], sl = sRs[b][l];
                for (int k = tid >> 5; k < half; k += KSTEP_A) {
                  const int p = sRp[b][k], q = sRq[b][k];
                  if (k == l) {
                    const double apq = sA[p * LD + q], t = sRt[b][k];
                    sA[p * LD + p] -= t * apq;
                    sA[q * LD + q] += t * apq;
                    if (t != 0.0) {
                      sA[p * LD + q] = 0.0;
                      sA[q * LD + p] = 0.0;
                    }
                  } else {
                    const double ck = sRc[b][k], sk = sRs[b][k];
                    const double b00 = sA[p * LD + pl], b01 = sA[p * LD + ql];
                    const double b10 = sA[q * LD + pl], b11 = sA[q * LD + ql];
                    const double r00 = ck * b00 - sk * b10, r01 = ck * b01 - sk * b11;
                    const double r10 = sk * b00 + ck * b10, r11 = sk * b01 + ck * b11;
                    sA[p * LD + pl] = cl * r00 - sl * r01;
                    sA[p * LD + ql] = sl * r00 + cl * r01;
                    sA[q * LD + pl] = cl * r10 - sl * r11;
                    sA[q * LD + ql] = sl * r10 + cl * r11;
                  }
                }
              }
            }
            if (RG == 1) {  // single-wave workgroups: X update in this phase
              for (int k = 0; k < half; ++k) {
                const int p = sRp[b][k], q = sRq[b][k];
                const double c = sRc[b][k], sn = sRs[b][k];
                for (int i = lane; i < n; i += 64) {
                  const double xp = sX[i * LD + p], xq = sX[i * LD + q];
                  sX[i * LD + p] = c * xp - sn * xq;
                  sX[i * LD + q] = sn * xp + c * xq;
                }
              }
            }
            __syncthreads();
          }
        }

        for (int i = tid; i < n; i += NT) sEig[i] = sA[i * LD + i];
        __syncthreads();
        for (int i = tid; i < n; i += NT) {
          const double li = sEig[i];
          int rank = 0;
          for (int j = 0; j < n; ++j) {
            const double lj = sEig[j];
            rank += (lj < li || (lj == li && j < i)) ? 1 : 0;
          }
          sRank[i] = rank;
          sQorb[rank] = li;
          if (rank == nocc - 1) sh.homo = li;
          if (rank == nocc) sh.lumo = li;
        }
        __syncthreads();
        for (int r = rgrp; r < n; r += RG)
          for (int c = lane; c < n; c += 64) sT[r * LD + sRank[c]] = sX[r * LD + c];
        for (int i = tid; i < n; i += NT) sEig[i] = sQorb[i];
        __syncthreads();
        double* tmp = sX;
        sX = sT;
        sT = tmp;
        }  // cyclic Jacobi
        ordered = true;
        }  // full diagonalisation

        // ---- aufbau: the first n_occ columns of X are the occupied orbitals
        // ---- P = 2 C_occ C_occ^T into sT; Mulliken populations (P S)_ii = sum_j P_ji S_ji
        // (P, S symmetric) as RG partial sums over j = rgrp (mod RG) in sA rows [0, RG)
        gemm_g<NMAX, NT, false, true>(sX, sX, sT, n, n, nocc, 2.0);
        __syncthreads();
        for (int i = lane; i < n; i += 64)
          sA[rgrp * LD + i] = dotp(sT + rgrp * LD + i, RG * LD, gS + rgrp * NMAX + i, RG * NMAX, (n - rgrp + RG - 1) / RG);
        __syncthreads();
        double res = 0.0;
        for (int t = tid; t < na; t += NT) {
          double q = 0.0;
          for (int o = sAtomOff[t]; o < sAtomOff[t + 1]; ++o)
#pragma unroll
            for (int g = 0; g < RG; ++g) q += sA[g * LD + o];
          sDqOut[t] = q - sQ0[t];
          const double dlt = fabs(sDqOut[t] - sDqIn[t]);
          res = (dlt == dlt) ? fmax(res, dlt) : INFINITY;
        }
        res = block_max<NT>(res, sRed);
        if (res < a.tol && kmax < 10.0 * a.tol) break;  // block-uniform
        if (!(res < INFINITY)) {
          status |= CAVDFTB_ST_NAN;
          break;
        }
        if (res < res_best) {
          res_best = res;
          it_best = it;
        } else if (it - it_best >= stag_window) {  // no new best residual for stag_window iterations
          status |= CAVDFTB_ST_NOT_CONVERGED;
          break;
        }
        res_prev = res;

        // ---- Johnson's modified Broyden mixing (Gram matrix of stored dF kept in LDS)
        int slot_new = -1;
        if (it > 1) {
          double part = 0.0;
          for (int t = tid; t < na; t += NT) {
            const double df = (sDqOut[t] - sDqIn[t]) - bFp[t];
            part += df * df;
          }
          const double nrm = sqrt(block_sum<NT>(part, sRed));
          if (nrm > 1.0e-300) slot_new = sh.bcount < kMaxHist ? sh.bcount : sh.bhead;
          const double inrm = slot_new >= 0 ? 1.0 / nrm : 0.0;
          // new history pair; each thread then overwrites only the entries it read
          for (int t = tid; t < na; t += NT) {
            const double f = sDqOut[t] - sDqIn[t];
            if (slot_new >= 0) {
              const double df = (f - bFp[t]) * inrm;
              bDF[slot_new * NMAX + t] = df;
              if (gDF) gDF[slot_new * NMAX + t] = df;
              bU[slot_new * NMAX + t] = a.alpha * df + (sDqIn[t] - bXp[t]) * inrm;
            }
            bXp[t] = sDqIn[t];
            bFp[t] = f;
            sQorb[t] = f;  // LDS copy of the residual for the dot products below
          }
          __syncthreads();
          if (tid == 0 && slot_new >= 0) {
            if (sh.bcount < kMaxHist)
              sh.bcount += 1;
            else
              sh.bhead = (sh.bhead + 1) % kMaxHist;
          }
        } else {
          for (int t = tid; t < na; t += NT) {
            bXp[t] = sDqIn[t];
            bFp[t] = sDqOut[t] - sDqIn[t];
            sQorb[t] = bFp[t];
          }
        }
        __syncthreads();
        const int m = sh.bcount;
        if (m > 0) {
          // Gram row of the new slot and c = dF . f: lane k of the first wave takes dot
          // product k whole (no cross-lane reduction); the solve below runs in the same
          // wave, ordered by a wave-level barrier only
          if (tid < 64) {
            const int k = tid;
            if (k < 2 * m && (k >= m || slot_new >= 0)) {
              const int kk = k < m ? k : k - m;
              const double* y = k < m ? bDF + slot_new * NMAX : sQorb;
              const double sd = dotp(bDF + kk * NMAX, 1, y, 1, na);
              if (k < m) {
                sBa[slot_new * kMaxHist + kk] = sd;
                sBa[kk * kMaxHist + slot_new] = sd;
              } else {
                sBc[kk] = sd;
              }
            }
            wave_sync();
          }
          // (w0^2 I + a) g = c by Gauss-Jordan in the first wave: lane l holds row l of the
          // system padded to kMaxHist x kMaxHist with the identity (right-hand side in the
          // last register); pivot rows are broadcast with readlane, no LDS traffic
          if (tid < 64) {
            int lt = tid;
            asm volatile("" : "+v"(lt));  // keep the per-lane compares below inside this block
            const double* ba = sBa + (lt < kMaxHist ? lt : 0) * kMaxHist;
            const bool live = lt < m;
            double row[kMaxHist + 1];
#pragma unroll
            for (int j = 0; j < kMaxHist; ++j) {
              const double v = ba[j];
              row[j] = (live && j < m) ? v + (lt == j ? a.w0 * a.w0 : 0.0) : (lt == j ? 1.0 : 0.0);
            }
            row[kMaxHist] = live ? sBc[lt] : 0.0;
            // pivots beyond m are identity rows: nothing to eliminate.  Columns left of the
            // pivot are already zero in the pivot row and are skipped.
#pragma unroll
            for (int k = 0; k < kMaxHist; ++k) {
              if (k < m) {
                // broadcast outside any lane-dependent branch: lane k must hold row[k] when read
                const double pk = lane_bcast(row[k], k);
                const double f = lt == k ? 0.0 : row[k] / pk;
#pragma unroll
                for (int j = k + 1; j <= kMaxHist; ++j) row[j] = fma(-f, lane_bcast(row[j], k), row[j]);
              }
            }
            double rd = 1.0;
#pragma unroll
            for (int j = 0; j < kMaxHist; ++j) rd = j == lt ? row[j] : rd;
            if (live) sBg[lt] = row[kMaxHist] / rd;
          }
          __syncthreads();
        }
        for (int t = tid; t < na; t += NT) {
          double x = sDqIn[t] + a.alpha * bFp[t];
          constexpr int UG = kMaxHist / 2;  // history loads issued in two groups, unconditionally
#pragma unroll
          for (int k0 = 0; k0 < kMaxHist; k0 += UG) {
            double uv[UG];
#pragma unroll
            for (int q = 0; q < UG; ++q) uv[q] = bU[(k0 + q) * NMAX + t];
#pragma unroll
            for (int q = 0; q < UG; ++q)
              if (k0 + q < m) x = fma(-sBg[k0 + q], uv[q], x);
          }
          sDqIn[t] = x;
        }
        __syncthreads();
      }
      if (it > a.max_iter) {
        status |= CAVDFTB_ST_NOT_CONVERGED;
        it = a.max_iter;
      }
      if (nocc < n && sh.lumo - sh.homo < kGapMin) status |= CAVDFTB_ST_DEGENERATE;
    }

    // ---- outputs
    if (status == 0 && (a.flags & JF_STORE)) {
      double* wc = a.ws_C + a.ws_off[u];
      for (int i = rgrp; i < n; i += RG)
        for (int j = lane; j < n; j += 64) wc[i * NMAX + j] = sX[i * LD + j];
      for (int t = tid; t < na; t += NT) {
        if (a.ws_dq_hist) {  // shift the charge history of the unit (MD steps)
          a.ws_dq_hist[(int64_t)a.n_atoms + a0 + t] = a.ws_dq_hist[a0 + t];
          a.ws_dq_hist[a0 + t] = a.ws_dq[a0 + t];
        }
        a.ws_dq[a0 + t] = sDqOut[t];
      }
    }
    if (own_hist && (a.flags & JF_STORE_HIST)) {
      const int m0 = status == 0 ? sh.bcount : 0;
      for (int e = tid; e < m0 * kMaxHist; e += NT) hst[2 + e] = sBa[e];
      if (tid == 0) {
        hst[0] = (double)m0;
        hst[1] = (double)(status == 0 ? sh.bhead : 0);
      }
    }
    if (status & (CAVDFTB_ST_NOT_PD | CAVDFTB_ST_NAN)) {
      for (int t = tid; t < na; t += NT) sDqOut[t] = 0.0;
    }
    __syncthreads();
    // dipole mu = sum_A Q_A R_A with Q = -Dq; zero for a unit without a valid
    // density (its positions may be non-finite), so it drops out of the cavity sums
    const bool dead = (status & (CAVDFTB_ST_NOT_PD | CAVDFTB_ST_NAN)) != 0;
    if (tid < 3) {
      double m = 0.0;
      for (int t = 0; !dead && t < na; ++t) m -= sDqOut[t] * sPos[t * 3 + tid];
      if (disp != -1) {
        if (a.mu_job) a.mu_job[(int64_t)job * 3 + tid] = m;
      } else if (a.dipole) {
        a.dipole[(int64_t)u * 3 + tid] = m;
      }
    }
    if (disp == -1) {
      for (int t = tid; t < na; t += NT)
        if (a.charges) a.charges[a0 + t] = -sDqOut[t];
    }
    if (a.fd_pass == 1 && pm_sign == 0)
      for (int t = tid; t < na; t += NT) {
        const double dqc = (a.flags & JF_WARM_DQ) ? a.ws_dq[a0 + t] : 0.0;
        a.fd_dq[a.fd_dq_off[u] + fd_slot * na + t] = status == 0 ? sDqOut[t] - dqc : NAN;
      }
    if ((a.flags & JF_FORCES) && disp < 0) {  // undisplaced and field jobs
      // W = 2 C_occ diag(eps_occ) C_occ^T = 1/2 P H P with H of the last iteration
      // (sV still holds its V; X_occ spans the occupied eigenspace, so no
      // eigenvalues are needed).  X is free after the basis store above.
      ew_global<NMAX, NT>(gH0, gS, n, [&](int i, int j, double h, double sv) {
        sA[i * LD + j] = 0.5 * (h + 0.5 * sv * (sV[sOrbAtom[i]] + sV[sOrbAtom[j]]));
      });
      __syncthreads();
      gemm<NMAX, NT, false>(sA, sT, sX, n);  // (H / 2) P
      __syncthreads();
      gemm<NMAX, NT, false>(sT, sX, sA, n);  // W = P (H / 2) P
      // V from the output charges (with the field potential)
      site_potential<NT>(gG, NMAX, sDqOut, sPos, sh.fld, na, sV);
      __syncthreads();
      double ebp = 0.0;
      ew_global<NMAX, NT>(gH0, gH0, n, [&](int i, int j, double h, double) { ebp += sT[i * LD + j] * h; });
      // 1/2 Dq gamma Dq + Dq (field . R): V already holds the field potential once
      double ecp = 0.0;
      for (int t = tid; t < na; t += NT) {
        const double vx = sh.fld[0] * sPos[t * 3] + sh.fld[1] * sPos[t * 3 + 1] + sh.fld[2] * sPos[t * 3 + 2];
        ecp += 0.5 * sDqOut[t] * (sV[t] + vx);
      }
      // pair forces: task (A, part) sums g(A,B) over its B's; the NT / na
      // parts of an atom keep every thread busy (na <= NT)
      const int split = na > 0 && na < NT ? NT / na : 1;
      double erp = 0.0;
      double fa[3] = {0.0, 0.0, 0.0};
      const int A = tid / split, part = tid - A * split;
      if (A < na && (status & (CAVDFTB_ST_NOT_PD | CAVDFTB_ST_NAN)) == 0) {
        const int oA = sAtomOff[A];
        for (int B = part; B < na; B += split) {
          if (B == A) continue;
          const int oB = sAtomOff[B];
          double d[3];
          for (int g = 0; g < 3; ++g) d[g] = sPos[B * 3 + g] - sPos[A * 3 + g];
          const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
          pair_band_grad(P, sSp[A], sSp[B], d, sT, sA, LD, oA, oB, sV[A] + sV[B], fa);
          double gm, dgm;
          gamma_pair(P.U[sSp[A]], P.U[sSp[B]], r, gm, dgm);
          const int pt = sSp[A] + sSp[B];
          const double vrep = P.rep_a[pt] * exp(-P.rep_alpha[pt] * r);
          erp += 0.5 * vrep;
          const double radial_g = sDqOut[A] * sDqOut[B] * dgm - P.rep_alpha[pt] * vrep;
          for (int g = 0; g < 3; ++g) fa[g] += radial_g * d[g] / r;
        }
        if (part == 0)  // direct force of the field on the atom's excess charge
          for (int g = 0; g < 3; ++g) fa[g] -= sDqOut[A] * sh.fld[g];
      }
      __syncthreads();  // sF may alias the X buffer
      double* sF = F_IN_X ? sX : sFbuf;
      for (int g = 0; g < 3; ++g) sF[tid * 3 + g] = fa[g];
      const double etot = block_sum<NT>(ebp + ecp + erp, sRed);  // contains the barrier for sF
      double* fo = disp == -1 ? a.forces : (a.f_job ? a.f_job + (int64_t)fcode * a.n_atoms * 3 : nullptr);
      for (int t = tid; t < na; t += NT) {
        for (int g = 0; g < 3; ++g) {
          double f = 0.0;
          for (int pp = 0; pp < split; ++pp) f += sF[(t * split + pp) * 3 + g];
          if (fo) fo[(int64_t)(a0 + t) * 3 + g] = f;
        }
      }
      if (tid == 0 && a.energy && disp == -1) a.energy[u] = dead ? 0.0 : etot;
    }
    if (tid == 0) {
      if (disp == -1 && a.status) a.status[u] = status;
      if (disp == -1 && a.unit_fail) a.unit_fail[u] = (status & CAVDFTB_ST_NOT_CONVERGED) ? 1 : 0;
      if (fcode >= 0 && a.f_status) a.f_status[(int64_t)u * 6 + fcode] = status;
      if (a.job_status) a.job_status[job] = status;
      if (a.job_iters) a.job_iters[job] = it;
      if (a.counters) {
        const unsigned long long nn = n, no = nocc;
        const unsigned long long per_it = 10ull * nn * nn * nn + 2ull * nn * nn * no;
        const unsigned long long per_geo = nn * nn * nn / 3ull + 2ull * nn * nn * no;
        atomicAdd(&a.counters[0], 1ull);
        atomicAdd(&a.counters[1], (unsigned long long)it);
        atomicAdd(&a.counters[2], per_it * (unsigned long long)it + per_geo);
        atomicAdd(&a.counters[3], (unsigned long long)sh.sweeps);
        atomicAdd(&a.counters[5], (unsigned long long)sh.jac_iters);
        if (sh.hh_solves) atomicAdd(&a.counters[6], (unsigned long long)sh.hh_solves);
        if (sh.hh_fails) atomicAdd(&a.counters[7], (unsigned long long)sh.hh_fails);
      }
    }
    __syncthreads();
  }
}

}  // namespace

int64_t scc_scratch_per_wg(int nmax) {
  return 3LL * nmax * nmax + (2LL + 2LL * kMaxHist) * nmax + (nmax > 64 ? 4LL * nmax * (nmax + 1) : 0);
}

__global__ void reset_counter_kernel(unsigned int* c) {
  if (threadIdx.x == 0) c[0] = 0u;
}

template <int NMAX, int NT>
static hipError_t launch_t(int n_wg, const SccArgs& args, hipStream_t stream) {
  if (args.job_counter) {  // a kernel, not a memset: the step may be captured in a graph
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, args.job_counter);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((scc_kernel<NMAX, NT>), dim3(n_wg), dim3(NT), 0, stream, args);
  return hipGetLastError();
}

template <int NMAX, int NT>
static int occ_t() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, scc_kernel<NMAX, NT>, NT, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

hipError_t launch_scc(int nmax, int n_wg, const SccArgs& args, hipStream_t stream) {
  switch (nmax) {
    case 8: return launch_t<8, 64>(n_wg, args, stream);
    case 16: return launch_t<16, 64>(n_wg, args, stream);
    case 32: return launch_t<32, 256>(n_wg, args, stream);
    case 48: return launch_t<48, 256>(n_wg, args, stream);
    case 64: return launch_t<64, 256>(n_wg, args, stream);
    case 96: return launch_t<96, 256>(n_wg, args, stream);
    case 128: return launch_t<128, 256>(n_wg, args, stream);
    case 192: return launch_t<192, 256>(n_wg, args, stream);
    default: return hipErrorInvalidValue;
  }
}

int scc_blocks_per_cu(int nmax) {
  switch (nmax) {
    case 8: return occ_t<8, 64>();
    case 16: return occ_t<16, 64>();
    case 32: return occ_t<32, 256>();
    case 48: return occ_t<48, 256>();
    case 64: return occ_t<64, 256>();
    case 96: return occ_t<96, 256>();
    case 128: return occ_t<128, 256>();
    case 192: return occ_t<192, 256>();
    default: return 1;
  }
}

}  // namespace cavdftb
