// Learned Born-charge surrogate kernels (gfx950).
//
// The paper obtains the Born charges by finite differences and names them the
// bottleneck of the method (Results; Conclusion).  These kernels evaluate and
// train the replacement: radial and frame-resolved direction descriptors and
// atom-local frames, a per-species 80 -> 128 -> 128 -> 9 SiLU network ensemble with BF16 operands and FP32
// accumulation (the products of the forward and backward passes on the matrix
// cores), the ensemble mean/spread with the acoustic-sum projection, and
// the Adam update of the FP32 master weights.  Every reduction has a fixed
// order (per-tile partial sums reduced in tile order), so results do not depend
// on scheduling.
#include <math.h>

#include <algorithm>

#include "internal.h"

namespace cavdftb {
namespace {

constexpr int NIN = CAVDFTB_SG_N_IN, NHID = CAVDFTB_SG_N_HID, NOUT = CAVDFTB_SG_N_OUT;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NIN * NHID, OFF_W2 = OFF_B1 + NHID, OFF_B2 = OFF_W2 + NHID * NHID,
              OFF_W3 = OFF_B2 + NHID, OFF_B3 = OFF_W3 + NHID * NOUT, NPAR = OFF_B3 + NOUT;
static_assert(NPAR == CAVDFTB_SG_N_PARAM, "parameter layout");
static_assert(NIN == 80, "descriptors: per neighbour species 16 radial Gaussians and 8 x 3 direction moments");
constexpr int TILE = 64;  // atoms per workgroup of the backward pass
constexpr int NT = 256;
// forward pass: 512-thread workgroups on 128-atom tiles (16 atoms per wave),
// one per CU (124 KB of LDS), persistent over the tiles
constexpr int FNT = 512, FTILE = 128;
constexpr int kForwardGrid = 256;

constexpr double kAng = 1.8897261246;

// float -> bfloat16 -> float, round to nearest even (finite inputs)
__device__ __forceinline__ float bf16r(float x) {
  unsigned int u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------- descriptors and frames
__device__ void unit3(double v[3]) {
  const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= r;
  v[1] /= r;
  v[2] /= r;
}
__device__ void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// two nearest atoms of species `sp` to atom a within [a0, a1), excluding `skip`
// (ties broken by the lower index)
__device__ void nearest2(const double* pos, const int8_t* species, int a0, int a1, int a, int sp, int skip,
                         int& i1, int& i2) {
  double d1 = INFINITY, d2 = INFINITY;
  i1 = -1;
  i2 = -1;
  for (int b = a0; b < a1; ++b) {
    if (b == a || b == skip || species[b] != sp) continue;
    const double dx = pos[b * 3] - pos[a * 3], dy = pos[b * 3 + 1] - pos[a * 3 + 1],
                 dz = pos[b * 3 + 2] - pos[a * 3 + 2];
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    if (d < d1) {
      d2 = d1;
      i2 = i1;
      d1 = d;
      i1 = b;
    } else if (d < d2) {
      d2 = d;
      i2 = b;
    }
  }
}

// e2 for an H whose O has no second H: the lab y axis (z when y is within 0.9
// of e1) with its e1 part removed
__device__ void complete_frame(const double e1[3], double e2[3]) {
  const bool use_y = fabs(e1[1]) <= 0.9;
  const double t[3] = {0.0, use_y ? 1.0 : 0.0, use_y ? 0.0 : 1.0};
  const double p = t[0] * e1[0] + t[1] * e1[1] + t[2] * e1[2];
  for (int c = 0; c < 3; ++c) e2[c] = t[c] - p * e1[c];
  unit3(e2);
}

// the atom's frame R = [e1 e2 e3].  O: e1 = bisector of the two nearest H,
// e2 = normal of their plane; H: e1 = nearest O -> H, e2 = normal of the plane
// of that O, the H and the O's nearest other H.  An O with fewer than two H and
// an H without an O keep the lab frame; an H whose O has no other H takes e2
// from complete_frame.
__device__ void atom_frame(const double* pos, const int8_t* species, int a0, int a1, int a, double e1[3],
                           double e2[3], double e3[3]) {
  for (int c = 0; c < 3; ++c) {
    e1[c] = c == 0 ? 1.0 : 0.0;
    e2[c] = c == 1 ? 1.0 : 0.0;
  }
  if (species[a] == 0) {
    int h1, h2;
    nearest2(pos, species, a0, a1, a, 1, -1, h1, h2);
    if (h2 >= 0) {
      double v1[3], v2[3];
      for (int c = 0; c < 3; ++c) {
        v1[c] = pos[h1 * 3 + c] - pos[a * 3 + c];
        v2[c] = pos[h2 * 3 + c] - pos[a * 3 + c];
      }
      unit3(v1);
      unit3(v2);
      for (int c = 0; c < 3; ++c) e1[c] = v1[c] + v2[c];
      unit3(e1);
      cross3(v1, v2, e2);
      unit3(e2);
    }
  } else {
    int o, o2;
    nearest2(pos, species, a0, a1, a, 0, -1, o, o2);
    if (o >= 0) {
      int hh, hh2;
      nearest2(pos, species, a0, a1, o, 1, a, hh, hh2);
      double v1[3], v2[3];
      for (int c = 0; c < 3; ++c) v1[c] = pos[a * 3 + c] - pos[o * 3 + c];
      for (int c = 0; c < 3; ++c) e1[c] = v1[c];
      unit3(e1);
      if (hh >= 0) {
        for (int c = 0; c < 3; ++c) v2[c] = pos[hh * 3 + c] - pos[o * 3 + c];
        cross3(v1, v2, e2);
        unit3(e2);
        const double pr = e2[0] * e1[0] + e2[1] * e1[1] + e2[2] * e1[2];
        for (int c = 0; c < 3; ++c) e2[c] -= pr * e1[c];
        unit3(e2);
      } else {
        complete_frame(e1, e2);
      }
    }
  }
  cross3(e1, e2, e3);
}

// Descriptors of one atom per thread, over the atoms of its unit within 6 A:
//   columns s*16 + k        radial comb: sum_B g_k(R_AB) fc(R_AB), 16 Gaussians
//   columns 32 + s*24 + 3k + i  direction moments in the atom's frame:
//                           sum_B g'_k(R_AB) fc(R_AB) (e_i . u_AB), 8 Gaussians
// (s = species of B, u_AB the unit vector A -> B), and the frame itself.
__global__ __launch_bounds__(NT) void features_kernel(int n_atoms, const int32_t* __restrict__ atom_unit,
                                                      const int32_t* __restrict__ unit_off,
                                                      const int8_t* __restrict__ species,
                                                      const double* __restrict__ pos, double* __restrict__ feat,
                                                      double* __restrict__ frames) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n_atoms) return;
  const int u = atom_unit[a];
  const int a0 = unit_off[u], a1 = unit_off[u + 1];
  double e1[3], e2[3], e3[3];
  atom_frame(pos, species, a0, a1, a, e1, e2, e3);
  if (frames)
    for (int c = 0; c < 3; ++c) {  // R = [e1 e2 e3], row-major R[c][j]
      frames[(int64_t)a * 9 + c * 3 + 0] = e1[c];
      frames[(int64_t)a * 9 + c * 3 + 1] = e2[c];
      frames[(int64_t)a * 9 + c * 3 + 2] = e3[c];
    }
  if (!feat) return;
  const double rc = 6.0 * kAng;
  const double r0 = 0.5 * kAng, dr = (6.0 - 0.5) * kAng / 15.0, drv = (6.0 - 0.5) * kAng / 7.0;
  // accumulators in register arrays indexed at compile time only (a runtime-
  // indexed array would live in scratch memory)
  double gO[16], gH[16], mO[24], mH[24];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    gO[k] = 0.0;
    gH[k] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < 24; ++k) {
    mO[k] = 0.0;
    mH[k] = 0.0;
  }
  constexpr double kInvE = 0.36787944117144233;  // exp(-1)
  for (int b = a0; b < a1; ++b) {
    if (b == a) continue;
    const double dx = pos[b * 3] - pos[a * 3], dy = pos[b * 3 + 1] - pos[a * 3 + 1], dz = pos[b * 3 + 2] - pos[a * 3 + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r >= rc) continue;
    const double fc = 0.5 * (cos(M_PI * r / rc) + 1.0);
    const int s = species[b];
    // Gaussians exp(-(v - k)^2 / 2) at v = (r - r0) / dr for k = 0, 1, ... by the
    // exact product recurrence g_{k+1} = g_k exp(v - k - 1/2): two exponentials
    // per pair and comb
    const double v = (r - r0) / dr;
    double gk = exp(-0.5 * v * v) * fc, ck = exp(v - 0.5);
    const double w = (r - r0) / drv;
    double hk = exp(-0.5 * w * w) * fc, dk = exp(w - 0.5);
    const double ir = 1.0 / r;
    const double u1 = (e1[0] * dx + e1[1] * dy + e1[2] * dz) * ir;
    const double u2 = (e2[0] * dx + e2[1] * dy + e2[2] * dz) * ir;
    const double u3 = (e3[0] * dx + e3[1] * dy + e3[2] * dz) * ir;
    if (s == 0) {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        gO[k] += gk;
        gk *= ck;
        ck *= kInvE;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        mO[3 * k] += hk * u1;
        mO[3 * k + 1] += hk * u2;
        mO[3 * k + 2] += hk * u3;
        hk *= dk;
        dk *= kInvE;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        gH[k] += gk;
        gk *= ck;
        ck *= kInvE;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        mH[3 * k] += hk * u1;
        mH[3 * k + 1] += hk * u2;
        mH[3 * k + 2] += hk * u3;
        hk *= dk;
        dk *= kInvE;
      }
    }
  }
  double* f = feat + (int64_t)a * NIN;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    f[k] = gO[k];
    f[16 + k] = gH[k];
  }
#pragma unroll
  for (int k = 0; k < 24; ++k) {
    f[32 + k] = mO[k];
    f[56 + k] = mH[k];
  }
}

// standardised FP32 rows of the listed atoms: x = (v - mean) / scale, with
// norm = [mean(width) | scale(width)]
__global__ __launch_bounds__(NT) void prep_kernel(int n, int width, const int32_t* __restrict__ idx,
                                                  const double* __restrict__ v, const float* __restrict__ norm,
                                                  float* __restrict__ x) {
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= n * width) return;
  const int i = e / width, k = e % width;
  const int a = idx ? idx[i] : i;
  x[e] = (float)((v[(int64_t)a * width + k] - (double)norm[k]) / (double)norm[width + k]);
}

// ---------------------------------------------------------------- network
// bfloat16 bits of x, round to nearest even (the rounding of bf16r)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  const unsigned int u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// LDS row strides (bf16 elements) of the forward pass: 4 extra elements per
// row spread the 8-byte operand reads of neighbouring rows over the banks
constexpr int LDX = NIN + 4, LDH = NHID + 4;

// one hidden layer of an atom tile (16 atoms per wave) on the matrix cores:
// z[a][j] = sum_k in[a][k] W[k][j] + b[j] with bf16 operands (in: bf16 rows
// of stride ldin, Wt: W transposed in bf16, rows of stride ldw) and FP32
// accumulation by v_mfma_f32_16x16x16_bf16; wave w takes atoms 16w..16w+15 and
// all NHID outputs (8 tiles of 16x16).  z goes to act (pre-activation, for the
// backward pass) and bf16(silu(z)) to hout.
template <int K>
__device__ void dense_hidden_mfma(const unsigned short* __restrict__ in, int ldin,
                                  const unsigned short* __restrict__ Wt, int ldw, const float* __restrict__ b,
                                  float* __restrict__ act, int m, unsigned short* __restrict__ hout) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = (lane >> 4) * 4;
  f32x4 acc[NHID / 16];
#pragma unroll
  for (int t = 0; t < NHID / 16; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x4 av = *reinterpret_cast<const bf16x4*>(in + (16 * w + r16) * ldin + k0 + kq);
    bf16x4 bv[NHID / 16];
#pragma unroll
    for (int t = 0; t < NHID / 16; ++t) bv[t] = *reinterpret_cast<const bf16x4*>(Wt + (16 * t + r16) * ldw + k0 + kq);
#pragma unroll
    for (int t = 0; t < NHID / 16; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[t], acc[t], 0, 0, 0);
  }
  // lane holds rows 16w + kq + i (i = 0..3) of output column 16t + r16
#pragma unroll
  for (int t = 0; t < NHID / 16; ++t) {
    const int j = 16 * t + r16;
    const float bj = b[j];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int a = 16 * w + kq + i;
      const float z = acc[t][i] + bj;
      if (act && a < m) act[(int64_t)a * 2 * NHID + j] = z;
      hout[a * LDH + j] = bf16_bits(silu(z));
    }
  }
}

// forward pass of one member over n atoms: y = W3 h2 + b3, h2 = silu(W2 h1 + b2),
// h1 = silu(W1 x + b1), every product with bf16 operands and FP32 accumulation
// on the matrix cores (the 9 outputs padded to one 16-wide tile).
// Persistent workgroups: the weights are converted to transposed bf16 in LDS
// once, then the workgroup takes 128-atom tiles blockIdx.x, blockIdx.x + gridDim.x, ...
// act (or null) receives the pre-activations z1, z2 per atom for the backward pass.
__global__ __launch_bounds__(FNT) void forward_kernel(const float* __restrict__ P, const float* __restrict__ x, int n,
                                                     float* __restrict__ y, float* __restrict__ act) {
  __shared__ __align__(16) unsigned short sW1t[NHID * LDX];
  __shared__ __align__(16) unsigned short sW2t[NHID * LDH];
  __shared__ __align__(16) unsigned short sH1[FTILE * LDH];
  __shared__ __align__(16) unsigned short sXH2[FTILE * LDH];  // x tile (stride LDX) for layer 1, then h2
  __shared__ __align__(16) unsigned short sW3t[16 * LDH];     // W3 transposed, outputs 9..15 zero
  for (int e = threadIdx.x; e < NIN * NHID; e += FNT) sW1t[(e % NHID) * LDX + e / NHID] = bf16_bits(P[OFF_W1 + e]);
  for (int e = threadIdx.x; e < NHID * NHID; e += FNT) sW2t[(e % NHID) * LDH + e / NHID] = bf16_bits(P[OFF_W2 + e]);
  for (int e = threadIdx.x; e < 16 * NHID; e += FNT) {
    const int o = e / NHID, k = e % NHID;
    sW3t[o * LDH + k] = o < NOUT ? bf16_bits(P[OFF_W3 + k * NOUT + o]) : (unsigned short)0;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = (lane >> 4) * 4;
  const float b3 = r16 < NOUT ? P[OFF_B3 + r16] : 0.0f;
  const int n_tiles = (n + FTILE - 1) / FTILE;
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int t0 = tile * FTILE;
    const int m = min(FTILE, n - t0);
    for (int e = threadIdx.x; e < FTILE * NIN; e += FNT) {
      const int a = e / NIN, k = e % NIN;
      sXH2[a * LDX + k] = a < m ? bf16_bits(x[(int64_t)t0 * NIN + e]) : (unsigned short)0;
    }
    __syncthreads();
    dense_hidden_mfma<NIN>(sXH2, LDX, sW1t, LDX, P + OFF_B1, act ? act + (int64_t)t0 * 2 * NHID : nullptr, m, sH1);
    __syncthreads();
    dense_hidden_mfma<NHID>(sH1, LDH, sW2t, LDH, P + OFF_B2, act ? act + (int64_t)t0 * 2 * NHID + NHID : nullptr, m,
                            sXH2);
    __syncthreads();
    // output layer: wave w takes atoms 16w..16w+15, one 16x16 tile over K = NHID
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k0 = 0; k0 < NHID; k0 += 16) {
      const bf16x4 av = *reinterpret_cast<const bf16x4*>(sXH2 + (16 * wv + r16) * LDH + k0 + kq);
      const bf16x4 bv = *reinterpret_cast<const bf16x4*>(sW3t + r16 * LDH + k0 + kq);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    if (r16 < NOUT)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = 16 * wv + kq + i;
        if (a < m) y[(int64_t)(t0 + a) * NOUT + r16] = acc[i] + b3;
      }
    __syncthreads();
  }
}

// Partial gradients of sum(dy . y) for one 64-atom tile into work[tile][NPAR],
// every product on the matrix cores (v_mfma_f32_16x16x16_bf16: bf16 operands,
// FP32 accumulation), rounded to bf16 at the same points as the forward pass:
//   dW3 = h2^T dy          dh2 = dy W3^T,  dz2 = dh2 silu'(z2)
//   dW2 = h1^T dz2         dh1 = dz2 W2^T, dz1 = dh1 silu'(z1)
//   dW1 = x^T dz1          db = sums of dy, dz2, dz1 (FP32, before rounding)
// An MFMA lane feeds four consecutive k of one row of A and of one column of B,
// so the operands of the weight gradients (contractions over atoms) are kept
// atom-contiguous (transposed) in LDS; rows of 64 atoms have stride LDA.
// Bias sums: per-lane partials over its four atoms, then a fixed-order sum
// over the 16 lane groups and waves.
constexpr int LDA = TILE + 4, LDO = 16 + 4;
__global__ __launch_bounds__(NT) void backward_mfma_kernel(const float* __restrict__ P, const float* __restrict__ x,
                                                           const float* __restrict__ act,
                                                           const float* __restrict__ dy, int n,
                                                           float* __restrict__ work) {
  __shared__ __align__(16) unsigned short sW2[NHID * LDH];    // W2[k][j]
  __shared__ __align__(16) unsigned short sW3[NHID * LDO];    // W3[k][o], o padded to 16
  __shared__ __align__(16) unsigned short sXT[NIN * LDA];     // x^T
  __shared__ __align__(16) unsigned short sH1T[NHID * LDA];   // h1^T
  __shared__ __align__(16) unsigned short sH2T[NHID * LDA];   // h2^T, later dz1^T
  __shared__ __align__(16) unsigned short sDY[TILE * LDO];    // dy (o padded)
  __shared__ __align__(16) unsigned short sDYT[16 * LDA];     // dy^T
  __shared__ __align__(16) unsigned short sDZ2[TILE * LDH];   // dz2
  __shared__ __align__(16) unsigned short sDZ2T[NHID * LDA];  // dz2^T
  __shared__ float sPb[2][NT / 64][4][NHID];                  // bias partials of dz2, dz1 [wave][lane group][j]
  float* g = work + (int64_t)blockIdx.x * NPAR;
  const int t0 = blockIdx.x * TILE;
  const int m = min(TILE, n - t0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = (lane >> 4) * 4, grp = lane >> 4;
  for (int e = threadIdx.x; e < NHID * NHID; e += NT) sW2[(e / NHID) * LDH + e % NHID] = bf16_bits(P[OFF_W2 + e]);
  for (int e = threadIdx.x; e < NHID * 16; e += NT) {
    const int k = e / 16, o = e % 16;
    sW3[k * LDO + o] = o < NOUT ? bf16_bits(P[OFF_W3 + k * NOUT + o]) : (unsigned short)0;
  }
  for (int e = threadIdx.x; e < TILE * NIN; e += NT) {
    const int a = e / NIN, i = e % NIN;
    sXT[i * LDA + a] = a < m ? bf16_bits(x[(int64_t)t0 * NIN + e]) : (unsigned short)0;
  }
  for (int e = threadIdx.x; e < TILE * NHID; e += NT) {
    const int a = e / NHID, k = e % NHID;
    const float* z = act + (int64_t)(t0 + a) * 2 * NHID;
    sH1T[k * LDA + a] = a < m ? bf16_bits(silu(z[k])) : (unsigned short)0;
    sH2T[k * LDA + a] = a < m ? bf16_bits(silu(z[NHID + k])) : (unsigned short)0;
  }
  for (int e = threadIdx.x; e < TILE * 16; e += NT) {
    const int a = e / 16, o = e % 16;
    const unsigned short v = (a < m && o < NOUT) ? bf16_bits(dy[(int64_t)(t0 + a) * NOUT + o]) : (unsigned short)0;
    sDY[a * LDO + o] = v;
    sDYT[o * LDA + a] = v;
  }
  if (threadIdx.x < NOUT) {  // db3 in atom order
    float sum = 0.0f;
    for (int a = 0; a < m; ++a) sum += dy[(int64_t)(t0 + a) * NOUT + threadIdx.x];
    g[OFF_B3 + threadIdx.x] = sum;
  }
  __syncthreads();
  // dW3 (128 x 16 tiles: wave w takes k-tiles w and w + 4) and dh2 -> dz2
  for (int t = wv; t < NHID / 16; t += NT / 64) {
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k0 = 0; k0 < TILE; k0 += 16) {
      const bf16x4 av = *reinterpret_cast<const bf16x4*>(sH2T + (16 * t + r16) * LDA + k0 + kq);
      const bf16x4 bv = *reinterpret_cast<const bf16x4*>(sDYT + r16 * LDA + k0 + kq);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    if (r16 < NOUT)
#pragma unroll
      for (int i = 0; i < 4; ++i) g[OFF_W3 + (16 * t + kq + i) * NOUT + r16] = acc[i];
  }
  {
    const bf16x4 av = *reinterpret_cast<const bf16x4*>(sDY + (16 * wv + r16) * LDO + kq);
#pragma unroll
    for (int t = 0; t < NHID / 16; ++t) {
      const bf16x4 bv = *reinterpret_cast<const bf16x4*>(sW3 + (16 * t + r16) * LDO + kq);
      const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, f32x4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
      const int j = 16 * t + r16;
      float bsum = 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = 16 * wv + kq + i;
        const float dz = a < m ? acc[i] * dsilu(act[(int64_t)(t0 + a) * 2 * NHID + NHID + j]) : 0.0f;
        bsum += dz;
        const unsigned short b = bf16_bits(dz);
        sDZ2[a * LDH + j] = b;
        sDZ2T[j * LDA + a] = b;
      }
      sPb[0][wv][grp][j] = bsum;
    }
  }
  __syncthreads();
  // dW2 (128 x 128: wave w takes 16 of the 64 tiles) and dh1 -> dz1 (into sH2T)
  for (int tt = wv; tt < (NHID / 16) * (NHID / 16); tt += NT / 64) {
    const int ti = tt / (NHID / 16), tj = tt % (NHID / 16);
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k0 = 0; k0 < TILE; k0 += 16) {
      const bf16x4 av = *reinterpret_cast<const bf16x4*>(sH1T + (16 * ti + r16) * LDA + k0 + kq);
      const bf16x4 bv = *reinterpret_cast<const bf16x4*>(sDZ2T + (16 * tj + r16) * LDA + k0 + kq);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) g[OFF_W2 + (16 * ti + kq + i) * NHID + 16 * tj + r16] = acc[i];
  }
  {
    f32x4 acc[NHID / 16];
#pragma unroll
    for (int t = 0; t < NHID / 16; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k0 = 0; k0 < NHID; k0 += 16) {
      const bf16x4 av = *reinterpret_cast<const bf16x4*>(sDZ2 + (16 * wv + r16) * LDH + k0 + kq);
#pragma unroll
      for (int t = 0; t < NHID / 16; ++t) {
        const bf16x4 bv = *reinterpret_cast<const bf16x4*>(sW2 + (16 * t + r16) * LDH + k0 + kq);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < NHID / 16; ++t) {
      const int k = 16 * t + r16;
      float bsum = 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = 16 * wv + kq + i;
        const float dz = a < m ? acc[t][i] * dsilu(act[(int64_t)(t0 + a) * 2 * NHID + k]) : 0.0f;
        bsum += dz;
        sH2T[k * LDA + a] = bf16_bits(dz);
      }
      sPb[1][wv][grp][k] = bsum;
    }
  }
  __syncthreads();
  // dW1 (32 x 128: wave w takes 4 of the 16 tiles); the bias sums in fixed order
  for (int tt = wv; tt < (NIN / 16) * (NHID / 16); tt += NT / 64) {
    const int ti = tt / (NHID / 16), tj = tt % (NHID / 16);
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k0 = 0; k0 < TILE; k0 += 16) {
      const bf16x4 av = *reinterpret_cast<const bf16x4*>(sXT + (16 * ti + r16) * LDA + k0 + kq);
      const bf16x4 bv = *reinterpret_cast<const bf16x4*>(sH2T + (16 * tj + r16) * LDA + k0 + kq);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) g[OFF_W1 + (16 * ti + kq + i) * NHID + 16 * tj + r16] = acc[i];
  }
  for (int j = threadIdx.x; j < 2 * NHID; j += NT) {
    const int which = j / NHID, jj = j % NHID;
    float sum = 0.0f;
    for (int w = 0; w < NT / 64; ++w)
      for (int q = 0; q < 4; ++q) sum += sPb[which][w][q][jj];
    g[(which == 0 ? OFF_B2 : OFF_B1) + jj] = sum;
  }
}

__global__ __launch_bounds__(NT) void reduce_tiles_kernel(const float* __restrict__ work, int n_tiles, int width,
                                                          float* __restrict__ out) {
  const int p = blockIdx.x * NT + threadIdx.x;
  if (p >= width) return;
  float s = 0.0f;
  for (int t = 0; t < n_tiles; ++t) s += work[(int64_t)t * width + p];
  out[p] = s;
}

// loss = mean (y - t)^2 ; dy = 2 (y - t) / (n * 9); per-block partial losses in work
__global__ __launch_bounds__(NT) void mse_kernel(const float* __restrict__ y, const float* __restrict__ t, int count,
                                                 float* __restrict__ dy, float* __restrict__ work) {
  __shared__ float red[NT];
  const int e = blockIdx.x * NT + threadIdx.x;
  float d = 0.0f;
  if (e < count) {
    d = y[e] - t[e];
    dy[e] = 2.0f * d / (float)count;
  }
  red[threadIdx.x] = d * d;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) work[blockIdx.x] = red[0];
}

__global__ void mse_finish_kernel(const float* __restrict__ work, int nb, int count, float* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.0f;
    for (int b = 0; b < nb; ++b) s += work[b];
    loss[0] = s / (float)count;
  }
}

__global__ __launch_bounds__(NT) void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, int count, float lr,
                                                  float b1, float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * NT + threadIdx.x;
  if (p >= count) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

__global__ __launch_bounds__(NT) void gather_kernel_f(const float* __restrict__ src, const int32_t* __restrict__ idx,
                                                      int n, int width, float* __restrict__ dst) {
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= n * width) return;
  const int i = e / width, k = e % width;
  dst[e] = src[(int64_t)idx[i] * width + k];
}

// mean and standard deviation of each column (two passes, fixed order)
__global__ __launch_bounds__(NT) void moments_kernel(const double* __restrict__ x, const int32_t* __restrict__ idx,
                                                     int n, int width, float* __restrict__ out) {
  __shared__ double red[NT];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += x[(int64_t)(idx ? idx[i] : i) * width + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double mean = red[0] / n;
  __syncthreads();
  double q = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double d = x[(int64_t)(idx ? idx[i] : i) * width + k] - mean;
    q += d * d;
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[k] = (float)mean;
    const double sd = sqrt(red[0] / n);
    out[width + k] = (float)(sd > 1e-12 ? sd : 1.0);
  }
}

// training targets: R^T Z R - Q I (Q optional) for the listed atoms, FP64
__global__ __launch_bounds__(NT) void to_local_kernel(int n, const int32_t* __restrict__ idx,
                                                      const double* __restrict__ frames,
                                                      const double* __restrict__ born,
                                                      const double* __restrict__ charges, double* __restrict__ out) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int64_t a = idx ? idx[i] : i;
  const double* R = frames + a * 9;
  const double* Z = born + a * 9;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) {
      double s = 0.0;
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) s += R[j * 3 + p] * Z[j * 3 + k] * R[k * 3 + q];
      if (charges && p == q) s -= charges[a];
      out[(int64_t)i * 9 + p * 3 + q] = s;
    }
}

// ensemble combination: per atom, member outputs y_m -> Z_m = Q I + R (y y_scale + y_mean) R^T
// (Q the Mulliken charge); mean over members into born, largest per-component
// standard deviation into std
__global__ __launch_bounds__(NT) void combine_kernel(int n_atoms, const int8_t* __restrict__ species,
                                                     const int32_t* __restrict__ pos_in_species,
                                                     const int32_t* __restrict__ n_species,
                                                     const float* __restrict__ ybuf, const float* __restrict__ norm,
                                                     const double* __restrict__ frames,
                                                     const double* __restrict__ charges, double* __restrict__ born,
                                                     double* __restrict__ std) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n_atoms) return;
  const int s = species[a];
  const int i = pos_in_species[a];
  const float* nm = norm + s * CAVDFTB_SG_N_NORM;
  const double* R = frames + (int64_t)a * 9;
  double mean[9], m2[9];
  for (int e = 0; e < 9; ++e) mean[e] = m2[e] = 0.0;
  const int64_t base_s = s == 0 ? 0 : (int64_t)CAVDFTB_SG_MEMBERS * n_species[0] * NOUT;
  for (int mb = 0; mb < CAVDFTB_SG_MEMBERS; ++mb) {
    const float* y = ybuf + base_s + ((int64_t)mb * n_species[s] + i) * NOUT;
    double zl[9];
    for (int e = 0; e < 9; ++e) zl[e] = (double)y[e] * nm[2 * NIN + NOUT + e] + nm[2 * NIN + e];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        double v = 0.0;
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k) v += R[p * 3 + j] * zl[j * 3 + k] * R[q * 3 + k];
        const double d = v - mean[p * 3 + q];  // Welford
        mean[p * 3 + q] += d / (mb + 1);
        m2[p * 3 + q] += d * (v - mean[p * 3 + q]);
      }
  }
  double smax = 0.0;
  const double qa = charges ? charges[a] : 0.0;
  for (int e = 0; e < 9; ++e) {
    born[(int64_t)a * 9 + e] = mean[e] + ((e % 4) == 0 ? qa : 0.0);
    smax = fmax(smax, sqrt(m2[e] / CAVDFTB_SG_MEMBERS));
  }
  if (std) std[a] = smax;
}

// per unit: acoustic-sum projection of the ensemble mean and the fallback flag
__global__ __launch_bounds__(NT) void asr_flag_kernel(int n_units, const int32_t* __restrict__ unit_off,
                                                      double* __restrict__ born, const double* __restrict__ std,
                                                      double thr, int32_t* __restrict__ flag,
                                                      unsigned long long* __restrict__ n_flagged) {
  const int u = blockIdx.x * NT + threadIdx.x;
  if (u >= n_units) return;
  const int a0 = unit_off[u], a1 = unit_off[u + 1];
  double s[9];
  for (int e = 0; e < 9; ++e) s[e] = 0.0;
  double smax = 0.0;
  for (int a = a0; a < a1; ++a) {
    for (int e = 0; e < 9; ++e) s[e] += born[(int64_t)a * 9 + e];
    smax = fmax(smax, std[a]);
  }
  for (int a = a0; a < a1; ++a)
    for (int e = 0; e < 9; ++e) born[(int64_t)a * 9 + e] -= s[e] / (a1 - a0);
  flag[u] = smax > thr ? 1 : 0;
  if (n_flagged && smax > thr) atomicAdd(n_flagged, 1ull);
}

__global__ __launch_bounds__(NT) void zpol_from_born_kernel(int n, const double* __restrict__ born, double e0,
                                                            double e1, double e2, double* __restrict__ zp) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n) return;
  for (int b = 0; b < 3; ++b)
    zp[a * 3 + b] = e0 * born[(int64_t)a * 9 + b] + e1 * born[(int64_t)a * 9 + 3 + b] + e2 * born[(int64_t)a * 9 + 6 + b];
}

// compact the displaced-job (or field-job) list of the flagged units of one
// bucket, in unit order (one workgroup; block scan over chunks of NT units)
__global__ __launch_bounds__(NT) void fd_compact_kernel(int n_units_b, const int32_t* __restrict__ units_b,
                                                        const int32_t* __restrict__ unit_off,
                                                        const int32_t* __restrict__ flag, int field,
                                                        int32_t* __restrict__ job_unit,
                                                        int32_t* __restrict__ job_disp, int32_t* __restrict__ job0,
                                                        int32_t* __restrict__ n_jobs) {
  __shared__ int scan[NT];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < n_units_b; c0 += NT) {
    const int w = c0 + threadIdx.x;
    int cnt = 0, u = -1, na = 0;
    if (w < n_units_b) {
      u = units_b[w];
      na = unit_off[u + 1] - unit_off[u];
      cnt = flag[u] ? (field ? 6 : 6 * na) : 0;
    }
    scan[threadIdx.x] = cnt;
    __syncthreads();
    for (int d = 1; d < NT; d <<= 1) {  // inclusive Hillis-Steele scan
      const int v = (int)threadIdx.x >= d ? scan[threadIdx.x - d] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    const int start = base + scan[threadIdx.x] - cnt;
    if (w < n_units_b) {
      job0[w] = cnt ? start : -1;
      for (int j = 0; j < cnt; ++j) {
        job_unit[start + j] = u;
        job_disp[start + j] = field ? -2 - j : j;  // field: -2 - (dir*2 + sign); else (atom*3 + dir)*2 + sign
      }
    }
    __syncthreads();
    if (threadIdx.x == NT - 1) base += scan[NT - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) n_jobs[0] = base;
}

inline int nb(int64_t n) { return (int)((n + NT - 1) / NT); }

}  // namespace

hipError_t launch_sg_features(int n_atoms, const int32_t* atom_unit, const int32_t* unit_off, const int8_t* species,
                              const double* pos, double* feat, double* frames, hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3(nb(n_atoms)), dim3(NT), 0, s, n_atoms, atom_unit, unit_off, species, pos,
                     feat, frames);
  return hipGetLastError();
}
hipError_t launch_sg_prep(int n, int width, const int32_t* idx, const double* v, const float* norm, float* x,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(prep_kernel, dim3(nb((int64_t)n * width)), dim3(NT), 0, s, n, width, idx, v, norm, x);
  return hipGetLastError();
}
hipError_t launch_sg_forward(const float* P, const float* x, int n, float* y, float* act, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int n_tiles = (n + FTILE - 1) / FTILE;
  hipLaunchKernelGGL(forward_kernel, dim3(std::min(n_tiles, kForwardGrid)), dim3(FNT), 0, s, P, x, n, y, act);
  return hipGetLastError();
}
hipError_t launch_sg_backward(const float* P, const float* x, const float* act, const float* dy, int n, float* grad,
                              float* work, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int tiles = (n + TILE - 1) / TILE;
  hipLaunchKernelGGL(backward_mfma_kernel, dim3(tiles), dim3(NT), 0, s, P, x, act, dy, n, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_tiles_kernel, dim3(nb(NPAR)), dim3(NT), 0, s, work, tiles, NPAR, grad);
  return hipGetLastError();
}
hipError_t launch_sg_mse(const float* y, const float* t, int count, float* dy, float* loss, float* work,
                         hipStream_t s) {
  const int blocks = nb(count);
  hipLaunchKernelGGL(mse_kernel, dim3(blocks), dim3(NT), 0, s, y, t, count, dy, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mse_finish_kernel, dim3(1), dim3(64), 0, s, work, blocks, count, loss);
  return hipGetLastError();
}
hipError_t launch_sg_adam(float* w, const float* g, float* m, float* v, int count, float lr, float b1, float b2,
                          float eps, int step, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(nb(count)), dim3(NT), 0, s, w, g, m, v, count, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t launch_sg_gather(const float* src, const int32_t* idx, int n, int width, float* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel_f, dim3(nb((int64_t)n * width)), dim3(NT), 0, s, src, idx, n, width, dst);
  return hipGetLastError();
}
hipError_t launch_sg_moments(const double* x, const int32_t* idx, int n, int width, float* out, hipStream_t s) {
  hipLaunchKernelGGL(moments_kernel, dim3(width), dim3(NT), 0, s, x, idx, n, width, out);
  return hipGetLastError();
}
hipError_t launch_sg_to_local(int n, const int32_t* idx, const double* frames, const double* born,
                              const double* charges, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_local_kernel, dim3(nb(n)), dim3(NT), 0, s, n, idx, frames, born, charges, out);
  return hipGetLastError();
}
hipError_t launch_sg_combine(int n_atoms, const int8_t* species, const int32_t* pos_in_species,
                             const int32_t* n_species, const float* ybuf, const float* norm, const double* frames,
                             const double* charges, double* born, double* std, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3(nb(n_atoms)), dim3(NT), 0, s, n_atoms, species, pos_in_species, n_species,
                     ybuf, norm, frames, charges, born, std);
  return hipGetLastError();
}
hipError_t launch_sg_asr_flag(int n_units, const int32_t* unit_off, double* born, const double* std, double thr,
                              int32_t* flag, unsigned long long* n_flagged, hipStream_t s) {
  hipLaunchKernelGGL(asr_flag_kernel, dim3(nb(n_units)), dim3(NT), 0, s, n_units, unit_off, born, std, thr, flag,
                     n_flagged);
  return hipGetLastError();
}
hipError_t launch_fd_compact(int n_units_b, const int32_t* units_b, const int32_t* unit_off, const int32_t* flag,
                             int field, int32_t* job_unit, int32_t* job_disp, int32_t* job0, int32_t* n_jobs,
                             hipStream_t s) {
  hipLaunchKernelGGL(fd_compact_kernel, dim3(1), dim3(NT), 0, s, n_units_b, units_b, unit_off, flag, field, job_unit,
                     job_disp, job0, n_jobs);
  return hipGetLastError();
}

hipError_t launch_zpol_from_born(int n, const double* born, const double pol[3], double* zp, hipStream_t s) {
  hipLaunchKernelGGL(zpol_from_born_kernel, dim3(nb(n)), dim3(NT), 0, s, n, born, pol[0], pol[1], pol[2], zp);
  return hipGetLastError();
}

}  // namespace cavdftb
