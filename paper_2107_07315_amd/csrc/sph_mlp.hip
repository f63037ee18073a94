// EoS surrogate network on the GPU: training (forward and backward passes on the matrix cores,
// Adam on FP32 master weights), evaluation, and the trust mask that decides, per cell of the EoS
// table, whether the density pass may use the network instead of table interpolation.
#include <math.h>
#include <string.h>

#include <vector>

#include "sph_internal.h"
#include "sph_mlp.h"

struct MlpState {
  float* w = nullptr;      // FP32 master parameters
  float* wr = nullptr;     // the parameters the kernels use (W2, W3 rounded to BF16)
  float* m = nullptr;      // Adam moments
  float* v = nullptr;
  uint2* pack = nullptr;   // wa2, wa3, wt2, wt3: 4 x 1024 entries
  float* gpart = nullptr;  // per-block gradient partials [kMaxBlocks][MLP_NPARAM]
  float* lpart = nullptr;  // per-block loss partials
  float* gsum = nullptr;   // summed gradient (sph_mlp_grad)
  float* scal = nullptr;   // [0] loss of the last step
  uint8_t* trust = nullptr;
  unsigned long long* served = nullptr;   // counter of sph_mlp_count_served
  int64_t trust_cells = 0;
  int64_t step = 0;        // Adam steps taken
  bool loaded = false;
  bool norm_set = false;
  MlpNorm norm;
  // the network's domain in (ln rho, ln u) (sph_mlp_set_domain): lnr_lo, lnr_hi, lnu_lo, lnu_hi;
  // the table's box when not set
  bool dom_set = false;
  double dom[4] = {0.0, 0.0, 0.0, 0.0};
  double* gpart64 = nullptr;  // readout fit: per-block Gram partials
};

namespace {

constexpr int kMaxBatch = 8192;   // samples per batch (a multiple of 64)
constexpr int kGradSamples = 16;  // samples per gradient workgroup: 512 workgroups for the largest batch
constexpr int kMaxBlocks = kMaxBatch / kGradSamples;
constexpr int LP = 68;            // padded row of the LDS matrices (8- and 16-byte aligned rows)

__device__ __forceinline__ float wave_sum_f(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ bf16x4 lds_b4(const uint16_t* p) {   // 4 consecutive BF16 (8-byte aligned)
  return as_bf16x4(*reinterpret_cast<const uint2*>(p));
}
__device__ __forceinline__ bf16x4 lds_b4_strided(const uint16_t* p, int stride) {
  bf16x4 v;
  v[0] = (short)p[0];
  v[1] = (short)p[stride];
  v[2] = (short)p[2 * stride];
  v[3] = (short)p[3 * stride];
  return v;
}
__device__ __forceinline__ void lds_store_b4(uint16_t* p, float a, float b, float c, float d) {
  *reinterpret_cast<uint2*>(p) = make_uint2(pk_bf16(a, b), pk_bf16(c, d));
}
// the BF16 parts hi = bf16(h) and lo = bf16(h - hi) of 4 activations (see split_bf16)
__device__ __forceinline__ void lds_store_split(uint16_t* hi, uint16_t* lo, float a, float b, float c, float d) {
  const uint32_t w0 = pk_bf16(a, b), w1 = pk_bf16(c, d);
  *reinterpret_cast<uint2*>(hi) = make_uint2(w0, w1);
  *reinterpret_cast<uint2*>(lo) =
      make_uint2(pk_bf16(a - bf16_lo(w0), b - bf16_hi(w0)), pk_bf16(c - bf16_lo(w1), d - bf16_hi(w1)));
}

struct GradArgs {
  MlpView M;
  const float* x;    // normalised inputs, 2 per sample
  const float* t;    // normalised targets
  int64_t off;       // first sample of the batch; samples wrap modulo n
  int64_t n;
  int batch;         // samples in the batch (multiple of 64); block b takes samples [NS b, NS b + NS)
  float* gpart;
  float* lpart;
};

// Gradient of L = 1/(2 batch) sum_s sum_o (y_so - t_so)^2 over the block's NS samples (lane l <
// NS = sample l), written as this block's partial.  Layers 2 and 3 and their weight gradients and
// back-propagated activations are products on the matrix cores (64 x 64 x NS and 64 x NS x 64);
// activations are kept in LDS sample-major (row = sample, column = feature).  The forward
// products take the activations as two BF16 parts, as the inference does (the loss is that of the
// network the kernels evaluate); the weight gradients use their high parts.  NS = 16 spreads a
// 4096-sample batch over 256 workgroups, one per CU.
template <int NS>
__global__ __launch_bounds__(64) void k_mlp_grad(GradArgs G) {
  static_assert(NS % 16 == 0 && NS <= 64, "whole 16-sample tiles");
  constexpr int NT = NS / 16;   // 16-sample tiles
  __shared__ __align__(16) uint16_t Ht1[NS * LP];
  __shared__ __align__(16) uint16_t Ht2[NS * LP];
  __shared__ __align__(16) uint16_t Lt1[NS * LP];   // low BF16 parts of the activations
  __shared__ __align__(16) uint16_t Lt2[NS * LP];
  __shared__ __align__(16) uint16_t Gt[NS * LP];
  __shared__ __align__(16) float Zt2[NS * LP];
  __shared__ __align__(16) float Zt3[NS * LP];
  __shared__ __align__(16) float G32[NS * LP];
  __shared__ float xs[NS][2], dys[NS][2];
  const int l = threadIdx.x, q = l >> 4, r = l & 15;
  const bool own = l < NS;   // the lane holds a sample
  const MlpView& M = G.M;
  const float* w = M.wr;
  const int64_t sg = (G.off + (int64_t)blockIdx.x * NS + (own ? l : 0)) % G.n;
  const float x0 = own ? G.x[2 * sg] : 0.f, x1 = own ? G.x[2 * sg + 1] : 0.f;
  const float t0 = own ? G.t[2 * sg] : 0.f, t1 = own ? G.t[2 * sg + 1] : 0.f;
  float* gp = G.gpart + (int64_t)blockIdx.x * MLP_NPARAM;
  if (own) {
    xs[l][0] = x0;
    xs[l][1] = x1;
    // ---- forward ------------------------------------------------------------------------------
    for (int f = 0; f < 64; f += 4) {
      float h[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        h[j] = silu_f(w[MLP_OW1 + 2 * (f + j)] * x0 + w[MLP_OW1 + 2 * (f + j) + 1] * x1 + w[MLP_OB1 + f + j]);
      lds_store_split(&Ht1[l * LP + f], &Lt1[l * LP + f], h[0], h[1], h[2], h[3]);
    }
  }
  __syncthreads();
  // hidden layers: C tile (features 16 mt + 4q + j, samples 16 nt + r)
  for (int layer = 0; layer < 2; ++layer) {
    const uint2* wa = layer == 0 ? M.wa2 : M.wa3;
    const int ob = layer == 0 ? MLP_OB2 : MLP_OB3;
    const uint16_t* Hin = layer == 0 ? Ht1 : Ht2;
    const uint16_t* Lin = layer == 0 ? Lt1 : Lt2;
    float* Z = layer == 0 ? Zt2 : Zt3;
    for (int nt = 0; nt < NT; ++nt) {
      bf16x4 b[4], bl[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        b[kk] = lds_b4(&Hin[(16 * nt + r) * LP + 16 * kk + 4 * q]);
        bl[kk] = lds_b4(&Lin[(16 * nt + r) * LP + 16 * kk + 4 * q]);
      }
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const bf16x4 wv = as_bf16x4(wa[(mt * 4 + kk) * 64 + l]);
          acc = mfma_bf16(wv, b[kk], acc);
          acc = mfma_bf16(wv, bl[kk], acc);
        }
        float z[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) z[j] = acc[j] + w[ob + 16 * mt + 4 * q + j];
        *reinterpret_cast<float4*>(&Z[(16 * nt + r) * LP + 16 * mt + 4 * q]) = make_float4(z[0], z[1], z[2], z[3]);
        if (layer == 0)
          lds_store_split(&Ht2[(16 * nt + r) * LP + 16 * mt + 4 * q], &Lt2[(16 * nt + r) * LP + 16 * mt + 4 * q],
                          silu_f(z[0]), silu_f(z[1]), silu_f(z[2]), silu_f(z[3]));
      }
    }
    __syncthreads();
  }
  // output layer and loss (lane = sample)
  const float inv = 1.0f / (float)G.batch;
  float loss = 0.f, d0 = 0.f, d1 = 0.f;
  if (own) {
    float y0 = w[MLP_OB4], y1 = w[MLP_OB4 + 1];
    for (int f = 0; f < 64; ++f) {
      const float h3 = silu_f(Zt3[l * LP + f]);
      y0 += w[MLP_OW4 + f] * h3;
      y1 += w[MLP_OW4 + MLP_H + f] * h3;
    }
    const float e0 = y0 - t0, e1 = y1 - t1;
    loss = 0.5f * (e0 * e0 + e1 * e1) * inv;
    d0 = e0 * inv;
    d1 = e1 * inv;
    dys[l][0] = d0;
    dys[l][1] = d1;
    // ---- backward -----------------------------------------------------------------------------
    // g3 = (W4^T dy) * silu'(z3)  (lane = sample)
    for (int f = 0; f < 64; f += 4) {
      float g[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        g[j] = (w[MLP_OW4 + f + j] * d0 + w[MLP_OW4 + MLP_H + f + j] * d1) * dsilu_f(Zt3[l * LP + f + j]);
      *reinterpret_cast<float4*>(&G32[l * LP + f]) = make_float4(g[0], g[1], g[2], g[3]);
      lds_store_b4(&Gt[l * LP + f], g[0], g[1], g[2], g[3]);
    }
  }
  __syncthreads();
  {  // dW4, db3 (lane = feature), db4
    const int f = l;
    float a0 = 0.f, a1 = 0.f, bsum = 0.f;
    for (int s = 0; s < NS; ++s) {
      const float h3 = silu_f(Zt3[s * LP + f]);
      a0 += dys[s][0] * h3;
      a1 += dys[s][1] * h3;
      bsum += G32[s * LP + f];
    }
    gp[MLP_OW4 + f] = a0;
    gp[MLP_OW4 + MLP_H + f] = a1;
    gp[MLP_OB3 + f] = bsum;
    const float s0 = wave_sum_f(d0), s1 = wave_sum_f(d1);
    if (l == 0) {
      gp[MLP_OB4] = s0;
      gp[MLP_OB4 + 1] = s1;
    }
  }
  // layers 3 and 2: dW = G * H_in^T (K = samples), dH_in = W^T * G (K = out features)
  for (int layer = 1; layer >= 0; --layer) {
    const uint16_t* Hin = layer == 1 ? Ht2 : Ht1;
    const uint2* wt = layer == 1 ? M.wt3 : M.wt2;
    const int ow = layer == 1 ? MLP_OW3 : MLP_OW2;
    for (int mt = 0; mt < 4; ++mt)
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < NT; ++kk) {
          // A[out 16mt + r][sample 16kk + 4q + j], B[sample 16kk + 4q + j][in 16nt + r]
          const bf16x4 a = lds_b4_strided(&Gt[(16 * kk + 4 * q) * LP + 16 * mt + r], LP);
          const bf16x4 b = lds_b4_strided(&Hin[(16 * kk + 4 * q) * LP + 16 * nt + r], LP);
          acc = mfma_bf16(a, b, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) gp[ow + MLP_H * (16 * mt + 4 * q + j) + 16 * nt + r] = acc[j];
      }
    f32x4 dh[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          acc = mfma_bf16(as_bf16x4(wt[(mt * 4 + kk) * 64 + l]), lds_b4(&Gt[(16 * nt + r) * LP + 16 * kk + 4 * q]), acc);
        dh[mt][nt] = acc;
      }
    __syncthreads();   // the G of this layer is consumed
    // g_in = dH_in * silu'(z_in): z2 from LDS, z1 recomputed from the inputs
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int s = 16 * nt + r, f0 = 16 * mt + 4 * q;
        float g[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int f = f0 + j;
          const float z = layer == 1 ? Zt2[s * LP + f]
                                     : w[MLP_OW1 + 2 * f] * xs[s][0] + w[MLP_OW1 + 2 * f + 1] * xs[s][1] + w[MLP_OB1 + f];
          g[j] = dh[mt][nt][j] * dsilu_f(z);
        }
        *reinterpret_cast<float4*>(&G32[s * LP + f0]) = make_float4(g[0], g[1], g[2], g[3]);
        lds_store_b4(&Gt[s * LP + f0], g[0], g[1], g[2], g[3]);
      }
    __syncthreads();
    const int f = l;
    if (layer == 1) {   // db2
      float bsum = 0.f;
      for (int s = 0; s < NS; ++s) bsum += G32[s * LP + f];
      gp[MLP_OB2 + f] = bsum;
    } else {            // dW1, db1
      float a0 = 0.f, a1 = 0.f, bsum = 0.f;
      for (int s = 0; s < NS; ++s) {
        const float g = G32[s * LP + f];
        a0 += g * xs[s][0];
        a1 += g * xs[s][1];
        bsum += g;
      }
      gp[MLP_OW1 + 2 * f] = a0;
      gp[MLP_OW1 + 2 * f + 1] = a1;
      gp[MLP_OB1 + f] = bsum;
    }
  }
  const float ls = wave_sum_f(loss);
  if (l == 0) G.lpart[blockIdx.x] = ls;
}

// Sums the block partials in block order (deterministic), then optionally one Adam step on the
// FP32 master weights and the copy the kernels use; block 0 also sums the loss.
__global__ __launch_bounds__(256) void k_mlp_adam(float* w, float* wr, float* m, float* v, const float* gpart,
                                                  const float* lpart, int nblk, float lr, float bc1, float bc2,
                                                  float* gsum, float* loss_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  // block partials summed in block order; their loads are issued 8 at a time (one wait per 8)
  auto sum_parts = [&](const float* part, int64_t stride, int64_t off) {
    float s = 0.f;
    int b = 0;
    for (; b + 8 <= nblk; b += 8) {
      float t[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) t[k] = part[(int64_t)(b + k) * stride + off];
#pragma unroll
      for (int k = 0; k < 8; ++k) s += t[k];
    }
    for (; b < nblk; ++b) s += part[(int64_t)b * stride + off];
    return s;
  };
  if (p < MLP_NPARAM) {
    const float g = sum_parts(gpart, MLP_NPARAM, p);
    if (gsum) gsum[p] = g;
    if (lr > 0.f) {
      const float mm = 0.9f * m[p] + 0.1f * g;
      const float vv = 0.999f * v[p] + 0.001f * g * g;
      m[p] = mm;
      v[p] = vv;
      const float wn = w[p] - lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
      w[p] = wn;
      wr[p] = mlp_bf16_param(p) ? bf16_round(wn) : wn;
    }
  }
  if (p == 0 && loss_out) *loss_out = sum_parts(lpart, 1, 0);
}

// MFMA A-operand packs of W2, W3 and their transposes from the rounded weights.
__global__ __launch_bounds__(256) void k_mlp_pack(const float* wr, uint2* pack) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;   // 4 packs x 16 tiles x 64 lanes
  if (i >= 4 * 1024) return;
  const int which = i >> 10, tile = (i >> 6) & 15, l = i & 63;
  const int mt = tile >> 2, kk = tile & 3, q = l >> 4, r = l & 15;
  const int ow = (which & 1) ? MLP_OW3 : MLP_OW2;
  const bool tr = which >= 2;
  uint32_t h[4];
  for (int j = 0; j < 4; ++j) {
    const int row = 16 * mt + r, col = 16 * kk + 4 * q + j;   // element (row, col) of W or W^T
    const float e = tr ? wr[ow + MLP_H * col + row] : wr[ow + MLP_H * row + col];
    h[j] = bf16_bits(e);
  }
  pack[i] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
}

// The parameters as the kernels use them: the matrix-core weights rounded to BF16, the rest FP32.
__global__ __launch_bounds__(256) void k_round(const float* w, float* wr, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wr[i] = mlp_bf16_param(i) ? bf16_round(w[i]) : w[i];
}

// min / max of the finite table nodes of ln P and ln c_s^2 in rows [i0, i1] and columns [j0, j1]
// of the nu-column table (one block)
__global__ __launch_bounds__(256) void k_table_range(const double* __restrict__ lnP, const double* __restrict__ lnc,
                                                     int i0, int i1, int j0, int j1, int nu, float* out) {
  __shared__ double red[4][256];
  double v[4] = {1e300, -1e300, 1e300, -1e300};
  const int64_t w = j1 - j0 + 1, n = (int64_t)(i1 - i0 + 1) * w;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    const int64_t i = (int64_t)(i0 + k / w) * nu + j0 + k % w;
    const double a = lnP[i], b = lnc[i];
    if (isfinite(a)) { v[0] = fmin(v[0], a); v[1] = fmax(v[1], a); }
    if (isfinite(b)) { v[2] = fmin(v[2], b); v[3] = fmax(v[3], b); }
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 4; ++k)
        red[k][threadIdx.x] = (k & 1) ? fmax(red[k][threadIdx.x], red[k][threadIdx.x + s])
                                      : fmin(red[k][threadIdx.x], red[k][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = (float)(0.5 * (red[0][0] + red[1][0]));
    out[1] = (float)(0.5 * (red[2][0] + red[3][0]));
    out[2] = (float)(0.5 * (red[1][0] - red[0][0]));
    out[3] = (float)(0.5 * (red[3][0] - red[2][0]));
  }
}

// training pairs: normalised inputs and table-interpolated normalised targets
__global__ __launch_bounds__(256) void k_mlp_targets(sph_params p, MlpNorm nm, const double* __restrict__ samples,
                                                     int64_t n, float* __restrict__ x, float* __restrict__ t,
                                                     DevStatus* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lnr = samples[2 * i], lnu = samples[2 * i + 1];
  double lp = 0.0, lc = 0.0;
  int64_t cell;
  if (eos_table_ln(p, lnr, lnu, lp, lc, cell)) latch_error(status, SPH_E_EOS_DOMAIN, (int)i);
  x[2 * i] = (float)((lnr - nm.in_lo[0]) * nm.in_sc[0] - 1.0);
  x[2 * i + 1] = (float)((lnu - nm.in_lo[1]) * nm.in_sc[1] - 1.0);
  t[2 * i] = (float)((lp - nm.out_c[0]) / nm.out_sc[0]);
  t[2 * i + 1] = (float)((lc - nm.out_c[1]) / nm.out_sc[1]);
}

// squared error of the network on normalised pairs (holdout loss), one partial per block
__global__ __launch_bounds__(64) void k_mlp_sqerr(MlpView M, const float* __restrict__ x, const float* __restrict__ t,
                                                  int64_t n, float* __restrict__ part) {
  float acc = 0.f;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
    const int64_t i = base + threadIdx.x;
    const bool ok = i < n;
    float y0 = 0.f, y1 = 0.f;
    mlp_wave(M, ok ? x[2 * i] : 0.f, ok ? x[2 * i + 1] : 0.f, y0, y1);
    if (ok) {
      const float e0 = y0 - t[2 * i], e1 = y1 - t[2 * i + 1];
      acc += 0.5f * (e0 * e0 + e1 * e1);
    }
  }
  acc = wave_sum_f(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// network outputs in physical units: ln P, ln c_s^2 at (ln rho, ln u)
__global__ __launch_bounds__(64) void k_mlp_eval(MlpView M, const double* __restrict__ lnr,
                                                 const double* __restrict__ lnu, int64_t n, double* __restrict__ lp,
                                                 double* __restrict__ lc) {
  const MlpNorm& nm = M.norm;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
    const int64_t i = base + threadIdx.x;
    const bool ok = i < n;
    const float x0 = ok ? (float)((lnr[i] - nm.in_lo[0]) * nm.in_sc[0] - 1.0) : 0.f;
    const float x1 = ok ? (float)((lnu[i] - nm.in_lo[1]) * nm.in_sc[1] - 1.0) : 0.f;
    float y0 = 0.f, y1 = 0.f;
    mlp_wave(M, x0, x1, y0, y1);
    if (ok) {
      lp[i] = (double)y0 * nm.out_sc[0] + nm.out_c[0];
      lc[i] = (double)y1 * nm.out_sc[1] + nm.out_c[1];
    }
  }
}

// Least-squares readout: with the hidden layers fixed, the outputs are linear in (W4, b4), so the
// readout that minimises the squared error over the training samples solves the normal equations
// (G + lambda I) [W4 b4]^T = H^T T, G = H^T H, H the samples' last hidden layer (as the kernels
// compute it) extended by a constant 1.  Per block, thread f accumulates row f of G over the
// block's samples in FP64 (columns 0..63, then the constant column, then the two right-hand
// sides): 67 values per row, 64 rows, and the sums of the targets.
constexpr int kGramRow = 67, kGramStride = 64 * kGramRow + 2;
__global__ __launch_bounds__(64) void k_mlp_gram(MlpView M, const float* __restrict__ x, const float* __restrict__ t,
                                                 int64_t n, double* __restrict__ part) {
  __shared__ float H[64][MLP_H + 4];
  __shared__ float T[64][2];
  const int l = threadIdx.x, q = l >> 4, r = l & 15;
  double acc[kGramRow];
#pragma unroll
  for (int g = 0; g < kGramRow; ++g) acc[g] = 0.0;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
    const int64_t i = base + l;
    const bool ok = i < n;
    mlp_wave_hidden(M, ok ? x[2 * i] : 0.f, ok ? x[2 * i + 1] : 0.f,
                    [&](int nt, int mt, const float h3[4], const MlpP&) {
                      const bool oks = base + 16 * nt + r < n;
#pragma unroll
                      for (int j = 0; j < 4; ++j) H[16 * nt + r][16 * mt + 4 * q + j] = oks ? h3[j] : 0.f;
                    });
    T[l][0] = ok ? t[2 * i] : 0.f;
    T[l][1] = ok ? t[2 * i + 1] : 0.f;
    __syncthreads();
    const int ns = n - base < 64 ? (int)(n - base) : 64;
    for (int sI = 0; sI < ns; ++sI) {
      const double hf = (double)H[sI][l];
#pragma unroll
      for (int g = 0; g < MLP_H; ++g) acc[g] += hf * (double)H[sI][g];
      const double t0 = (double)T[sI][0], t1 = (double)T[sI][1];
      acc[MLP_H] += hf;
      acc[MLP_H + 1] += hf * t0;
      acc[MLP_H + 2] += hf * t1;
      s0 += t0;
      s1 += t1;
    }
    __syncthreads();
  }
  double* o = part + (int64_t)blockIdx.x * kGramStride;
#pragma unroll
  for (int g = 0; g < kGramRow; ++g) o[l * kGramRow + g] = acc[g];
  if (l == 0) {
    o[64 * kGramRow] = s0;
    o[64 * kGramRow + 1] = s1;
  }
}

// Sums the block partials in block order (deterministic), adds lambda = ridge * mean diagonal,
// solves by Cholesky (one workgroup, in LDS) and writes W4, b4 into the master weights and the
// copy the kernels use (both FP32).
__global__ __launch_bounds__(256) void k_mlp_solve(const double* __restrict__ part, int nblk, int64_t n, double ridge,
                                                   float* __restrict__ w, float* __restrict__ wr) {
  constexpr int N = MLP_H + 1;
  __shared__ double A[N][N + 1];
  __shared__ double B[N][2];
  __shared__ double X[N][2];
  const int tid = threadIdx.x;
  for (int e = tid; e < kGramStride; e += blockDim.x) {
    double v = 0.0;
    for (int b = 0; b < nblk; ++b) v += part[(int64_t)b * kGramStride + e];
    if (e < 64 * kGramRow) {
      const int f = e / kGramRow, g = e % kGramRow;
      if (g < MLP_H) A[f][g] = v;
      else if (g == MLP_H) { A[f][MLP_H] = v; A[MLP_H][f] = v; }
      else B[f][g - MLP_H - 1] = v;
    } else {
      B[MLP_H][e - 64 * kGramRow] = v;
    }
  }
  if (tid == 0) A[MLP_H][MLP_H] = (double)n;
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < N; ++i) tr += A[i][i];
    const double lam = ridge * tr / N;
    for (int i = 0; i < N; ++i) A[i][i] += lam;
  }
  __syncthreads();
  for (int k = 0; k < N; ++k) {   // A = L L^T, L in the lower triangle
    if (tid == 0) A[k][k] = sqrt(fmax(A[k][k], 1e-300));
    __syncthreads();
    for (int i = k + 1 + tid; i < N; i += blockDim.x) A[i][k] /= A[k][k];
    __syncthreads();
    const int m = N - k - 1;
    for (int idx = tid; idx < m * m; idx += blockDim.x) {
      const int i = k + 1 + idx / m, j = k + 1 + idx % m;
      if (j <= i) A[i][j] -= A[i][k] * A[j][k];
    }
    __syncthreads();
  }
  if (tid < 2) {
    const int o = tid;
    for (int i = 0; i < N; ++i) {   // L y = b
      double v = B[i][o];
      for (int j = 0; j < i; ++j) v -= A[i][j] * X[j][o];
      X[i][o] = v / A[i][i];
    }
    for (int i = N - 1; i >= 0; --i) {   // L^T x = y
      double v = X[i][o];
      for (int j = i + 1; j < N; ++j) v -= A[j][i] * X[j][o];
      X[i][o] = v / A[i][i];
    }
    for (int f = 0; f < MLP_H; ++f) {
      const float v = (float)X[f][o];
      w[MLP_OW4 + MLP_H * o + f] = v;
      wr[MLP_OW4 + MLP_H * o + f] = v;
    }
    w[MLP_OB4 + o] = (float)X[MLP_H][o];
    wr[MLP_OB4 + o] = (float)X[MLP_H][o];
  }
}

// Interior test points of a table cell: four per cell from a counter-based generator (splitmix64
// of the cell index and the point number), fractions in [0, 1).
__device__ __forceinline__ double cell_uniform(uint64_t cell, int k) {
  uint64_t z = cell * 16u + (uint64_t)k + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// Trust mask: a table cell is trusted when the network's P and c_s^2 are within relative tolerance
// tol / 2 (a margin of 2 for the points in between) of the table at 13 points of the cell: its four
// nodes, the four edge midpoints, the centre and four seeded interior points.
constexpr int kTrustPoints = 13;
// Only cells inside the network's domain dom = (lnr_lo, lnr_hi, lnu_lo, lnu_hi) are tested; the
// others stay untrusted.
struct Domain {
  double d[4];
};
__global__ __launch_bounds__(64) void k_mlp_trust(MlpView M, sph_params p, Domain D, double tol,
                                                  uint8_t* __restrict__ mask, unsigned long long* count) {
  const MlpNorm& nm = M.norm;
  const int nu1 = p.tab_nu - 1;
  const int64_t ncell = (int64_t)(p.tab_nr - 1) * nu1;
  unsigned long long good = 0;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < ncell; base += (int64_t)gridDim.x * 64) {
    const int64_t c = base + threadIdx.x;
    const bool ok = c < ncell;
    const int i = ok ? (int)(c / nu1) : 0, j = ok ? (int)(c % nu1) : 0;
    const double e = 1e-9;   // a cell whose edge lies on the domain's edge is inside
    const bool inside = p.tab_lnr0 + i * p.tab_dlnr >= D.d[0] - e * p.tab_dlnr &&
                        p.tab_lnr0 + (i + 1) * p.tab_dlnr <= D.d[1] + e * p.tab_dlnr &&
                        p.tab_lnu0 + j * p.tab_dlnu >= D.d[2] - e * p.tab_dlnu &&
                        p.tab_lnu0 + (j + 1) * p.tab_dlnu <= D.d[3] + e * p.tab_dlnu;
    double err = 0.0;
    bool finite = inside;
    const double fa9[9] = {0.0, 1.0, 0.0, 1.0, 0.5, 0.5, 0.0, 1.0, 0.5}, fb9[9] = {0.0, 0.0, 1.0, 1.0, 0.0, 1.0, 0.5, 0.5, 0.5};
#pragma unroll 1
    for (int k = 0; k < kTrustPoints; ++k) {
      const double fak = k < 9 ? fa9[k] : cell_uniform((uint64_t)c, 2 * k);
      const double fbk = k < 9 ? fb9[k] : cell_uniform((uint64_t)c, 2 * k + 1);
      const double lnr = p.tab_lnr0 + ((double)i + fak) * p.tab_dlnr;
      const double lnu = p.tab_lnu0 + ((double)j + fbk) * p.tab_dlnu;
      float y0 = 0.f, y1 = 0.f;
      mlp_wave(M, (float)((lnr - nm.in_lo[0]) * nm.in_sc[0] - 1.0), (float)((lnu - nm.in_lo[1]) * nm.in_sc[1] - 1.0),
               y0, y1);
      const int64_t o = (int64_t)i * p.tab_nu + j;
      double tp, tc;
      finite = finite && table_bilinear(p.tab_lnP, o, p.tab_nu, fak, fbk, tp) &&
               table_bilinear(p.tab_lncs2, o, p.tab_nu, fak, fbk, tc);
      if (finite) {
        const double ep = fabs(expm1((double)y0 * nm.out_sc[0] + nm.out_c[0] - tp));
        const double ec = fabs(expm1((double)y1 * nm.out_sc[1] + nm.out_c[1] - tc));
        err = fmax(err, fmax(ep, ec));
      }
    }
    if (ok) {
      const bool t = finite && err <= 0.5 * tol;
      mask[c] = t ? 1 : 0;
      good += t ? 1ull : 0ull;
    }
  }
  for (int off = 32; off > 0; off >>= 1) good += __shfl_xor(good, off, 64);
  if (threadIdx.x == 0) atomicAdd(count, good);
}

template <typename T>
sph_status dalloc(T** p, size_t count) {
  *p = nullptr;
  if (hipMalloc((void**)p, sizeof(T) * count) != hipSuccess) {
    *p = nullptr;
    return SPH_E_OOM;
  }
  return SPH_OK;
}

sph_status mlp_alloc(sph_ctx* c) {
  if (c->mlp) return SPH_OK;
  MlpState* s = new MlpState();
  c->mlp = s;
  sph_status e;
  if ((e = dalloc(&s->w, MLP_NPARAM)) || (e = dalloc(&s->wr, MLP_NPARAM)) || (e = dalloc(&s->m, MLP_NPARAM)) ||
      (e = dalloc(&s->v, MLP_NPARAM)) || (e = dalloc(&s->pack, 4 * 1024)) ||
      (e = dalloc(&s->gpart, (size_t)kMaxBlocks * MLP_NPARAM)) || (e = dalloc(&s->lpart, kMaxBlocks)) ||
      (e = dalloc(&s->gsum, MLP_NPARAM)) || (e = dalloc(&s->scal, 4)))
    return e;
  return SPH_OK;
}

bool table_ok(const sph_ctx* c) {
  const sph_params& p = c->p;
  return p.tab_lnP && p.tab_lncs2 && p.tab_nr >= 2 && p.tab_nu >= 2;
}

// The network's domain: the one set by sph_mlp_set_domain, else the table's box.
Domain domain_of(const sph_ctx* c) {
  const sph_params& p = c->p;
  const MlpState* s = c->mlp;
  if (s && s->dom_set) return Domain{{s->dom[0], s->dom[1], s->dom[2], s->dom[3]}};
  return Domain{{p.tab_lnr0, p.tab_lnr0 + (p.tab_nr - 1) * p.tab_dlnr, p.tab_lnu0, p.tab_lnu0 + (p.tab_nu - 1) * p.tab_dlnu}};
}

// input normalisation from the domain, output normalisation from the value range of the table
// nodes that cover it
sph_status mlp_norm(sph_ctx* c) {
  MlpState* s = c->mlp;
  if (s->norm_set) return SPH_OK;
  const sph_params& p = c->p;
  const Domain D = domain_of(c);
  auto node = [](double v, double v0, double dv, int nmax, bool up) {
    const double f = (v - v0) / dv;
    int i = up ? (int)ceil(f - 1e-9) : (int)floor(f + 1e-9);
    return i < 0 ? 0 : (i > nmax ? nmax : i);
  };
  const int i0 = node(D.d[0], p.tab_lnr0, p.tab_dlnr, p.tab_nr - 1, false);
  const int i1 = node(D.d[1], p.tab_lnr0, p.tab_dlnr, p.tab_nr - 1, true);
  const int j0 = node(D.d[2], p.tab_lnu0, p.tab_dlnu, p.tab_nu - 1, false);
  const int j1 = node(D.d[3], p.tab_lnu0, p.tab_dlnu, p.tab_nu - 1, true);
  hipLaunchKernelGGL(k_table_range, dim3(1), dim3(256), 0, c->stream, p.tab_lnP, p.tab_lncs2, i0, i1, j0, j1, p.tab_nu,
                     s->scal);
  float r[4];
  HIP_TRY(hipMemcpyAsync(r, s->scal, sizeof(r), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  MlpNorm& nm = s->norm;
  nm.in_lo[0] = (float)D.d[0];
  nm.in_lo[1] = (float)D.d[2];
  nm.in_sc[0] = (float)(2.0 / (D.d[1] - D.d[0]));
  nm.in_sc[1] = (float)(2.0 / (D.d[3] - D.d[2]));
  nm.out_c[0] = r[0];
  nm.out_c[1] = r[1];
  nm.out_sc[0] = r[2] > 0.f ? r[2] : 1.f;
  nm.out_sc[1] = r[3] > 0.f ? r[3] : 1.f;
  s->norm_set = true;
  return SPH_OK;
}

MlpView view_of(const MlpState* s) {
  MlpView v;
  v.wr = s->wr;
  v.wa2 = s->pack;
  v.wa3 = s->pack + 1024;
  v.wt2 = s->pack + 2048;
  v.wt3 = s->pack + 3072;
  v.trust = s->trust;
  v.norm = s->norm;
  return v;
}

sph_status launch_grad(sph_ctx* c, const float* x, const float* t, int64_t n, int64_t off, int batch) {
  GradArgs G;
  G.M = view_of(c->mlp);
  G.x = x;
  G.t = t;
  G.off = off;
  G.n = n;
  G.batch = batch;
  G.gpart = c->mlp->gpart;
  G.lpart = c->mlp->lpart;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mlp_grad<kGradSamples>), dim3(batch / kGradSamples), dim3(64), 0, c->stream, G);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

}  // namespace

bool mlp_view(const sph_ctx* c, MlpView* v) {
  if (!c->mlp || !c->mlp->loaded || !c->mlp->norm_set) return false;
  *v = view_of(c->mlp);
  return true;
}

int64_t mlp_trusted_cells(const sph_ctx* c) {
  return (c->mlp && c->mlp->trust) ? c->mlp->trust_cells : 0;
}

void mlp_free(sph_ctx* c) {
  MlpState* s = c->mlp;
  if (!s) return;
  void* bufs[] = {s->w, s->wr, s->m, s->v, s->pack, s->gpart, s->lpart, s->gsum, s->scal, s->trust, s->served, s->gpart64};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete s;
  c->mlp = nullptr;
}

extern "C" {

sph_status sph_mlp_set_params(sph_ctx* c, const float* params) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!params) return note(c, SPH_E_ARG, "params is NULL");
  if (!table_ok(c)) return note(c, SPH_E_ARG, "the network needs the context's EoS table");
  sph_status e;
  if ((e = mlp_alloc(c)) || (e = mlp_norm(c))) return e;
  MlpState* s = c->mlp;
  HIP_TRY(hipMemcpyAsync(s->w, params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(s->m, 0, sizeof(float) * MLP_NPARAM, c->stream));
  HIP_TRY(hipMemsetAsync(s->v, 0, sizeof(float) * MLP_NPARAM, c->stream));
  hipLaunchKernelGGL(k_round, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, c->stream, s->w, s->wr, MLP_NPARAM);
  hipLaunchKernelGGL(k_mlp_pack, dim3(16), dim3(256), 0, c->stream, s->wr, s->pack);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (s->trust) {   // a mask belongs to the weights it was built for
    (void)hipFree(s->trust);
    s->trust = nullptr;
    s->trust_cells = 0;
  }
  s->step = 0;
  s->loaded = true;
  ++c->graph_epoch;
  return SPH_OK;
}

sph_status sph_mlp_load(sph_ctx* c, const uint16_t* bf16_weights) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!bf16_weights) return note(c, SPH_E_ARG, "bf16_weights is NULL");
  std::vector<float> w(MLP_NPARAM);
  for (int k = 0; k < MLP_NPARAM; ++k) {   // a BF16 value is the upper half of an FP32 one
    const uint32_t b = (uint32_t)bf16_weights[k] << 16;
    memcpy(&w[k], &b, sizeof(float));
  }
  return sph_mlp_set_params(c, w.data());
}

sph_status sph_mlp_get_params(sph_ctx* c, float* params, int32_t rounded) {
  if (!c || !params || !c->mlp || !c->mlp->loaded) return SPH_E_ARG;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(params, rounded ? c->mlp->wr : c->mlp->w, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
  return SPH_OK;
}

sph_status sph_mlp_get_norm(sph_ctx* c, float* norm8) {
  if (!c || !norm8 || !c->mlp || !c->mlp->norm_set) return SPH_E_ARG;
  const MlpNorm& nm = c->mlp->norm;
  const float v[8] = {nm.in_lo[0], nm.in_lo[1], nm.in_sc[0], nm.in_sc[1], nm.out_c[0], nm.out_c[1], nm.out_sc[0],
                      nm.out_sc[1]};
  memcpy(norm8, v, sizeof(v));
  return SPH_OK;
}

sph_status sph_mlp_grad(sph_ctx* c, const float* x, const float* t, int64_t n, float* grad, double* loss) {
  if (!c || !x || !t || !grad || !c->mlp || !c->mlp->loaded) return SPH_E_ARG;
  if (n < 64 || n % 64 || n > kMaxBatch) return SPH_E_ARG;
  MlpState* s = c->mlp;
  sph_status e = launch_grad(c, x, t, n, 0, (int)n);
  if (e) return e;
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, c->stream, s->w, s->wr, s->m, s->v,
                     s->gpart, s->lpart, (int)(n / kGradSamples), 0.f, 1.f, 1.f, s->gsum, s->scal);
  HIP_TRY(hipGetLastError());
  float l = 0.f;
  HIP_TRY(hipMemcpyAsync(grad, s->gsum, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&l, s->scal, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (loss) *loss = l;
  return SPH_OK;
}

sph_status sph_mlp_train(sph_ctx* c, const double* samples, int64_t n, int64_t n_holdout, int32_t epochs,
                         int32_t batch, float lr, float* history) {
  if (!c || !samples || !c->mlp || !c->mlp->loaded || !table_ok(c)) return SPH_E_ARG;
  if (n_holdout < 0 || n - n_holdout < batch || epochs < 0 || batch < 64 || batch % 64 || batch > kMaxBatch ||
      !(lr > 0.f))
    return SPH_E_ARG;
  MlpState* s = c->mlp;
  float *x = nullptr, *t = nullptr, *part = nullptr;
  sph_status e = SPH_OK;
  if ((e = dalloc(&x, (size_t)2 * n)) || (e = dalloc(&t, (size_t)2 * n)) || (e = dalloc(&part, 1024))) {
    if (x) (void)hipFree(x);
    if (t) (void)hipFree(t);
    return e;
  }
  hipLaunchKernelGGL(k_mlp_targets, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, c->p, s->norm, samples, n, x, t,
                     c->status);
  const int64_t ntrain = n - n_holdout;
  const int64_t per_epoch = ntrain / batch;
  const int64_t total = per_epoch * epochs;
  const int nblk = batch / kGradSamples;
  const unsigned hold_blocks = n_holdout > 0 ? (unsigned)((n_holdout + 63) / 64 < 1024 ? (n_holdout + 63) / 64 : 1024) : 0;
  for (int32_t ep = 0; ep < epochs && !e; ++ep) {
    for (int64_t k = 0; k < per_epoch && !e; ++k) {
      const int64_t it = (int64_t)ep * per_epoch + k;
      const double lr_t = 0.5 * lr * (1.0 + cos(M_PI * (double)it / (double)total));   // cosine schedule
      ++s->step;
      const float bc1 = (float)(1.0 - pow(0.9, (double)s->step)), bc2 = (float)(1.0 - pow(0.999, (double)s->step));
      // samples rotate through the training set; each epoch starts at a different offset
      const int64_t off = (k * batch + (int64_t)ep * 7919) % ntrain;
      if ((e = launch_grad(c, x, t, ntrain, off, batch))) break;
      hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, c->stream, s->w, s->wr, s->m,
                         s->v, s->gpart, s->lpart, nblk, (float)lr_t, bc1, bc2, (float*)nullptr, s->scal);
      hipLaunchKernelGGL(k_mlp_pack, dim3(16), dim3(256), 0, c->stream, s->wr, s->pack);
    }
    if (e) break;
    float hl = 0.f;
    if (n_holdout > 0) {
      hipLaunchKernelGGL(k_mlp_sqerr, dim3(hold_blocks), dim3(64), 0, c->stream, view_of(s), x + 2 * ntrain,
                         t + 2 * ntrain, n_holdout, part);
      std::vector<float> hp(hold_blocks);
      if (hipMemcpyAsync(hp.data(), part, sizeof(float) * hold_blocks, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        e = SPH_E_HIP;
      float tl = 0.f;
      if (!e && hipMemcpyAsync(&tl, s->scal, sizeof(float), hipMemcpyDeviceToHost, c->stream) != hipSuccess) e = SPH_E_HIP;
      if (!e && hipStreamSynchronize(c->stream) != hipSuccess) e = SPH_E_HIP;
      for (float v : hp) hl += v;
      hl /= (float)n_holdout;
      if (history) {
        history[2 * ep] = tl;
        history[2 * ep + 1] = hl;
      }
    }
  }
  if (!e && hipStreamSynchronize(c->stream) != hipSuccess) e = SPH_E_HIP;
  (void)hipFree(x);
  (void)hipFree(t);
  (void)hipFree(part);
  if (s->trust) {   // the weights changed
    (void)hipFree(s->trust);
    s->trust = nullptr;
    s->trust_cells = 0;
  }
  ++c->graph_epoch;
  return e;
}

sph_status sph_mlp_set_domain(sph_ctx* c, double lnrho_lo, double lnrho_hi, double lnu_lo, double lnu_hi) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!table_ok(c)) return note(c, SPH_E_ARG, "the network needs the context's EoS table");
  const sph_params& p = c->p;
  const double r1 = p.tab_lnr0 + (p.tab_nr - 1) * p.tab_dlnr, u1 = p.tab_lnu0 + (p.tab_nu - 1) * p.tab_dlnu;
  if (!(lnrho_lo < lnrho_hi) || !(lnu_lo < lnu_hi) || lnrho_lo < p.tab_lnr0 || lnrho_hi > r1 || lnu_lo < p.tab_lnu0 ||
      lnu_hi > u1)
    return note(c, SPH_E_ARG, "domain [%g, %g] x [%g, %g] is empty or leaves the table's box [%g, %g] x [%g, %g]",
                lnrho_lo, lnrho_hi, lnu_lo, lnu_hi, p.tab_lnr0, r1, p.tab_lnu0, u1);
  sph_status e;
  if ((e = mlp_alloc(c))) return e;
  MlpState* s = c->mlp;
  s->dom_set = true;
  s->dom[0] = lnrho_lo;
  s->dom[1] = lnrho_hi;
  s->dom[2] = lnu_lo;
  s->dom[3] = lnu_hi;
  s->norm_set = false;
  if ((e = mlp_norm(c))) return e;
  if (s->trust) {   // a mask belongs to the normalisation it was built with
    (void)hipFree(s->trust);
    s->trust = nullptr;
    s->trust_cells = 0;
  }
  ++c->graph_epoch;
  return SPH_OK;
}

sph_status sph_mlp_fit_readout(sph_ctx* c, const double* samples, int64_t n, int64_t n_holdout, double ridge,
                               double* holdout_loss) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!samples || !c->mlp || !c->mlp->loaded || !table_ok(c))
    return note(c, SPH_E_ARG, "the fit needs samples, a loaded network and the EoS table");
  if (n_holdout < 0 || n - n_holdout < 64 || !(ridge >= 0.0))
    return note(c, SPH_E_ARG, "n = %lld, n_holdout = %lld (at least 64 fit samples), ridge = %g", (long long)n,
                (long long)n_holdout, ridge);
  MlpState* s = c->mlp;
  constexpr int kGramBlocks = 1024;
  if (!s->gpart64 && hipMalloc((void**)&s->gpart64, sizeof(double) * (size_t)kGramBlocks * kGramStride) != hipSuccess) {
    s->gpart64 = nullptr;
    return note(c, SPH_E_OOM, "readout fit partials");
  }
  float *x = nullptr, *t = nullptr, *part = nullptr;
  sph_status e = SPH_OK;
  if ((e = dalloc(&x, (size_t)2 * n)) || (e = dalloc(&t, (size_t)2 * n)) || (e = dalloc(&part, 1024))) {
    if (x) (void)hipFree(x);
    if (t) (void)hipFree(t);
    return note(c, e, "readout fit scratch");
  }
  hipLaunchKernelGGL(k_mlp_targets, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, c->p, s->norm, samples, n, x, t,
                     c->status);
  const int64_t nfit = n - n_holdout;
  const unsigned nb = (unsigned)((nfit + 63) / 64 < kGramBlocks ? (nfit + 63) / 64 : kGramBlocks);
  hipLaunchKernelGGL(k_mlp_gram, dim3(nb), dim3(64), 0, c->stream, view_of(s), x, t, nfit, s->gpart64);
  hipLaunchKernelGGL(k_mlp_solve, dim3(1), dim3(256), 0, c->stream, s->gpart64, (int)nb, nfit, ridge, s->w, s->wr);
  if (hipGetLastError() != hipSuccess) e = SPH_E_HIP;
  float hl = 0.f;
  if (!e && n_holdout > 0) {
    const unsigned hb = (unsigned)((n_holdout + 63) / 64 < 1024 ? (n_holdout + 63) / 64 : 1024);
    hipLaunchKernelGGL(k_mlp_sqerr, dim3(hb), dim3(64), 0, c->stream, view_of(s), x + 2 * nfit, t + 2 * nfit,
                       n_holdout, part);
    std::vector<float> hp(hb);
    if (hipMemcpyAsync(hp.data(), part, sizeof(float) * hb, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      e = SPH_E_HIP;
    if (!e && hipStreamSynchronize(c->stream) != hipSuccess) e = SPH_E_HIP;
    for (float v : hp) hl += v;
    hl /= (float)n_holdout;
  }
  if (!e && hipStreamSynchronize(c->stream) != hipSuccess) e = SPH_E_HIP;
  (void)hipFree(x);
  (void)hipFree(t);
  (void)hipFree(part);
  if (s->trust) {   // the weights changed
    (void)hipFree(s->trust);
    s->trust = nullptr;
    s->trust_cells = 0;
  }
  ++c->graph_epoch;
  if (holdout_loss) *holdout_loss = hl;
  return e ? note(c, e, "readout fit on the device") : SPH_OK;
}

sph_status sph_mlp_eval(sph_ctx* c, const double* lnrho, const double* lnu, int64_t n, double* lnP, double* lncs2) {
  if (!c || n < 0 || (n > 0 && (!lnrho || !lnu || !lnP || !lncs2)) || !c->mlp || !c->mlp->loaded ||
      !c->mlp->norm_set)
    return SPH_E_ARG;
  if (n == 0) return SPH_OK;
  const unsigned nb = (unsigned)((n + 63) / 64 < 65536 ? (n + 63) / 64 : 65536);
  hipLaunchKernelGGL(k_mlp_eval, dim3(nb), dim3(64), 0, c->stream, view_of(c->mlp), lnrho, lnu, n, lnP, lncs2);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

// Particles whose (rho, u) lies in a trusted table cell (those the EoS network serves).
__global__ __launch_bounds__(256) void k_mlp_served(const double* __restrict__ rho, const double* __restrict__ u,
                                                    int64_t n, sph_params p, const uint8_t* __restrict__ trust,
                                                    unsigned long long* __restrict__ count) {
  unsigned long long k = 0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
    if (!(rho[a] > 0.0) || !(u[a] > 0.0)) continue;
    const double fr = (log(rho[a]) - p.tab_lnr0) / p.tab_dlnr, fu = (log(u[a]) - p.tab_lnu0) / p.tab_dlnu;
    if (!(fr >= 0.0) || !(fu >= 0.0) || fr > (double)(p.tab_nr - 1) || fu > (double)(p.tab_nu - 1)) continue;
    int i = (int)floor(fr), j = (int)floor(fu);
    i = i > p.tab_nr - 2 ? p.tab_nr - 2 : i;
    j = j > p.tab_nu - 2 ? p.tab_nu - 2 : j;
    k += trust[(int64_t)i * (p.tab_nu - 1) + j] ? 1ull : 0ull;
  }
  for (int off = 32; off > 0; off >>= 1) k += __shfl_xor(k, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(count, k);
}

sph_status sph_mlp_build_trust_mask(sph_ctx* c, double tol, int64_t* trusted_cells) {
  if (!c || !(tol >= 0.0) || !c->mlp || !c->mlp->loaded || !table_ok(c)) return SPH_E_ARG;
  MlpState* s = c->mlp;
  const int64_t ncell = (int64_t)(c->p.tab_nr - 1) * (c->p.tab_nu - 1);
  if (!s->trust && hipMalloc((void**)&s->trust, (size_t)ncell) != hipSuccess) {
    s->trust = nullptr;
    return SPH_E_OOM;
  }
  unsigned long long* cnt = nullptr;
  if (hipMalloc((void**)&cnt, sizeof(unsigned long long)) != hipSuccess) return SPH_E_OOM;
  sph_status e = SPH_OK;
  unsigned long long h = 0;
  if (hipMemcpyAsync(cnt, &h, sizeof(h), hipMemcpyHostToDevice, c->stream) != hipSuccess) e = SPH_E_HIP;
  if (!e) {
    MlpView v = view_of(s);
    v.trust = nullptr;
    const unsigned nb = (unsigned)((ncell + 63) / 64 < 65536 ? (ncell + 63) / 64 : 65536);
    hipLaunchKernelGGL(k_mlp_trust, dim3(nb), dim3(64), 0, c->stream, v, c->p, domain_of(c), tol, s->trust, cnt);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      e = SPH_E_HIP;
  }
  (void)hipFree(cnt);
  s->trust_cells = (int64_t)h;
  ++c->graph_epoch;
  if (trusted_cells) *trusted_cells = (int64_t)h;
  return e;
}

}  // extern "C"

extern "C" sph_status sph_mlp_count_served(sph_ctx* c, const sph_state* st, int64_t* served) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!st || !served) return note(c, SPH_E_ARG, "state and served must not be NULL");
  *served = 0;
  if (!c->mlp || !c->mlp->trust || st->n <= 0) return SPH_OK;
  if (!st->rho || !st->u) return note(c, SPH_E_ARG, "the count needs rho and u");
  unsigned long long* cnt = c->mlp->served;
  if (!cnt && hipMalloc((void**)&c->mlp->served, sizeof(unsigned long long)) != hipSuccess) {
    c->mlp->served = nullptr;
    return note(c, SPH_E_OOM, "served counter");
  }
  cnt = c->mlp->served;
  unsigned long long h = 0;
  HIP_TRY(hipMemcpyAsync(cnt, &h, sizeof(h), hipMemcpyHostToDevice, c->stream));
  unsigned nb = grid_for(st->n, 256);
  nb = nb < 1024 ? nb : 1024;
  hipLaunchKernelGGL(k_mlp_served, dim3(nb), dim3(256), 0, c->stream, st->rho, st->u, st->n, c->p, c->mlp->trust, cnt);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *served = (int64_t)h;
  return SPH_OK;
}
