// EoS surrogate network: 2 -> 64 -> 64 -> 64 -> 2 with SiLU activations, mapping normalised
// (ln rho, ln u) to normalised (ln P, ln c_s^2).  The two 64x64 layers run on the matrix cores
// (v_mfma_f32_16x16x16_bf16) with BF16 weights (the BF16-rounded values of FP32 master weights)
// and FP32 accumulation; the 2-wide input and output layers, the biases and the activations run
// on the vector ALUs in FP32.
//
// MFMA operand layouts (16x16x16, wave64; lane l, q = l / 16, r = l % 16, j = 0..3):
//   A (M x K):  lane holds A[r][4q + j]      B (K x N):  lane holds B[4q + j][r]
//   C (M x N):  lane holds C[4q + j][r]
// A layer is computed transposed, H_next^T (features x samples) = W (out x in) * H^T (in x
// samples): the weights are the A operand and a C tile, after bias and activation, is exactly
// the B operand of the next layer, so activations never leave the registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MLP_H 64
#define MLP_NPARAM 8642
// offsets of the parameter blocks in the flat array (W[out][in] row-major)
#define MLP_OW1 0
#define MLP_OB1 128
#define MLP_OW2 192
#define MLP_OB2 4288
#define MLP_OW3 4352
#define MLP_OB3 8448
#define MLP_OW4 8512
#define MLP_OB4 8640

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// x_n = (v - in_lo) * in_sc - 1 for v = ln rho, ln u;  v = y_n * out_sc + out_c for ln P, ln c_s^2
struct MlpNorm {
  float in_lo[2], in_sc[2], out_c[2], out_sc[2];
};

// Read-only view of the network for the kernels.
struct MlpView {
  const float* wr;     // the parameters as used: W2, W3 rounded to BF16, the rest FP32 (flat layout)
  const uint2* wa2;    // W2 packed as MFMA A operands: [(mt * 4 + kk) * 64 + lane] = 4 BF16
  const uint2* wa3;    // W3 likewise
  const uint2* wt2;    // W2^T packed as A operands (backward pass)
  const uint2* wt3;
  const uint8_t* trust;  // per EoS-table cell: 1 where the network is within tolerance, may be null
  MlpNorm norm;
};

__device__ __forceinline__ uint32_t bf16_bits(float f) {   // round to nearest even
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float(bf16_bits(f) << 16); }
// Two FP32 values rounded to BF16 (nearest even) by one hardware conversion, a in the low half.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
// the FP32 values of the low and the high BF16 of a packed pair
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ bf16x4 as_bf16x4(uint2 u) { return __builtin_bit_cast(bf16x4, u); }
__device__ __forceinline__ bf16x4 pack_bf16(float a, float b, float c, float d) {
  return as_bf16x4(make_uint2(pk_bf16(a, b), pk_bf16(c, d)));
}
__device__ __forceinline__ float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
  const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}
__device__ __forceinline__ f32x4 mfma_bf16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// The BF16 parameters: the two 64x64 matrix-core layers (W2, W3).  The 2 -> 64 input layer, the
// 64 -> 2 readout and the biases run on the vector ALUs and stay FP32.
__host__ __device__ __forceinline__ bool mlp_bf16_param(int p) {
  return (p >= MLP_OW2 && p < MLP_OB2) || (p >= MLP_OW3 && p < MLP_OB3);
}

// An activation tile as the B operand of a BF16 product, split in two BF16 parts: hi = bf16(h),
// lo = bf16(h - hi).  W (hi + lo) carries h to about 2^-17, so the products see the weights'
// BF16 values but not a BF16 rounding of the activations.
__device__ __forceinline__ void split_bf16(const float h[4], bf16x4& hi, bf16x4& lo) {
  const uint32_t w0 = pk_bf16(h[0], h[1]), w1 = pk_bf16(h[2], h[3]);
  hi = as_bf16x4(make_uint2(w0, w1));
  lo = as_bf16x4(make_uint2(pk_bf16(h[0] - bf16_lo(w0), h[1] - bf16_hi(w0)),
                            pk_bf16(h[2] - bf16_lo(w1), h[3] - bf16_hi(w1))));
}

// Where a wave finds the parameters: the FP32 blocks of the input layer, the biases and the
// readout, and the MFMA packs of W2, W3.
struct MlpP {
  const float *w1, *b1, *b2, *b3, *w4, *b4;
  const uint2 *wa2, *wa3;
};

// The network up to its last hidden layer for the 64 inputs held one per lane (x0, x1
// normalised).  Every lane of the wave must call it (matrix instructions).  For each block of 16
// inputs nt it calls out(nt, mt, h, P) with the lane's part of the last hidden layer: h[j] is
// feature 16 mt + 4 q + j of input 16 nt + r.  ptrs() gives the parameters, through pointers the
// compiler does not hoist loads out of the loop over nt (the weights are the same for every nt;
// hoisted, their loads would occupy ~180 registers across it).
template <typename Ptrs, typename Out>
__device__ __forceinline__ void mlp_wave_layers(Ptrs&& ptrs, float x0, float x1, Out&& out) {
  const int l = threadIdx.x & 63, q = l >> 4, r = l & 15;
#pragma unroll 1
  for (int nt = 0; nt < 4; ++nt) {
    const MlpP P = ptrs();
    const int pp = 16 * nt + r;   // the input this lane's B-operand column belongs to
    const float a0 = __shfl(x0, pp, 64), a1 = __shfl(x1, pp, 64);
    bf16x4 h1[4], l1[4];
    // scheduling barriers between the stages bound the weight loads in flight (registers)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      __builtin_amdgcn_sched_barrier(0);
      float h[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int f = 16 * kk + 4 * q + j;
        h[j] = silu_f(P.w1[2 * f] * a0 + P.w1[2 * f + 1] * a1 + P.b1[f]);
      }
      split_bf16(h, h1[kk], l1[kk]);
    }
    bf16x4 h2[4], l2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      __builtin_amdgcn_sched_barrier(0);
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const bf16x4 wv = as_bf16x4(P.wa2[(mt * 4 + kk) * 64 + l]);
        acc = mfma_bf16(wv, h1[kk], acc);
        acc = mfma_bf16(wv, l1[kk], acc);
      }
      float h[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) h[j] = silu_f(acc[j] + P.b2[16 * mt + 4 * q + j]);
      split_bf16(h, h2[mt], l2[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      __builtin_amdgcn_sched_barrier(0);
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const bf16x4 wv = as_bf16x4(P.wa3[(mt * 4 + kk) * 64 + l]);
        acc = mfma_bf16(wv, h2[kk], acc);
        acc = mfma_bf16(wv, l2[kk], acc);
      }
      float h3[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) h3[j] = silu_f(acc[j] + P.b3[16 * mt + 4 * q + j]);
      out(nt, mt, h3, P);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The same with the parameters in global memory (the view's arrays).
template <typename Out>
__device__ __forceinline__ void mlp_wave_hidden(const MlpView& M, float x0, float x1, Out&& out) {
  mlp_wave_layers(
      [&]() {
        const float* w = M.wr;
        const uint2* wa2 = M.wa2;
        const uint2* wa3 = M.wa3;
        asm volatile("" : "+s"(w), "+s"(wa2), "+s"(wa3));
        return MlpP{w + MLP_OW1, w + MLP_OB1, w + MLP_OB2, w + MLP_OB3, w + MLP_OW4, w + MLP_OB4, wa2, wa3};
      },
      x0, x1, out);
}

// The parameters staged in LDS by a kernel that evaluates the network for many full waves
// (mlp_stage_lds, then a barrier): the 450 FP32 parameters the forward pass reads (W1, b1, b2,
// b3, W4, b4, packed in that order) and the MFMA packs of W2, W3 (18 KB in all).
#define MLP_LDS_W 450
static __shared__ float s_mlp_w[MLP_LDS_W];
static __shared__ uint2 s_mlp_a[2048];
__device__ __forceinline__ void mlp_stage_lds(const MlpView& M) {
  for (int i = threadIdx.x; i < MLP_LDS_W; i += blockDim.x) {
    // [0, 192): W1, b1;  [192, 256): b2;  [256, 450): b3, W4, b4
    const int src = i < 192 ? MLP_OW1 + i : (i < 256 ? MLP_OB2 + (i - 192) : MLP_OB3 + (i - 256));
    s_mlp_w[i] = M.wr[src];
  }
  for (int i = threadIdx.x; i < 1024; i += blockDim.x) {
    s_mlp_a[i] = M.wa2[i];
    s_mlp_a[1024 + i] = M.wa3[i];
  }
}
template <typename Out>
__device__ __forceinline__ void mlp_wave_hidden_lds(float x0, float x1, Out&& out) {
  mlp_wave_layers(
      [&]() {
        int z = 0;   // an offset the compiler cannot see through keeps the loads in the loop
        asm volatile("" : "+s"(z));
        const float* w = s_mlp_w + z;
        return MlpP{w, w + 128, w + 192, w + 256, w + 256 + (MLP_OW4 - MLP_OB3), w + 256 + (MLP_OB4 - MLP_OB3),
                    s_mlp_a + z, s_mlp_a + 1024 + z};
      },
      x0, x1, out);
}

// Network outputs for the 64 inputs held one per lane (x0, x1 normalised).  Every lane of the
// wave must call it; lane l receives the outputs of its own input.  LDS: the parameters staged by
// mlp_stage_lds.
template <bool LDS = false>
__device__ __forceinline__ void mlp_wave(const MlpView& M, float x0, float x1, float& y0, float& y1) {
  const int q = (threadIdx.x & 63) >> 4;
  float p0 = 0.f, p1 = 0.f;
  auto out = [&](int nt, int mt, const float h3[4], const MlpP& P) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = 16 * mt + 4 * q + j;
      p0 += P.w4[f] * h3[j];
      p1 += P.w4[MLP_H + f] * h3[j];
    }
    if (mt == 3) {
      // the four lanes r, r + 16, r + 32, r + 48 hold the partial sums of input 16 nt + r
      p0 += __shfl_xor(p0, 16, 64);
      p0 += __shfl_xor(p0, 32, 64);
      p1 += __shfl_xor(p1, 16, 64);
      p1 += __shfl_xor(p1, 32, 64);
      if (q == nt) {
        y0 = p0 + P.b4[0];
        y1 = p1 + P.b4[1];
      }
      p0 = p1 = 0.f;
    }
  };
  if constexpr (LDS) mlp_wave_hidden_lds(x0, x1, out);
  else mlp_wave_hidden(M, x0, x1, out);
}
