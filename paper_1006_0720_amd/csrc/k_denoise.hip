// Learned denoiser of nodal statistics: BF16 matrix-core (MFMA) GEMM and the
// element-wise kernels of a 4-layer MLP (forward, backward, Adam), the nodal
// feature kernel and the merge with the plain estimator.
//
// Matrix cores: gfx950's v_mfma_f32_16x16x32_bf16 computes a 16x16 FP32 tile
// D = A(16x32) B(32x16) + C over one wave.  Operand layout per lane l:
//   A: row l%16, columns 8*(l/16) .. +7      B: rows 8*(l/16) .. +7, column l%16
//   C/D: rows 4*(l/16) .. +3, column l%16
// A K tail of 16 uses v_mfma_f32_16x16x16bf16_1k (A: columns 4*(l/16) .. +3,
// B: rows 4*(l/16) .. +3, the same C/D).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <hip/hip_bf16.h>

#include "pdf_internal.h"

namespace pdfk {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even binary32 -> bfloat16 bits
// fp32 -> bf16 bits, to nearest with ties to even (the conversion instruction)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
// two values in one word, a in the low half
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v){a, b}, bf16x2v));
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// C (MxN, fp32, row-major, ldc) = op(A) op(B) + beta C;  A, B bf16 row-major.
// op(A)(i,k) = ta ? A[k*lda+i] : A[i*lda+k];  op(B)(k,j) = tb ? B[j*ldb+k] : B[k*ldb+j]
// Workgroup tile 64x64, four waves of 32x32 (2x2 MFMA tiles), K steps of 32.
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 32;

__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t *__restrict__ A,
                                                   int lda, int ta, const uint16_t *__restrict__ B,
                                                   int ldb, int tb, float *__restrict__ C, int ldc,
                                                   float beta, int kchunk) {
  __shared__ uint16_t sA[GT][GK + 4];  // [row i][k]
  __shared__ uint16_t sB[GK][GT + 4];  // [k][col j]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  f32x4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  // split-K: workgroup z covers k in [kb, ke) and adds its partial product
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const bool split = gridDim.z > 1;
  for (int k0 = kb; k0 < ke; k0 += GK) {
    // stage 64x32 of op(A) and 32x64 of op(B) (eight elements per thread each)
    for (int t = tid; t < GT * GK; t += 256) {
      const int r = t / GK, k = t % GK;
      const int gi = i0 + r, gk = k0 + k;
      uint16_t v = 0;
      if (gi < M && gk < ke) v = ta ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk];
      sA[r][k] = v;
      const int kb = t / GT, c = t % GT;
      const int gj = j0 + c, gkb = k0 + kb;
      uint16_t w = 0;
      if (gj < N && gkb < ke) w = tb ? B[(size_t)gj * ldb + gkb] : B[(size_t)gkb * ldb + gj];
      sB[kb][c] = w;
    }
    __syncthreads();
    const int kq = 8 * (lane >> 4), rc = lane & 15;
    for (int a = 0; a < 2; ++a) {
      bf16x8 fa;
      for (int q = 0; q < 8; ++q) fa[q] = __builtin_bit_cast(__bf16, sA[wi + 16 * a + rc][kq + q]);
      for (int b = 0; b < 2; ++b) {
        bf16x8 fb;
        for (int q = 0; q < 8; ++q) fb[q] = __builtin_bit_cast(__bf16, sB[kq + q][wj + 16 * b + rc]);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int rq = 4 * (lane >> 4), cc = lane & 15;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int q = 0; q < 4; ++q) {
        const int gi = i0 + wi + 16 * a + rq + q, gj = j0 + wj + 16 * b + cc;
        if (gi < M && gj < N) {
          float *c = &C[(size_t)gi * ldc + gj];
          if (split)
            unsafeAtomicAdd(c, acc[a][b][q]);
          else
            *c = (beta != 0.f ? beta * *c : 0.f) + acc[a][b][q];
        }
      }
}

__global__ void k_zero2d(int M, int N, float *C, int ldc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (int64_t)M * N) C[(t / N) * ldc + t % N] = 0.f;
}

void launch_gemm_bf16(hipStream_t s, int M, int N, int K, const uint16_t *A, int lda, int ta,
                      const uint16_t *B, int ldb, int tb, float *C, int ldc, float beta) {
  const int tiles = ((N + GT - 1) / GT) * ((M + GT - 1) / GT);
  // few output tiles and a long K (weight gradients over a batch): split K
  // so that the grid fills the GPU; partial products are added atomically
  int splits = 1;
  if (beta == 0.f && tiles < 512 && K >= 4 * 256) splits = std::min((K + 255) / 256, std::max(1, 2048 / tiles));
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + GK - 1) / GK * GK;
  splits = (K + kchunk - 1) / kchunk;
  if (splits > 1)
    hipLaunchKernelGGL(k_zero2d, dim3((unsigned)(((int64_t)M * N + 255) / 256)), dim3(256), 0, s, M, N, C, ldc);
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, splits);
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, M, N, K, A, lda, ta, B, ldb, tb, C, ldc, beta, kchunk);
}

// erf by the rational approximation of Abramowitz & Stegun (Handbook of
// Mathematical Functions, formula 7.1.26; absolute error at most 1.5e-7):
// one reciprocal and one exponential, no branches, where the library erff
// takes about four times the instructions (it dominated the fused inference)
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  const float poly =
      fmaf(fmaf(fmaf(fmaf(1.061405429f, t, -1.453152027f), t, 1.421413741f), t, -0.284496736f), t, 0.254829592f) * t;
  return copysignf(fmaf(-poly, __expf(-ax * ax), 1.0f), x);
}

// GELU through erf, and its derivative
__device__ __forceinline__ float gelu(float x) {
  const float h = 0.5f * x;
  return fmaf(h, erf_as(x * 0.70710678118654752f), h);
}
__device__ __forceinline__ float dgelu(float x) {
  return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) + x * 0.3989422804014327f * __expf(-0.5f * x * x);
}

// ---------------------------------------------------------------------------
// Fused inference: the whole MLP in one kernel.  A workgroup of MLPF_WAVES
// waves stages all four layers' weights (transposed, [n][k] with k contiguous,
// so that both MFMA operands are 8-byte LDS reads) and biases in LDS once;
// each wave then takes 16-row tiles in turn and keeps a tile's activations
// (bf16) in LDS through the four layers, so neither weights nor activations
// are re-read from memory, and the next tile's inputs are loaded while the
// current one is computed.  Rounding points are those of the layer-by-layer
// path: fp32 accumulation, + bias, GELU, bf16.
// ---------------------------------------------------------------------------
constexpr int MLP_PAD = 8, MLPF_WAVES = 8;

__device__ __forceinline__ bf16x4 lds_frag(const uint16_t *p) {
  const uint2 v = *(const uint2 *)p;
  bf16x4 r;
  r[0] = (short)(v.x & 0xFFFFu);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xFFFFu);
  r[3] = (short)(v.y >> 16);
  return r;
}

// eight bf16 from 16-byte-aligned LDS
__device__ __forceinline__ bf16x8 lds_frag8(const uint16_t *p) { return __builtin_bit_cast(bf16x8, *(const uint4 *)p); }

// W [K][N] (row-major) -> Wt [Np][K + MLP_PAD] (Np = N rounded up to 16,
// columns N .. Np-1 zero): the LDS layout of a layer, kept in global memory
// so that a workgroup stages it with 16-byte copies
__global__ void k_transpose_w(const uint16_t *W, int K, int N, uint16_t *Wt) {
  const int Np = (N + 15) & ~15, ld = K + MLP_PAD;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Np * ld) return;
  const int n = t / ld, k = t % ld;
  Wt[t] = (n < N && k < K) ? W[(size_t)k * N + n] : (uint16_t)0;
}

__host__ __device__ inline size_t mlp_wt_elems(int K, int N) { return (size_t)((N + 15) & ~15) * (K + MLP_PAD); }

void launch_transpose_weights(hipStream_t s, int H, const uint16_t *W1, const uint16_t *W2, const uint16_t *W3,
                              const uint16_t *W4, uint16_t *Wt) {
  const uint16_t *W[4] = {W1, W2, W3, W4};
  const int K[4] = {48, H, H, H}, N[4] = {H, H, H, 8};
  for (int l = 0; l < 4; ++l) {
    const size_t ne = mlp_wt_elems(K[l], N[l]);
    hipLaunchKernelGGL(k_transpose_w, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, W[l], K[l], N[l], Wt);
    Wt += ne;
  }
}

__device__ __forceinline__ void stage_copy(const uint16_t *src, size_t n, uint16_t *dst) {
  const uint4 *s4 = (const uint4 *)src;
  uint4 *d4 = (uint4 *)dst;
  for (size_t t = threadIdx.x; t < n / 8; t += blockDim.x) d4[t] = s4[t];
}

// NT 16-column tiles of one layer, starting at column n0, for the calling
// wave's 16 rows: fp32 accumulation over K, then + bias and GELU (bf16 into
// out) or + bias (fp32 into y, rows below nrows).  The product is formed
// transposed (weights as the first MFMA operand), so that each lane ends
// with four adjacent columns of one row: one 8-byte LDS store per tile.
template <int NT>
__device__ __forceinline__ void mlp_pass(const uint16_t *in, int K, const uint16_t *Wt, int N, int n0,
                                         const float *b, bool gelu_act, uint16_t *out, float *y, int64_t row0,
                                         int64_t nrows) {
  const int lane = threadIdx.x & 63;
  const int ldi = K + MLP_PAD;
  const int kq = 4 * (lane >> 4), rc = lane & 15, kq8 = 8 * (lane >> 4);
  f32x4 acc[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) acc[u] = (f32x4){0.f, 0.f, 0.f, 0.f};
  int k0 = 0;
  for (; k0 + 32 <= K; k0 += 32) {
    const bf16x8 fa = lds_frag8(in + rc * ldi + k0 + kq8);
    bf16x8 fb[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) fb[u] = lds_frag8(Wt + (n0 + 16 * u + rc) * ldi + k0 + kq8);
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[u], fa, acc[u], 0, 0, 0);
  }
  if (k0 < K) {  // K a multiple of 16: a tail of 16
    const bf16x4 fa = lds_frag(in + rc * ldi + k0 + kq);
    bf16x4 fb[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) fb[u] = lds_frag(Wt + (n0 + 16 * u + rc) * ldi + k0 + kq);
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fb[u], fa, acc[u], 0, 0, 0);
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int c0 = n0 + 16 * u + kq;  // this lane's columns c0 .. c0 + 3 of row rc
    if (c0 >= N) continue;
    if (y) {
      if (row0 + rc < nrows)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (c0 + q < N) y[(row0 + rc) * N + c0 + q] = acc[u][q] + b[c0 + q];
    } else {  // N is a multiple of 16 here
      float g[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float z = acc[u][q] + b[c0 + q];
        g[q] = gelu_act ? gelu(z) : z;
      }
      uint2 w;
      w.x = f2bf2(g[0], g[1]);
      w.y = f2bf2(g[2], g[3]);
      *(uint2 *)(out + rc * (N + MLP_PAD) + c0) = w;
    }
  }
}

// one layer for the calling wave: out[16][N] = act(in[16][K] W + b), in
// passes of four 16-column tiles and a narrower last pass
__device__ __forceinline__ void mlp_layer(const uint16_t *in, int K, const uint16_t *Wt, int N,
                                          const float *b, bool gelu_act, uint16_t *out, float *y,
                                          int64_t row0, int64_t nrows) {
  const int Np = (N + 15) & ~15;
  int n0 = 0;
  for (; n0 + 64 <= Np; n0 += 64) mlp_pass<4>(in, K, Wt, N, n0, b, gelu_act, out, y, row0, nrows);
  switch ((Np - n0) / 16) {
    case 3: mlp_pass<3>(in, K, Wt, N, n0, b, gelu_act, out, y, row0, nrows); break;
    case 2: mlp_pass<2>(in, K, Wt, N, n0, b, gelu_act, out, y, row0, nrows); break;
    case 1: mlp_pass<1>(in, K, Wt, N, n0, b, gelu_act, out, y, row0, nrows); break;
    default: break;
  }
}

// orders one wave's LDS writes before its later LDS reads (no other wave
// takes part)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one 16-row tile of inputs (16 x 48 fp32, contiguous): 192 float4, three per
// lane; rows at or beyond n read as zero
__device__ __forceinline__ void mlp_load_tile(const float *__restrict__ x, int64_t tile, int64_t n, int lane,
                                              float4 v[3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int q = lane + 64 * j;
    const int64_t g = tile * 16 + q / 12;
    v[j] = g < n ? ldg((const float4 *)(x + g * 48), (size_t)(q % 12)) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

__global__ __launch_bounds__(64 * MLPF_WAVES) void k_mlp_forward(int64_t n, int H, const float *__restrict__ x,
                                                                 const uint16_t *__restrict__ Wt_all,
                                                                 const float *b1, const float *b2,
                                                                 const float *b3, const float *b4, float *y) {
  extern __shared__ uint16_t lds[];
  const int ldh = H + MLP_PAD, ldx = 48 + MLP_PAD;
  const size_t n1 = mlp_wt_elems(48, H), n2 = mlp_wt_elems(H, H), n4 = mlp_wt_elems(H, 8);
  const size_t nw = n1 + 2 * n2 + n4;  // a multiple of 8 (H is)
  uint16_t *Wt1 = lds, *Wt2 = Wt1 + n1, *Wt3 = Wt2 + n2, *Wt4 = Wt3 + n2;
  float *bl = (float *)(lds + nw);  // biases: H, H, H, 8
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint16_t *actA = (uint16_t *)(bl + 3 * H + 8) + wave * 32 * ldh;  // two [16][H + PAD] buffers
  uint16_t *actB = actA + 16 * ldh;
  {  // weights: four 16-byte loads in flight per thread before they are stored
    const uint4 *s4 = (const uint4 *)Wt_all;
    uint4 *d4 = (uint4 *)lds;
    const int n16 = (int)(nw / 8), nt = (int)blockDim.x;
    for (int t0 = (int)threadIdx.x; t0 < n16; t0 += 4 * nt) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = s4[min(t0 + u * nt, n16 - 1)];  // in bounds; extra copies unused
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (t0 + u * nt < n16) d4[t0 + u * nt] = v[u];
    }
    for (int t = (int)threadIdx.x; t < 3 * H + 8; t += nt)
      bl[t] = t < H ? b1[t] : t < 2 * H ? b2[t - H] : t < 3 * H ? b3[t - 2 * H] : b4[t - 3 * H];
  }
  const int64_t ntiles = (n + 15) / 16, tstride = (int64_t)gridDim.x * MLPF_WAVES;
  int64_t tile = (int64_t)blockIdx.x * MLPF_WAVES + wave;
  float4 xv[3];
  mlp_load_tile(x, tile, n, lane, xv);
  __syncthreads();  // every wave passes here exactly once
  for (; tile < ntiles; tile += tstride) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int q = lane + 64 * j, r = q / 12, k = 4 * (q % 12);
      uint2 w;
      w.x = (uint32_t)f2bf(xv[j].x) | ((uint32_t)f2bf(xv[j].y) << 16);
      w.y = (uint32_t)f2bf(xv[j].z) | ((uint32_t)f2bf(xv[j].w) << 16);
      *(uint2 *)(actA + r * ldx + k) = w;
    }
    if (tile + tstride < ntiles) mlp_load_tile(x, tile + tstride, n, lane, xv);
    const int64_t row0 = tile * 16;
    wave_lds_sync();
    mlp_layer(actA, 48, Wt1, H, bl, true, actB, nullptr, row0, n);
    wave_lds_sync();
    mlp_layer(actB, H, Wt2, H, bl + H, true, actA, nullptr, row0, n);
    wave_lds_sync();
    mlp_layer(actA, H, Wt3, H, bl + 2 * H, true, actB, nullptr, row0, n);
    wave_lds_sync();
    mlp_layer(actB, H, Wt4, 8, bl + 3 * H, false, nullptr, y, row0, n);
    wave_lds_sync();
  }
}

size_t mlp_transposed_elems(int H) { return mlp_wt_elems(48, H) + 2 * mlp_wt_elems(H, H) + mlp_wt_elems(H, 8); }

size_t mlp_forward_lds(int H) {
  return mlp_transposed_elems(H) * sizeof(uint16_t) + (3 * (size_t)H + 8) * sizeof(float) +
         (size_t)MLPF_WAVES * 2 * 16 * (size_t)(H + MLP_PAD) * sizeof(uint16_t);
}

bool launch_mlp_forward(hipStream_t s, int64_t n, int H, const float *x, const uint16_t *Wt_all, const float *b1,
                        const float *b2, const float *b3, const float *b4, float *y) {
  // LDS holds all weights and each wave's activations: hidden widths 48..128, multiples of 16
  if (H < 48 || H > 128 || H % 16 || n <= 0) return false;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
    return false;
  const int64_t tiles = (n + 15) / 16, wgs = (tiles + MLPF_WAVES - 1) / MLPF_WAVES;
  const unsigned g = (unsigned)(wgs < ncu ? wgs : ncu);  // one workgroup per CU: the LDS holds one
  hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(64 * MLPF_WAVES), mlp_forward_lds(H), s, n, H, x, Wt_all, b1,
                     b2, b3, b4, y);
  return true;
}

// ---------------------------------------------------------------------------
// element-wise pieces of the MLP
// ---------------------------------------------------------------------------

// Z += b (in place, fp32) and H = gelu(Z) (bf16) or H = Z (bf16) when act == 0
__global__ void k_bias_act(int M, int N, float *Z, const float *b, uint16_t *H, int act) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * N) return;
  const int j = (int)(t % N);
  const float z = Z[t] + b[j];
  Z[t] = z;
  if (H) H[t] = f2bf(act ? gelu(z) : z);
}

// dZ = dH * gelu'(Z)  (fp32 in, bf16 out; fp32 copy kept in place of dH)
__global__ void k_dgelu(int64_t n, float *dH, const float *Z, uint16_t *dZb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float g = dH[t] * dgelu(Z[t]);
  dH[t] = g;
  dZb[t] = f2bf(g);
}

// column sums of an M x N fp32 matrix (bias gradients): one block per column
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const float *G, float *out) {
  __shared__ float red[256];
  const int j = blockIdx.x;
  float acc = 0.f;
  for (int i = threadIdx.x; i < M; i += 256) acc += G[(size_t)i * N + j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

// MSE over the valid outputs: Y (M x ldy, first nout columns), targets T (M x nout)
// dY = 2 (Y - T) / (M nout) written as fp32 (in place of Y) and bf16; per-block
// partial losses in part[]
__global__ __launch_bounds__(256) void k_mse(int M, int nout, int ldy, float *Y, const float *T,
                                             uint16_t *dYb, float *part) {
  __shared__ float red[256];
  const int64_t n = (int64_t)M * ldy;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (t < n) {
    const int i = (int)(t / ldy), j = (int)(t % ldy);
    float g = 0.f;
    if (j < nout) {
      const float d = Y[t] - T[(size_t)i * nout + j];
      l = d * d;
      g = 2.f * d / ((float)M * (float)nout);
    }
    Y[t] = g;
    dYb[t] = f2bf(g);
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam (Kingma & Ba 2015) on fp32 master parameters; refreshes the bf16 copy
__global__ void k_adam(int64_t n, float *w, const float *g, float *m, float *v, uint16_t *wb, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gi = g[t];
  const float mi = b1 * m[t] + (1.f - b1) * gi;
  const float vi = b2 * v[t] + (1.f - b2) * gi * gi;
  m[t] = mi;
  v[t] = vi;
  const float wi = w[t] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[t] = wi;
  if (wb) wb[t] = f2bf(wi);
}

__global__ void k_to_bf16(int64_t n, const float *x, uint16_t *y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = f2bf(x[t]);
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_bias_act(hipStream_t s, int M, int N, float *Z, const float *b, uint16_t *H, int act) {
  hipLaunchKernelGGL(k_bias_act, dim3(nblk((int64_t)M * N)), dim3(256), 0, s, M, N, Z, b, H, act);
}
void launch_dgelu(hipStream_t s, int64_t n, float *dH, const float *Z, uint16_t *dZb) {
  hipLaunchKernelGGL(k_dgelu, dim3(nblk(n)), dim3(256), 0, s, n, dH, Z, dZb);
}
void launch_colsum(hipStream_t s, int M, int N, const float *G, float *out) {
  hipLaunchKernelGGL(k_colsum, dim3(N), dim3(256), 0, s, M, N, G, out);
}
int launch_mse(hipStream_t s, int M, int nout, int ldy, float *Y, const float *T, uint16_t *dYb,
               float *part) {
  const unsigned nb = nblk((int64_t)M * ldy);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, M, nout, ldy, Y, T, dYb, part);
  return (int)nb;
}
void launch_adam(hipStream_t s, int64_t n, float *w, const float *g, float *m, float *v, uint16_t *wb,
                 float lr, float b1, float b2, float eps, float c1, float c2) {
  hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, s, n, w, g, m, v, wb, lr, b1, b2, eps, c1, c2);
}
void launch_to_bf16(hipStream_t s, int64_t n, const float *x, uint16_t *y) {
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n)), dim3(256), 0, s, n, x, y);
}

// ---------------------------------------------------------------------------
// Nodal features for the denoiser.  For each of 8 statistics q (<U>, <V>,
// <phi>, <uu>, <vv>, <uv>, <phi'^2>, <omega>) at node n: the value, the mean,
// standard deviation, minimum and maximum over the node and its neighbours
// (points surrounding points), and the magnitude of the nodal gradient
// (eq:gradient in the surrounding elements, averaged).  Output row n: 48
// features, standardised with (x - mu) / sigma, as bf16 and fp32.
// ---------------------------------------------------------------------------
constexpr int kQuant[8] = {0, 1, 4, 5, 6, 8, 11, 3};
__constant__ int kQuantDev[8] = {0, 1, 4, 5, 6, 8, 11, 3};

// one thread per (node, statistic): the 6 features of statistic a at node
// n = n0 + r, written to row r of F (rows r < cnt)
__global__ __launch_bounds__(256) void k_features(MeshDev m, const int32_t *p2p_off, const int32_t *p2p,
                                                  const double2 *gw, const double *S, const float *mu,
                                                  const float *sig, int32_t n0, int32_t cnt, float *F,
                                                  uint16_t *Fb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t r = (int32_t)(t >> 3);
  const int a = (int)(t & 7);
  if (r >= cnt) return;
  const int32_t n = n0 + r;
  const int nn = m.nn;
  const int32_t q = m.master[n];
  const int fld = kQuantDev[a];
  const double *Sf = S + (size_t)fld * nn;
  const double v0 = Sf[q];
  double sum = v0, sum2 = v0 * v0, mn = v0, mx = v0;
  const double2 w0 = gw[q];
  double gx = w0.x * v0, gy = w0.y * v0;  // the averaged element gradient, through the ring weights
  int c = 1;
  // neighbours four at a time, so that their gathers are in flight together
  // (the sums still run in list order)
  const int32_t pb = p2p_off[q], pe = p2p_off[q + 1];
  for (int32_t i = pb; i < pe; i += 4) {
    int32_t jn[4];
    double v[4];
    double2 w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) jn[u] = p2p[min(i + u, pe - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = gw[m.nn + min(i + u, pe - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = Sf[jn[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u < pe) {
        gx += w[u].x * v[u];
        gy += w[u].y * v[u];
        sum += v[u];
        sum2 += v[u] * v[u];
        mn = v[u] < mn ? v[u] : mn;
        mx = v[u] > mx ? v[u] : mx;
        c++;
      }
  }
  const double mean = sum / c;
  double var = sum2 / c - mean * mean;
  var = var > 0.0 ? var : 0.0;
  const float f[6] = {(float)v0, (float)mean, (float)sqrt(var), (float)mn, (float)mx,
                      (float)sqrt(gx * gx + gy * gy)};
  for (int j = 0; j < 6; ++j) {
    const int k = 6 * a + j;
    const float z = mu ? (f[j] - mu[k]) / sig[k] : f[j];
    F[(size_t)r * 48 + k] = z;
    if (Fb) Fb[(size_t)r * 48 + k] = f2bf(z);
  }
}

void launch_features_range(hipStream_t s, const MeshDev &m, const int32_t *p2p_off, const int32_t *p2p,
                           const double2 *gw, const double *S, const float *mu, const float *sig, int32_t n0,
                           int32_t cnt, float *F, uint16_t *Fb) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_features, dim3((unsigned)(((int64_t)cnt * 8 + 255) / 256)), dim3(256), 0, s, m, p2p_off,
                     p2p, gw, S, mu, sig, n0, cnt, F, Fb);
}

void launch_features(hipStream_t s, const MeshDev &m, const int32_t *p2p_off, const int32_t *p2p,
                     const double2 *gw, const double *S, const float *mu, const float *sig, float *F,
                     uint16_t *Fb) {
  launch_features_range(s, m, p2p_off, p2p, gw, S, mu, sig, 0, m.nn, F, Fb);
}

// Merge: q = q_plain + scale_q * r_q, except where |scale_q r_q| exceeds
// tau * kappa_q times the plain estimator's standard error at the node (then
// q = q_plain).  scale holds 16 values: scale_q (0..7), then kappa_q (8..15),
// the calibration of the standard error to the plain estimator's actual error.
// Standard errors from the plain second moments and the particle support N:
// <U>: sqrt(<uu>/N), <V>: sqrt(<vv>/N), <phi>: sqrt(<phi'^2>/N), second
// moments s: s sqrt(2/N), <uv>: sqrt((<uu><vv> + <uv>^2)/N), <omega>: <omega>
// sqrt(C4/N).  Every other statistic is copied from the plain estimate.
// Node n = n0 + r takes its network output from row r of R (rows r < cnt).
__global__ void k_merge(int nn, const int32_t *__restrict__ master, const double *__restrict__ S, int32_t n0,
                        int32_t cnt, const float *__restrict__ R, int ldr, const float *__restrict__ scale,
                        double tau, double C4, double *__restrict__ out, unsigned long long *nfall) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t n = n0 + r;
  int fb = 0;
  if (r < cnt) {
    const int32_t q = master[n];
    const double N = S[24 * (size_t)nn + q];
    const double uu = S[5 * (size_t)nn + q], vv = S[6 * (size_t)nn + q], uv = S[8 * (size_t)nn + q];
    const double pp = S[11 * (size_t)nn + q], om = S[3 * (size_t)nn + q];
    const double iN = N > 0.0 ? 1.0 / N : 1.0;
    double se[8];
    se[0] = sqrt(fabs(uu) * iN);
    se[1] = sqrt(fabs(vv) * iN);
    se[2] = sqrt(fabs(pp) * iN);
    se[3] = fabs(uu) * sqrt(2.0 * iN);
    se[4] = fabs(vv) * sqrt(2.0 * iN);
    se[5] = sqrt((fabs(uu * vv) + uv * uv) * iN);
    se[6] = fabs(pp) * sqrt(2.0 * iN);
    se[7] = fabs(om) * sqrt(C4 * iN);
    double mv[8];
    bool ok[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int fld = kQuant[a];
      const double corr = (double)scale[a] * (double)R[(size_t)r * ldr + a];
      // taken unless it exceeds the limit; tau = +inf takes every finite
      // correction (inf * 0 at a node of zero spread is NaN, not a limit)
      const double lim = tau * (double)scale[8 + a] * se[a];
      ok[a] = isfinite(corr) && !(fabs(corr) > lim);
      mv[a] = S[(size_t)fld * nn + q] + corr;
      fb += ok[a] ? 0 : 1;
    }
    // all statistics written, every line whole
#pragma unroll
    for (int f = 0; f < PDF_NSTAT; ++f) {
      double v = S[(size_t)f * nn + n];
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (kQuant[a] == f && ok[a]) v = mv[a];
      out[(size_t)f * nn + n] = v;
    }
  }
  // one atomic per wave: many nodes reject a correction, and one counter
  // taking an atomic from each of them serialises the launch
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) fb += __shfl_xor(fb, o, 64);
  if (nfall && fb && (threadIdx.x & 63) == 0) atomicAdd(nfall, (unsigned long long)fb);
}

void launch_merge_range(hipStream_t s, int nn, const int32_t *master, const double *S, int32_t n0, int32_t cnt,
                        const float *R, int ldr, const float *scale, double tau, double C4, double *out,
                        unsigned long long *nfall) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_merge, dim3((cnt + 255) / 256), dim3(256), 0, s, nn, master, S, n0, cnt, R, ldr, scale,
                     tau, C4, out, nfall);
}

void launch_merge(hipStream_t s, int nn, const int32_t *master, const double *S, const float *R, int ldr,
                  const float *scale, double tau, double C4, double *out, unsigned long long *nfall) {
  launch_merge_range(s, nn, master, S, 0, nn, R, ldr, scale, tau, C4, out, nfall);
}

}  // namespace pdfk
