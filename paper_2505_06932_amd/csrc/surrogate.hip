// surrogate.hip -- learned curvature: a 30-64-64-1 network that maps what the
// PPIC volume fit (paper section 3.2) sees around an interfacial cell -- the
// 27 volume fractions of the 3x3x3 block of cells centred on it and the fit's
// frame normal (the area-weighted normal of the closest front vertex) -- to
// kappa h.  Evaluated and trained with bfloat16 matrix-core products
// (v_mfma_f32_16x16x32_bf16) and single-precision sums.
//
// Network: z1 = W1 x + b1, h1 = bf16(tanh z1), z2 = W2 h1 + b2,
// h2 = bf16(tanh z2), y = w3 . h2 + b3; weights rounded to bfloat16, biases in
// single precision.  Each single-precision input x is fed as the pair
// x_hi = bf16(x), x_lo = bf16(x - x_hi) through the same weights, which keeps
// 16 significant bits of every volume fraction.
//
// Matrix-core layout (lane l, lane group g = l / 16, r = l % 16): the A
// operand holds row r of a 16-row block and the B operand column r, each
// with the 8 reduction slots 8 g .. 8 g + 7 of a 32-wide step; the 16x16
// result holds rows 4 g .. 4 g + 3 of column r.  Products run transposed
// (hidden units x samples), so a lane's results are 4 hidden units of one
// sample, and the reduction slots are assigned so that those results are
// the next layer's B operand in the same lane:
//   layer 1, step ks, slot j: input feature 16 ks + 4 g + j / 2, part j % 2;
//   layers 2 and the backward product, step ks, slot j: hidden unit
//   16 (2 ks + j / 4) + 4 g + j % 4.
//
// Training: the mean squared error over a batch, its gradient by the
// backward pass with the derivative of tanh taken from the stored (rounded)
// activation, dz rounded to bfloat16 before each product; weight gradients
// are products over samples staged through LDS; per-workgroup partial sums
// are reduced in a fixed order, then Adam updates the single-precision
// parameters.
//
// Error estimate and fallback: kappa is invariant under the 48 symmetries of
// the cube applied to the stencil and the normal together; the predictions
// under four of them (identity, a quarter turn about z, the cyclic exchange
// of the axes, the point reflection) give the mean (the estimate) and the
// spread (max - min).  A cell whose spread exceeds the bound, or without a
// closest vertex within 1.5 h of its centre, is handed to the PPIC kernels,
// which then run on those cells only.
#include <mutex>

#include "ftc_ws.hpp"

namespace ftc {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kIn = 30, kHid = 64, kFeat = FTC_MLP_FEATURES;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
              kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid, kNP = kOffB3 + 1;
static_assert(kNP == FTC_MLP_PARAMS, "parameter count");
constexpr int kPartStride = FTC_MLP_PARAMS + 3;  // parameters, loss, padding to 16 bytes
static_assert(kPartStride % 4 == 0, "partial rows are float4 aligned");
constexpr int kGradBlocks = FTC_MLP_WORK_FLOATS / kPartStride;
static_assert(kGradBlocks >= 1, "work size");

// ------------------------------------------------------------- symmetries
// Symmetry s in [0, 48): permutation s / 8 of the axes (lexicographic), axis a
// negated where bit a of s % 8 is set: (P x)_a = sign_a x_perm[a].  The mapped
// configuration has stencil entry alpha'(d) = alpha(P^T d) and normal P n;
// the table gives, per entry of the mapped feature row, its source entry
// and sign (0 for the two padding entries).
struct SymTab {
  int8_t src[48][kFeat];
  int8_t sgn[48][kFeat];
};
constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
constexpr SymTab make_symtab() {
  SymTab T{};
  for (int s = 0; s < 48; ++s) {
    const int* p = kPerm[s / 8];
    int sg[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) sg[a] = ((s % 8) >> a) & 1 ? -1 : 1;
    for (int q = 0; q < 27; ++q) {
      const int d[3] = {q % 3 - 1, (q / 3) % 3 - 1, q / 9 - 1};
      int e[3] = {0, 0, 0};  // e = P^T d: (P^T d)_{perm[a]} = sign_a d_a
      for (int a = 0; a < 3; ++a) e[p[a]] = sg[a] * d[a];
      T.src[s][q] = (int8_t)(9 * (e[2] + 1) + 3 * (e[1] + 1) + (e[0] + 1));
      T.sgn[s][q] = 1;
    }
    for (int a = 0; a < 3; ++a) {
      T.src[s][27 + a] = (int8_t)(27 + p[a]);
      T.sgn[s][27 + a] = (int8_t)sg[a];
    }
    for (int q = 30; q < kFeat; ++q) {
      T.src[s][q] = 30;
      T.sgn[s][q] = 0;
    }
  }
  return T;
}
__constant__ SymTab kSym = make_symtab();
constexpr int kErrSet[4] = {0, 17, 24, 7};

// ----------------------------------------------------------- bfloat16 bits
__device__ inline uint32_t bf16_bits(float x) {  // nearest, ties to even (finite x)
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline float bf16_val(uint32_t b) { return __uint_as_float(b << 16); }
__device__ inline float round_bf16(float x) { return bf16_val(bf16_bits(x)); }
__device__ inline uint32_t pack2(float lo, float hi) { return bf16_bits(lo) | (bf16_bits(hi) << 16); }
__device__ inline bf16x8 as_bf16(u32x4 u) { return __builtin_bit_cast(bf16x8, u); }
__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// tanh x = 1 - 2 / (1 + e^(2x)) with the hardware exponential and reciprocal
// (e^(2x) = +inf for large x gives 1; about 1e-7 absolute error, below the
// bfloat16 rounding that follows every activation).
__device__ inline float tanh_f(float x) { return 1.f - __fdividef(2.f, 1.f + __expf(2.f * x)); }

__device__ inline int wave_max(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// hidden unit of slot j of step ks in lane group g (layers 2 and backward)
__device__ inline int hid_slot(int ks, int g, int j) { return 16 * (2 * ks + (j >> 2)) + 4 * g + (j & 3); }

// The network's operands in this lane's registers.
struct Net {
  bf16x8 w1[4][2];         // layer 1 A operand [row block][step]
  bf16x8 w2[4][2];         // layer 2 A operand
  float b1[4][4], b2[4][4];  // result layout: unit 16 mb + 4 g + i
  float w3[4][4];
  float b3;
};
struct NetT {
  bf16x8 w2t[4][2];  // W2 transposed: A operand of dh1 = W2^T dz2
};

__device__ inline void load_net(const float* __restrict__ th, Net& N) {
  const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int o = 16 * mb + r;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      u32x4 u1, u2;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int f = 16 * ks + 4 * g + w;
        const uint32_t b = bf16_bits(f < kIn ? th[kOffW1 + o * kIn + f] : 0.f);
        u1[w] = b | (b << 16);  // the same weight for x_hi and x_lo
        u2[w] = pack2(th[kOffW2 + o * kHid + hid_slot(ks, g, 2 * w)], th[kOffW2 + o * kHid + hid_slot(ks, g, 2 * w + 1)]);
      }
      N.w1[mb][ks] = as_bf16(u1);
      N.w2[mb][ks] = as_bf16(u2);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int u = 16 * mb + 4 * g + i;
      N.b1[mb][i] = th[kOffB1 + u];
      N.b2[mb][i] = th[kOffB2 + u];
      N.w3[mb][i] = round_bf16(th[kOffW3 + u]);
    }
  }
  N.b3 = th[kOffB3];
}

__device__ inline void load_net_t(const float* __restrict__ th, NetT& T) {
  const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int o1 = 16 * mb + r;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      u32x4 u;
#pragma unroll
      for (int w = 0; w < 4; ++w)
        u[w] = pack2(th[kOffW2 + hid_slot(ks, g, 2 * w) * kHid + o1], th[kOffW2 + hid_slot(ks, g, 2 * w + 1) * kHid + o1]);
      T.w2t[mb][ks] = as_bf16(u);
    }
  }
}

// Layer-1 B operand from this lane's features x[ks][w] = feature 16 ks + 4 g + w.
__device__ inline void split_inputs(const float x[2][4], bf16x8 xb[2]) {
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    u32x4 u;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const uint32_t hb = bf16_bits(x[ks][w]);
      const float lo = x[ks][w] - bf16_val(hb);  // exact
      u[w] = hb | (bf16_bits(lo) << 16);
    }
    xb[ks] = as_bf16(u);
  }
}

// Forward pass of 16 samples (one per r); every lane of sample r gets y.
__device__ inline float forward_tile(const Net& N, const bf16x8 xb[2], float h1[4][4], float h2[4][4]) {
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f32x4 a = mfma(N.w1[mb][0], xb[0], zero4());
    a = mfma(N.w1[mb][1], xb[1], a);
#pragma unroll
    for (int i = 0; i < 4; ++i) h1[mb][i] = round_bf16(tanh_f(a[i] + N.b1[mb][i]));
  }
  bf16x8 hb[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    u32x4 u;
    u[0] = pack2(h1[2 * ks][0], h1[2 * ks][1]);
    u[1] = pack2(h1[2 * ks][2], h1[2 * ks][3]);
    u[2] = pack2(h1[2 * ks + 1][0], h1[2 * ks + 1][1]);
    u[3] = pack2(h1[2 * ks + 1][2], h1[2 * ks + 1][3]);
    hb[ks] = as_bf16(u);
  }
  float s = 0.f;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f32x4 a = mfma(N.w2[mb][0], hb[0], zero4());
    a = mfma(N.w2[mb][1], hb[1], a);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      h2[mb][i] = round_bf16(tanh_f(a[i] + N.b2[mb][i]));
      s += N.w3[mb][i] * h2[mb][i];
    }
  }
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s + N.b3;
}

// This lane's features of sample row `row` (mapped by symmetry sym), zero
// past the row count.
__device__ inline void load_features(const float* __restrict__ X, int64_t row, bool valid, int sym, float x[2][4]) {
  const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int f = 16 * ks + 4 * g + w;
      const int sg = kSym.sgn[sym][f];
      const float v = (valid && sg != 0) ? X[row * kFeat + kSym.src[sym][f]] : 0.f;
      x[ks][w] = sg < 0 ? -v : v;
    }
}

// ------------------------------------------------------------- inference
struct MlpArgs {
  const float* theta;
  const float* X;
  int64_t rows;  // rows of X (and t)
  const int32_t* idx;
  const int32_t* sym;
  const float* t;
  int32_t n;
  float dy_scale;  // 2 / n
  float* y;
  float* part;     // [blocks][kPartStride]
};

// Row and symmetry of batch sample s: row idx[s] (or s), symmetry sym[s] (or
// 0); a sample past n, or whose row lies outside [0, rows), is not valid
// (zero features, no contribution); a symmetry outside [0, 48) is taken as 0.
__device__ inline bool sample_of(const MlpArgs& A, int64_t s, int64_t& row, int& sym) {
  row = 0;
  sym = 0;
  if (s >= A.n) return false;
  const int64_t rw = A.idx ? (int64_t)A.idx[s] : s;
  if (rw < 0 || rw >= A.rows) return false;
  row = rw;
  if (A.sym) {
    const int sv = A.sym[s];
    sym = (sv >= 0 && sv < 48) ? sv : 0;
  }
  return true;
}

__global__ __launch_bounds__(64) void k_mlp_forward(MlpArgs A) {
  Net N;
  load_net(A.theta, N);
  const int r = threadIdx.x & 15, g = threadIdx.x >> 4;
  for (int64_t base = (int64_t)blockIdx.x * 16; base < A.n; base += (int64_t)gridDim.x * 16) {
    const int64_t s = base + r;
    int64_t row;
    int sym;
    const bool valid = sample_of(A, s, row, sym);
    float x[2][4], h1[4][4], h2[4][4];
    load_features(A.X, row, valid, sym, x);
    bf16x8 xb[2];
    split_inputs(x, xb);
    const float y = forward_tile(N, xb, h1, h2);
    if (valid && g == 0) A.y[s] = y;
  }
}

// ------------------------------------------------------------- training
// LDS staging of one 32-sample tile, transposed: [unit][sample] in bfloat16.
struct __align__(16) TrainLds {
  uint16_t xT[64][32];   // layer-1 inputs, effective index 2 f + part
  uint16_t h1T[64][32];
  uint16_t d1T[64][32];  // dz1
  uint16_t d2T[64][32];  // dz2
};

__device__ inline bf16x8 lds_row8(const uint16_t (*M)[32], int row, int g) {
  return as_bf16(*reinterpret_cast<const u32x4*>(&M[row][8 * g]));
}

__global__ __launch_bounds__(64) void k_mlp_grad(MlpArgs A) {
  __shared__ TrainLds L;
  Net N;
  NetT T;
  load_net(A.theta, N);
  load_net_t(A.theta, T);
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  f32x4 gW1[4][4], gW2[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      gW1[a][b] = zero4();
      gW2[a][b] = zero4();
    }
  float gb1[4][4], gb2[4][4], gw3[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) gb1[a][i] = gb2[a][i] = gw3[a][i] = 0.f;
  float gb3 = 0.f, loss = 0.f;

  for (int64_t base = (int64_t)blockIdx.x * 32; base < A.n; base += (int64_t)gridDim.x * 32) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int col = 16 * half + r;
      const int64_t s = base + col;
      int64_t row;
      int sym;
      const bool valid = sample_of(A, s, row, sym);
      float x[2][4], h1[4][4], h2[4][4];
      load_features(A.X, row, valid, sym, x);
      bf16x8 xb[2];
      split_inputs(x, xb);
      const float y = forward_tile(N, xb, h1, h2);
      const float tgt = valid ? A.t[row] : 0.f;
      const float res = valid ? y - tgt : 0.f;
      const float dy = A.dy_scale * res;
      if (g == 0) {
        loss += res * res;
        gb3 += dy;
      }
      // dz2 and the layer-2 weight vector's gradient
      float d2[4][4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          gw3[mb][i] += dy * h2[mb][i];
          d2[mb][i] = round_bf16((dy * N.w3[mb][i]) * (1.f - h2[mb][i] * h2[mb][i]));
          gb2[mb][i] += d2[mb][i];
        }
      // dh1 = W2^T dz2, dz1
      bf16x8 db[2];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        u32x4 u;
        u[0] = pack2(d2[2 * ks][0], d2[2 * ks][1]);
        u[1] = pack2(d2[2 * ks][2], d2[2 * ks][3]);
        u[2] = pack2(d2[2 * ks + 1][0], d2[2 * ks + 1][1]);
        u[3] = pack2(d2[2 * ks + 1][2], d2[2 * ks + 1][3]);
        db[ks] = as_bf16(u);
      }
      float d1[4][4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        f32x4 a = mfma(T.w2t[mb][0], db[0], zero4());
        a = mfma(T.w2t[mb][1], db[1], a);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          d1[mb][i] = round_bf16(a[i] * (1.f - h1[mb][i] * h1[mb][i]));
          gb1[mb][i] += d1[mb][i];
        }
      }
      // stage the tile's operands of the weight gradients
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int u = 16 * mb + 4 * g + i;
          L.h1T[u][col] = (uint16_t)bf16_bits(h1[mb][i]);
          L.d1T[u][col] = (uint16_t)bf16_bits(d1[mb][i]);
          L.d2T[u][col] = (uint16_t)bf16_bits(d2[mb][i]);
        }
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int f = 16 * ks + 4 * g + w;
          const uint32_t hb = bf16_bits(x[ks][w]);
          L.xT[2 * f][col] = (uint16_t)hb;
          L.xT[2 * f + 1][col] = (uint16_t)bf16_bits(x[ks][w] - bf16_val(hb));
        }
    }
    __syncthreads();
    // weight gradients over the tile's 32 samples: dW1eff = dz1^T x, dW2 = dz2^T h1
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      const bf16x8 a1 = lds_row8(L.d1T, 16 * mo + r, g);
      const bf16x8 a2 = lds_row8(L.d2T, 16 * mo + r, g);
#pragma unroll
      for (int nk = 0; nk < 4; ++nk) {
        gW1[mo][nk] = mfma(a1, lds_row8(L.xT, 16 * nk + r, g), gW1[mo][nk]);
        gW2[mo][nk] = mfma(a2, lds_row8(L.h1T, 16 * nk + r, g), gW2[mo][nk]);
      }
    }
    __syncthreads();
  }

  // sums over the samples of the per-lane gradients (the 16 lanes of a group)
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        gb1[mb][i] += __shfl_xor(gb1[mb][i], o, 64);
        gb2[mb][i] += __shfl_xor(gb2[mb][i], o, 64);
        gw3[mb][i] += __shfl_xor(gw3[mb][i], o, 64);
      }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    gb3 += __shfl_xor(gb3, o, 64);
    loss += __shfl_xor(loss, o, 64);
  }
  float* P = A.part + (int64_t)blockIdx.x * kPartStride;
#pragma unroll
  for (int mo = 0; mo < 4; ++mo)
#pragma unroll
    for (int nk = 0; nk < 4; ++nk)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = 16 * mo + 4 * g + i;
        // effective input 16 nk + r: feature 8 nk + r / 2, the hi and lo parts in neighbouring lanes
        const float v = gW1[mo][nk][i];
        const float pair = v + __shfl_xor(v, 1, 64);
        const int f = 8 * nk + (r >> 1);
        if ((r & 1) == 0 && f < kIn) P[kOffW1 + o * kIn + f] = pair;
        P[kOffW2 + o * kHid + 16 * nk + r] = gW2[mo][nk][i];
      }
  if (r == 0) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = 16 * mb + 4 * g + i;
        P[kOffB1 + u] = gb1[mb][i];
        P[kOffB2 + u] = gb2[mb][i];
        P[kOffW3 + u] = gw3[mb][i];
      }
  }
  if (lane == 0) {
    P[kOffB3] = gb3;
    P[kNP] = loss;
  }
}

// Sum of the partial rows in block order; loss = sum of squares / n.
__global__ void k_mlp_reduce(const float* __restrict__ part, int32_t nblk, int32_t n, float* grad, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNP) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * kPartStride + p];
  if (p < kNP) {
    grad[p] = s;
  } else if (loss) {
    *loss = s / (float)n;
  }
}

__global__ void k_mlp_adam(float* theta, float* m, float* v, const float* __restrict__ grad, float lr, float b1,
                           float b2, float eps, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNP) return;
  const float gp = grad[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  theta[p] -= lr * (mp / bc1) / (sqrtf(vp / bc2) + eps);
}

// ------------------------------------------------------ features, inference
struct SurArgs {
  Grid g;
  int32_t nv;
  const int32_t* cell_ids;
  const double* alpha;
  const int32_t* best_v;
  const double* best_d2;
  const int32_t* vt_off;
  const int32_t* vt_ids;
  const int4* tri4;
  const double2* vtx4;
  const int32_t* counters;
  int32_t cell_cap;
};

// Feature row of interfacial cell c (27 volume fractions, frame normal, two
// zeros); false if the cell has no closest vertex within 1.5 h (normal 0).
__device__ inline bool cell_features(const SurArgs& A, int32_t c, float* row, double nrm[3]) {
  const Grid& g = A.g;
  const Cell3 cc = unpack_cell(g, A.cell_ids[c]);
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const int32_t i = cc.i + q % 3 - 1, j = cc.j + (q / 3) % 3 - 1, k = cc.k + q / 9 - 1;
    const bool in = i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz;
    row[q] = in ? (float)A.alpha[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)] : 0.f;
  }
  const double reach = 1.5 * g.h;
  const double reach2 = reach * reach * (1.0 - 1e-12);
  const int32_t vs = A.best_v[c];
  const bool final = vs >= 0 && vs < A.nv && A.best_d2[c] < reach2;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (final) {
    // incident triangles in ascending order, cross products summed serially
    for (int32_t e = A.vt_off[vs]; e < A.vt_off[vs + 1]; ++e) {
      const int4 t4 = A.tri4[A.vt_ids[e]];
      const P3 a = vtx(A.vtx4, t4.x), b = vtx(A.vtx4, t4.y), d = vtx(A.vtx4, t4.z);
      const double ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
      const double wx = d.x - a.x, wy = d.y - a.y, wz = d.z - a.z;
      s0 += uy * wz - uz * wy;
      s1 += uz * wx - ux * wz;
      s2 += ux * wy - uy * wx;
    }
    const double nl = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
    s0 /= nl;
    s1 /= nl;
    s2 /= nl;
  }
  nrm[0] = s0;
  nrm[1] = s1;
  nrm[2] = s2;
  row[27] = (float)s0;
  row[28] = (float)s1;
  row[29] = (float)s2;
  row[30] = row[31] = 0.f;
  return final;
}

__global__ void k_features(SurArgs A, float* feat, int32_t* fstat) {
  const int32_t nif = min(A.counters[C_NIF], A.cell_cap);
  for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < nif; c += gridDim.x * blockDim.x) {
    float row[kFeat];
    double nrm[3];
    const bool final = cell_features(A, c, row, nrm);
    float4* out = reinterpret_cast<float4*>(feat + (int64_t)c * kFeat);
#pragma unroll
    for (int q = 0; q < kFeat / 4; ++q) out[q] = make_float4(row[4 * q], row[4 * q + 1], row[4 * q + 2], row[4 * q + 3]);
    if (fstat) fstat[c] = final ? 0 : 1;
  }
}

struct CurvArgs {
  SurArgs S;
  const float* theta;
  float bound;
  double* kappa;
  double *nx, *ny, *nz;
  float* spread;
  int32_t* status;
  int32_t* sel;
  int32_t* counters;
};

// Operand image of the network in LDS, shared by the wavefronts of a
// workgroup: the A operands of both layers per (row block, step, lane), and
// b1, b2, w3 (rounded) per unit.
struct NetLds {
  u32x4 w[2][4][2][64];
  float b1[64], b2[64], w3[64];
};

__device__ inline void fill_net_lds(const float* __restrict__ th, NetLds& L) {
  for (int e = threadIdx.x; e < 2 * 4 * 2 * 64; e += blockDim.x) {
    const int layer = e >> 9, mb = (e >> 7) & 3, ks = (e >> 6) & 1, l = e & 63, g = l >> 4, r = l & 15;
    const int o = 16 * mb + r;
    u32x4 u;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if (layer == 0) {
        const int f = 16 * ks + 4 * g + w;
        const uint32_t b = bf16_bits(f < kIn ? th[kOffW1 + o * kIn + f] : 0.f);
        u[w] = b | (b << 16);
      } else {
        u[w] = pack2(th[kOffW2 + o * kHid + hid_slot(ks, g, 2 * w)], th[kOffW2 + o * kHid + hid_slot(ks, g, 2 * w + 1)]);
      }
    }
    L.w[layer][mb][ks][l] = u;
  }
  for (int u = threadIdx.x; u < 64; u += blockDim.x) {
    L.b1[u] = th[kOffB1 + u];
    L.b2[u] = th[kOffB2 + u];
    L.w3[u] = round_bf16(th[kOffW3 + u]);
  }
}

// forward_tile with the operands read from the LDS image.
__device__ inline float forward_tile_lds(const NetLds& L, float b3, const bf16x8 xb[2]) {
  // the operands are read here, where they are used: hoisted out of the
  // callers' loops they would occupy about 110 registers
  asm volatile("" ::: "memory");
  const int l = threadIdx.x & 63, g = l >> 4;
  float h1[4][4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f32x4 a = mfma(as_bf16(L.w[0][mb][0][l]), xb[0], zero4());
    a = mfma(as_bf16(L.w[0][mb][1][l]), xb[1], a);
#pragma unroll
    for (int i = 0; i < 4; ++i) h1[mb][i] = round_bf16(tanh_f(a[i] + L.b1[16 * mb + 4 * g + i]));
  }
  bf16x8 hb[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    u32x4 u;
    u[0] = pack2(h1[2 * ks][0], h1[2 * ks][1]);
    u[1] = pack2(h1[2 * ks][2], h1[2 * ks][3]);
    u[2] = pack2(h1[2 * ks + 1][0], h1[2 * ks + 1][1]);
    u[3] = pack2(h1[2 * ks + 1][2], h1[2 * ks + 1][3]);
    hb[ks] = as_bf16(u);
  }
  float s = 0.f;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f32x4 a = mfma(as_bf16(L.w[1][mb][0][l]), hb[0], zero4());
    a = mfma(as_bf16(L.w[1][mb][1][l]), hb[1], a);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int u = 16 * mb + 4 * g + i;
      s += L.w3[u] * round_bf16(tanh_f(a[i] + L.b2[u]));
    }
  }
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s + b3;
}

// Feature row of cell c (or zeros, c < 0) by the four lane groups of its
// column r: volume fractions q = g, g + 4, ...; the normal's cross products
// four triangles at a time, one per group, added in ascending triangle
// order through shuffles (the same sums as one lane adding them in turn).
// Called by all 64 lanes.
__device__ inline bool cell_features_x4(const SurArgs& A, int32_t c, float* row, double nrm[3]) {
  const Grid& gr = A.g;
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const bool act = c >= 0;
  const Cell3 cc = unpack_cell(gr, act ? A.cell_ids[c] : 0);
  for (int q = g; q < 27; q += 4) {
    const int32_t i = cc.i + q % 3 - 1, j = cc.j + (q / 3) % 3 - 1, k = cc.k + q / 9 - 1;
    const bool in = act && i >= 0 && i < gr.nx && j >= 0 && j < gr.ny && k >= 0 && k < gr.nz;
    row[q] = in ? (float)A.alpha[i + (int64_t)gr.nx * (j + (int64_t)gr.ny * k)] : 0.f;
  }
  const double reach = 1.5 * gr.h;
  const double reach2 = reach * reach * (1.0 - 1e-12);
  const int32_t vs = act ? A.best_v[c] : -1;
  const bool final = act && vs >= 0 && vs < A.nv && A.best_d2[c] < reach2;
  const int32_t e0 = final ? A.vt_off[vs] : 0;
  const int32_t deg = final ? A.vt_off[vs + 1] - e0 : 0;
  // eight triangles per round (two per lane group), their loads issued together
  const int rounds = wave_max((deg + 7) >> 3);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < rounds; ++k) {
    double cx[2], cy[2], cz[2];
    int4 t4[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int m = 8 * k + 4 * hh + g;
      t4[hh] = m < deg ? A.tri4[A.vt_ids[e0 + m]] : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int m = 8 * k + 4 * hh + g;
      const P3 a = vtx(A.vtx4, t4[hh].x), b = vtx(A.vtx4, t4[hh].y), d = vtx(A.vtx4, t4[hh].z);
      const double ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
      const double wx = d.x - a.x, wy = d.y - a.y, wz = d.z - a.z;
      cx[hh] = m < deg ? uy * wz - uz * wy : 0.0;
      cy[hh] = m < deg ? uz * wx - ux * wz : 0.0;
      cz[hh] = m < deg ? ux * wy - uy * wx : 0.0;
    }
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const double x = __shfl(cx[hh], 16 * qq + r, 64), y = __shfl(cy[hh], 16 * qq + r, 64),
                     z = __shfl(cz[hh], 16 * qq + r, 64);
        if (8 * k + 4 * hh + qq < deg) {
          s0 += x;
          s1 += y;
          s2 += z;
        }
      }
  }
  if (final) {
    const double nl = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
    s0 /= nl;
    s1 /= nl;
    s2 /= nl;
  }
  nrm[0] = s0;
  nrm[1] = s1;
  nrm[2] = s2;
  if (g == 0) {
    row[27] = (float)s0;
    row[28] = (float)s1;
    row[29] = (float)s2;
    row[30] = row[31] = 0.f;
  }
  return final;
}

// Four wavefronts per workgroup, 16 cells per wavefront: feature rows in
// LDS, the network under the four symmetries of the error set, mean and
// spread; trusted cells are written, the others appended to the PPIC
// selection.
constexpr int kSurWaves = 4;
__global__ __launch_bounds__(64 * kSurWaves) void k_surrogate(CurvArgs A) {
  __shared__ NetLds L;
  __shared__ float F[kSurWaves][16][kFeat + 1];
  const float b3 = A.theta[kOffB3];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int32_t nif = min(A.S.counters[C_NIF], A.S.cell_cap);
  const double h = A.S.g.h;
  bool staged = false;
  // the loop bound is uniform over the workgroup
  for (int32_t blk = blockIdx.x * 16 * kSurWaves; blk < nif; blk += gridDim.x * 16 * kSurWaves) {
    const int32_t c = blk + 16 * wv + r;
    const bool act = c < nif;
    double nrm[3];
    const bool final = cell_features_x4(A.S, act ? c : -1, F[wv][r], nrm);
    if (!staged) {
      fill_net_lds(A.theta, L);
      staged = true;
    }
    __syncthreads();
    float y0 = 0.f, y1 = 0.f, y2 = 0.f, y3 = 0.f;
    // one symmetry at a time keeps the register footprint of one forward pass
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
      const int sym = t == 0 ? kErrSet[0] : (t == 1 ? kErrSet[1] : (t == 2 ? kErrSet[2] : kErrSet[3]));
      float x[2][4];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int f = 16 * ks + 4 * g + w;
          const int sg = kSym.sgn[sym][f];
          const float v = sg != 0 ? F[wv][r][kSym.src[sym][f]] : 0.f;
          x[ks][w] = sg < 0 ? -v : v;
        }
      bf16x8 xb[2];
      split_inputs(x, xb);
      const float yt = forward_tile_lds(L, b3, xb);
      y0 = t == 0 ? yt : y0;
      y1 = t == 1 ? yt : y1;
      y2 = t == 2 ? yt : y2;
      y3 = t == 3 ? yt : y3;
    }
    const float mean = ((y0 + y1) + (y2 + y3)) * 0.25f;
    const float spread = fmaxf(fmaxf(y0, y1), fmaxf(y2, y3)) - fminf(fminf(y0, y1), fminf(y2, y3));
    const bool fb = !final || !(spread <= A.bound);
    const bool push = g == 0 && act && fb;
    const uint64_t bal = __ballot(push);
    int32_t pos0 = 0;
    if (lane == 0 && bal) pos0 = atomicAdd(&A.counters[C_NSEL], (int32_t)__popcll(bal));
    pos0 = __shfl(pos0, 0, 64);
    if (g == 0 && act) {
      if (A.spread) A.spread[c] = spread;
      if (fb) {
        const int32_t pos = pos0 + (int32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (pos < A.S.cell_cap) A.sel[pos] = c;  // at most one entry per cell and call
      } else {
        A.kappa[c] = (double)mean / h;
        A.nx[c] = nrm[0];
        A.ny[c] = nrm[1];
        A.nz[c] = nrm[2];
        if (A.status) A.status[c] = (int32_t)FTC_CELL_SURROGATE;
      }
    }
    __syncthreads();
  }
}

SurArgs sur_args(const ftc_cells* ws, const Mesh& m, const double* alpha) {
  SurArgs S;
  S.g = ws->grid;
  S.nv = m.nv;
  S.cell_ids = ws->cell_ids;
  S.alpha = alpha;
  S.best_v = ws->best_v;
  S.best_d2 = ws->best_d2;
  S.vt_off = ws->vt_off;
  S.vt_ids = ws->vt_ids;
  S.tri4 = reinterpret_cast<const int4*>(ws->tri4);
  S.vtx4 = reinterpret_cast<const double2*>(ws->vtx4);
  S.counters = ws->counters;
  S.cell_cap = ws->cell_cap;
  return S;
}

}  // namespace

hipError_t launch_features(const ftc_cells* ws, const Mesh& m, const double* alpha, float* feat, int32_t* fstat,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(grid_blocks(ws->cell_cap, 256, 4096)), dim3(256), 0, s, sur_args(ws, m, alpha),
                     feat, fstat);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                              const int32_t* sym, int32_t n, float* y, hipStream_t s) {
  MlpArgs A{theta, X, rows, idx, sym, nullptr, n, 0.f, y, nullptr};
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid_blocks(n, 16, 8192)), dim3(64), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                                const int32_t* sym, const float* t, int32_t n, float* grad, float* loss, float* work,
                                hipStream_t s) {
  const int32_t nblk = grid_blocks(n, 32, kGradBlocks);
  MlpArgs A{theta, X, rows, idx, sym, t, n, 2.f / (float)n, nullptr, work};
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(64), 0, s, A);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNP + 1 + 255) / 256), dim3(256), 0, s, work, nblk, n, grad, loss);
  return hipGetLastError();
}

namespace {
// Scratch of the entry point that allocates nothing: the partial gradient
// rows of k_mlp_grad, as many as the caller's work buffer of
// ftc_mlp_loss_grad holds.  Each device holds its own copy for the life of
// the process.  In host code the array's name is not a device address: the
// kernels take the address hipGetSymbolAddress gives for the device.
__device__ __align__(256) float scratch[kGradBlocks * kPartStride];
constexpr int kMaxDevices = 64;
float* g_scratch[kMaxDevices] = {};  // the scratch's address on each device, once resolved
std::mutex g_scratch_mu;

// Address of the current device's scratch, resolved on its first use there.
hipError_t scratch_address(float** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<float*>(ptr);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}
}  // namespace

hipError_t launch_mlp_loss_grad_static(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                                       const int32_t* sym, const float* t, int32_t n, float* grad, float* loss,
                                       hipStream_t s) {
  float* work = nullptr;
  const hipError_t e = scratch_address(&work);
  if (e != hipSuccess) return e;
  return launch_mlp_loss_grad(theta, X, rows, idx, sym, t, n, grad, loss, work, s);
}

hipError_t launch_mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr, float beta1,
                           float beta2, float eps, hipStream_t s) {
  const float bc1 = (float)(1.0 - pow((double)beta1, step)), bc2 = (float)(1.0 - pow((double)beta2, step));
  hipLaunchKernelGGL(k_mlp_adam, dim3((kNP + 255) / 256), dim3(256), 0, s, theta, m, v, grad, lr, beta1, beta2, eps,
                     bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_surrogate(const ftc_cells* ws, const Mesh& m, const double* alpha, const float* theta, float bound,
                            const PPICParams& p, double* kappa, double* nx, double* ny, double* nz, float* spread,
                            int32_t* status, int32_t* n_fallback, hipStream_t s) {
  CurvArgs A{sur_args(ws, m, alpha), theta, bound, kappa, nx, ny, nz, spread, status, ws->sel_cells, ws->counters};
  time_start(ws, FTC_KERNEL_SURROGATE, s);
  hipLaunchKernelGGL(k_surrogate, dim3(grid_blocks(ws->cell_cap, 16 * kSurWaves, 8192)), dim3(64 * kSurWaves), 0, s, A);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = launch_ppic_cells(ws, m, p, kappa, nx, ny, nz, nullptr, status, nullptr, ws->sel_cells, n_fallback, s);
  time_stop(ws, FTC_KERNEL_SURROGATE, s);
  return e;
}

}  // namespace ftc
