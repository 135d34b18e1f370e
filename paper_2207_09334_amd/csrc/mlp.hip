// Surrogate network on gfx950: a 4-layer perceptron (3 exact-erf GELU hidden layers, linear
// output) whose products run on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation; weights are kept as an FP32 master copy and two BF16 shadows; Adam in FP32.
//
// Every product is C[M x N] = A B^T with both operands stored K-contiguous (A: M rows of K,
// B: N rows of K), so each operand tile arrives with 16-byte vector loads along K.  To keep it
// that way the network stores, beside each row-major activation it produces, its transpose
// (written by the producing product's epilogue), and keeps both W and W^T as BF16 shadows:
//   forward      Z_l = H_{l-1} W_l        A = H_{l-1} (rows x in),   B = W_l^T (out x in)
//   input grad   dH  = dZ_l W_l^T         A = dZ_l (rows x out),     B = W_l   (in x out)
//   weight grad  [dW_l; db_l] = [H^T; 1] dZ_l   A = [H_{l-1}^T; ones] (in+1 x rows),
//                                               B = dZ_l^T (out x rows)
// The row of ones appended to each transposed input makes the bias gradient (a column sum
// of dZ) the last row of the weight-gradient product, which lands exactly where the bias
// follows the weight in the parameter vector.  Widths are padded to multiples of 32 with zero
// weights, so padded activations are exactly zero.
//
// Tiling: a workgroup of 4 wavefronts computes a 64 x 64 tile of C, each wavefront a 32 x 32
// quarter as 2 x 2 MFMA tiles of 16 x 16, stepping K by 128 (or 64, 32) through two LDS buffers:
// the next K-step's operands are loaded into registers while the matrix cores work on the
// current one, then stored to the other buffer (one barrier per K-step).  The weight
// gradients (K = the minibatch rows) split K into chunks of 512 rows computed by separate
// workgroups into FP32 partials, laid out like the parameters, that Adam adds in a fixed
// order (or one more kernel, when the gradient itself is asked for).  Operand layouts
// of the 16x16x32 BF16 MFMA: lane l supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j]
// [l % 16], j = 0..7, and receives C[4 (l / 16) + r][l % 16], r = 0..3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64;   // workgroup tile
constexpr int kWidthPad = 32;       // widths are padded to multiples of this (the MFMA's K)
constexpr int kSplitRows = 512;     // K chunk of the weight-gradient products

enum Epilogue { kFwdGelu = 0, kLinear = 1, kBwdGelu = 2, kPartial = 3 };

struct GemmArgs {
    const bf16* A;
    long lda;             // A(m, k) = A[m * lda + k], m < M
    const bf16* B;
    long ldb;             // B(n, k) = B[n * ldb + k], n < N
    int M, N, K;          // K: a multiple of the K-step; lda, ldb: multiples of 8
    int k_chunk;          // K range of workgroup z: [z k_chunk, (z + 1) k_chunk)
    int n_real;           // columns below n_real get the bias, the transposed and FP32 outputs
    const float* bias;    // [n_real] (forward epilogues)
    float* Cf;            // FP32 output: Cf[m * ldcf + n] (+ z * part_stride for partials)
    long ldcf, part_stride;
    bf16* Cb;             // BF16 row-major output: Cb[m * ldcb + n], n < N
    long ldcb;
    bf16* Ct;             // BF16 transposed output: Ct[n * ldct + m], n < n_real
    long ldct;
    const float* Z;       // pre-activation Z[m * ldz + n] (backward GELU)
    long ldz;
    int nbx, nby, tiles;  // column tiles, row tiles and their product with the K-splits
    // linear output with the loss (T non-null): dY = 2 (Y - T) / (rows n_real) as BF16, row-major
    // dY[m * lddy + n] for n < N (zero beyond n_real and below M beyond `rows`) and transposed
    // dYt[n * lddyt + m] for n < n_real; the sum of squares of Y - T per row tile in loss_part
    const float* T;       // targets T[m * n_real + n], m < rows
    bf16* dY;
    long lddy;
    bf16* dYt;
    long lddyt;
    double* loss_part;
    int rows;
};

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ uint32_t pack2(bf16 lo, bf16 hi) {
    return (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}

constexpr int kMaxBK = 128;

// One workgroup's 64 x 64 tile (column tile bx, row tile by, K-split bz) of the product g,
// staged through As / Bs (two buffers of 64 rows of BK + 8 elements each, at least).
template <int EPI, int BK>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int bx, int by, int bz, bf16* __restrict__ As,
                                          bf16* __restrict__ Bs) {
    constexpr int LDK = BK + 8;               // LDS row pitch in elements (16-byte reads stay conflict-free)
    constexpr int CPR = BK / 8;               // 16-byte chunks per tile row
    constexpr int LOADS = kBM * CPR / 256;    // 16-byte loads per thread per operand per K-step
    constexpr int BUF = kBM * LDK;            // elements of one buffer
    static_assert(BK <= kMaxBK, "K-step deeper than the LDS buffers");
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = by * kBM, n0 = bx * kBN;
    const int kbeg = bz * g.k_chunk;
    const int kend = min(g.K, kbeg + g.k_chunk);
    const int nk = (kend - kbeg) / BK;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

    uint4 ra[LOADS], rb[LOADS];
    auto gload = [&](int kb) {
#pragma unroll
        for (int i = 0; i < LOADS; ++i) {
            const int c = t + 256 * i, row = c / CPR, kc = (c % CPR) * 8;
            const int m = m0 + row, n = n0 + row;
            ra[i] = m < g.M ? *reinterpret_cast<const uint4*>(g.A + (long)m * g.lda + kb + kc) : uint4{0u, 0u, 0u, 0u};
            rb[i] = n < g.N ? *reinterpret_cast<const uint4*>(g.B + (long)n * g.ldb + kb + kc) : uint4{0u, 0u, 0u, 0u};
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < LOADS; ++i) {
            const int c = t + 256 * i, row = c / CPR, kc = (c % CPR) * 8;
            *reinterpret_cast<uint4*>(&As[buf * BUF + row * LDK + kc]) = ra[i];
            *reinterpret_cast<uint4*>(&Bs[buf * BUF + row * LDK + kc]) = rb[i];
        }
    };

    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int r16 = lane & 15, k8 = (lane >> 4) * 8;
    // linear output with the loss: the targets this thread's outputs meet, loaded before the
    // K-loop so that their latency hides behind it
    float tgt[2][2][4] = {};
    if (EPI == kLinear && g.T) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int mb = m0 + wm + i * 16 + (lane >> 4) * 4, n = n0 + wn + j * 16 + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (n < g.n_real && mb + r < g.rows) tgt[i][j][r] = g.T[(long)(mb + r) * g.n_real + n];
            }
    }

    if (nk > 0) {
        gload(kbeg);
        sstore(0);
    }
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
        const int cur = it & 1;
        if (it + 1 < nk) gload(kbeg + (it + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 32) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(&As[cur * BUF + (wm + i * 16 + r16) * LDK + ks + k8]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur * BUF + (wn + j * 16 + r16) * LDK + ks + k8]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (it + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    double lsum = 0.0;   // linear output with the loss: this thread's squares of Y - T
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int mb = m0 + wm + i * 16 + (lane >> 4) * 4;   // rows mb .. mb + 3
            const int n = n0 + wn + j * 16 + (lane & 15);
            if (n >= g.N) continue;
            if (EPI == kPartial) {
                if (n >= g.n_real) continue;
                float* out = g.Cf + bz * g.part_stride;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (mb + r < g.M) out[(long)(mb + r) * g.ldcf + n] = acc[i][j][r];
            } else if (EPI == kLinear) {
                if (!g.T) {
                    if (n >= g.n_real) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (mb + r < g.M) g.Cf[(long)(mb + r) * g.ldcf + n] = acc[i][j][r] + g.bias[n];
                } else {
                    // M is a multiple of 64 here (padded minibatch rows)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = mb + r;
                        float d = 0.0f;
                        if (n < g.n_real) {
                            const float y = acc[i][j][r] + g.bias[n];
                            g.Cf[(long)row * g.ldcf + n] = y;
                            if (row < g.rows) {
                                d = y - tgt[i][j][r];
                                lsum += (double)d * (double)d;
                            }
                        }
                        // rows * n_real formed in float (one rounding of the exact product, as the
                        // integer product's conversion would give) cannot overflow 32 bits
                        const bf16 v = (bf16)(2.0f * d / ((float)g.rows * (float)g.n_real));
                        g.dY[(long)row * g.lddy + n] = v;
                        if (n < g.n_real) g.dYt[(long)n * g.lddyt + row] = v;
                    }
                }
            } else {
                // forward / backward GELU: M is a multiple of 64 (padded minibatch rows)
                bf16 hv[4];
                const float bn = (EPI == kFwdGelu && n < g.n_real) ? g.bias[n] : 0.0f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const long o = (long)(mb + r) * g.ldcb + n;
                    if (EPI == kFwdGelu) {
                        const float z = acc[i][j][r] + bn;
                        g.Cf[(long)(mb + r) * g.ldcf + n] = z;
                        hv[r] = (bf16)gelu(z);
                    } else {
                        hv[r] = (bf16)(acc[i][j][r] * gelu_grad(g.Z[(long)(mb + r) * g.ldz + n]));
                    }
                    g.Cb[o] = hv[r];
                }
                if (n < g.n_real)
                    *reinterpret_cast<uint2*>(g.Ct + (long)n * g.ldct + mb) = uint2{pack2(hv[0], hv[1]), pack2(hv[2], hv[3])};
            }
        }
    if (EPI == kLinear && g.T) {
        // the row tile's loss partial, summed over the workgroup in a fixed order (the K-loop
        // ended with a barrier, so As is free)
        double* red = reinterpret_cast<double*>(As);
        red[t] = lsum;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (t == 0) g.loss_part[by] = red[0];
    }
}

template <int EPI, int BK>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) bf16 As[2 * kBM * (BK + 8)];
    __shared__ __attribute__((aligned(16))) bf16 Bs[2 * kBN * (BK + 8)];
    gemm_tile<EPI, BK>(g, blockIdx.x, blockIdx.y, blockIdx.z, As, Bs);
}

// Two independent products in one launch (the backward's weight gradient of a layer and the
// gradient into its input both read only that layer's dZ): workgroups below g1's tile count
// take g1's tiles, the rest g2's, so both run side by side on the chip without a second
// stream.  Tiles are numbered column fastest, then row, then split.
template <int E1, int BK1, int E2, int BK2>
__global__ void __launch_bounds__(256) gemm_pair_kernel(GemmArgs g1, GemmArgs g2) {
    constexpr int BK = BK1 > BK2 ? BK1 : BK2;
    __shared__ __attribute__((aligned(16))) bf16 As[2 * kBM * (BK + 8)];
    __shared__ __attribute__((aligned(16))) bf16 Bs[2 * kBN * (BK + 8)];
    int tile = blockIdx.x;
    if (tile < g1.tiles) {
        gemm_tile<E1, BK1>(g1, tile % g1.nbx, (tile / g1.nbx) % g1.nby, tile / (g1.nbx * g1.nby), As, Bs);
    } else {
        tile -= g1.tiles;
        gemm_tile<E2, BK2>(g2, tile % g2.nbx, (tile / g2.nbx) % g2.nby, tile / (g2.nbx * g2.nby), As, Bs);
    }
}

// Sum of `splits` FP32 partials in split order: out[i] = part[0][i] + part[1][i] + ...
__global__ void splitk_sum_kernel(const float* part, long stride, int splits, float* out, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = part[i];
    for (int z = 1; z < splits; ++z) s += part[z * stride + i];
    out[i] = s;
}

// Where each layer's weights sit in the parameter vector and in the two BF16 shadows.
struct ShadowMap {
    long off_w[4], off_b[4];
    int K[4], N[4], Kp[4], Np[4];
    bf16* w[4];    // [Kp][Np]: W as stored (input-gradient products)
    bf16* wt[4];   // [Np][Kp]: W^T (forward products)
};

__device__ __forceinline__ void write_shadow(const ShadowMap& s, long i, float v) {
#pragma unroll
    for (int l = 0; l < 4; ++l)
        if (i >= s.off_w[l] && i < s.off_b[l]) {
            const long q = i - s.off_w[l];
            const int k = (int)(q / s.N[l]), n = (int)(q % s.N[l]);
            s.w[l][(long)k * s.Np[l] + n] = (bf16)v;
            s.wt[l][(long)n * s.Kp[l] + k] = (bf16)v;
        }
}

// Adam on the FP32 master copy; refreshes the BF16 shadows of the weight entries.  The
// gradient is the sum of `splits` partial gradients laid out like the parameters, `stride`
// apart, added in split order (the order splitk_sum_kernel uses).
__global__ void adam_kernel(float* p, float* m, float* v, const float* grad, int splits, long stride, ShadowMap sm,
                            long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = grad[i];
    for (int z = 1; z < splits; ++z) gi += grad[z * stride + i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    write_shadow(sm, i, pi);
}

__global__ void shadow_kernel(const float* p, ShadowMap sm, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) write_shadow(sm, i, p[i]);
}

// Minibatch rows r < padded_rows: X_b[r][c] = bf16(X[src][c]) (zero beyond n_in and beyond
// `rows`), X_t[c][r] for c < n_in, T_b[r] = T[src]; src = idx[r], or r when idx is NULL.
__global__ void gather_kernel(const float* X, const float* T, const int* idx, bf16* Xb, long ldx, bf16* Xt, long ldt,
                              float* Tb, int rows, int padded_rows, int n_in, int n_out) {
    const int r = blockIdx.x;
    if (r >= padded_rows) return;
    const long src = r < rows ? (idx ? (long)idx[r] : (long)r) : -1;
    for (int c = threadIdx.x; c < ldx; c += blockDim.x) {
        const bf16 v = (src >= 0 && c < n_in) ? (bf16)X[src * n_in + c] : (bf16)0.0f;
        Xb[(long)r * ldx + c] = v;
        if (c < n_in) Xt[(long)c * ldt + r] = v;
    }
    if (T)
        for (int c = threadIdx.x; c < n_out; c += blockDim.x) Tb[(long)r * n_out + c] = src >= 0 ? T[src * n_out + c] : 0.0f;
}

__global__ void fill_kernel(bf16* p, long n, float v) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (bf16)v;
}

uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int pad_width(int w) { return (w + kWidthPad - 1) / kWidthPad * kWidthPad; }

}  // namespace

using cronos::fail;

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(CRONOS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct cronos_mlp_t {
    int sizes[5];
    int wp[5];             // widths padded to multiples of 32
    int max_rows = 0;      // padded to a multiple of 64; row pitch of every transposed buffer
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    long n_params = 0;
    long off_w[4], off_b[4];
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    bf16 *w[4] = {}, *wt[4] = {};      // BF16 shadows [wp[l]][wp[l+1]] and [wp[l+1]][wp[l]]
    ShadowMap smap;
    int step = 0;
    // activations for max_rows rows (row-major [rows][width]; transposed [width (+1)][max_rows])
    float* xin = nullptr;              // [rows][sizes[0]] FP32 staging of uploaded inputs
    bf16* x = nullptr;                 // [rows][wp[0]]
    bf16* xt = nullptr;                // [sizes[0] + 1][max_rows], last row ones
    float* z[3] = {};                  // [rows][wp[l+1]]
    bf16* h[3] = {};
    bf16* ht[3] = {};                  // [sizes[l+1] + 1][max_rows], last row ones
    float* y = nullptr;                // [rows][sizes[4]]
    float* t = nullptr;
    bf16* dy = nullptr;                // [rows][wp[4]]
    bf16* dyt = nullptr;               // [sizes[4]][max_rows]
    bf16* dz[3] = {};                  // [rows][wp[l+1]]
    bf16* dzt[3] = {};                 // [sizes[l+1]][max_rows]
    float* part_w = nullptr;           // [splits][n_params] split-K partials of the weight gradients
    int grad_splits = 1;               // partials Adam adds (1: the gradient is in grad)
    double* part = nullptr;            // loss partials
    // training data
    float* data_x = nullptr;
    float* data_t = nullptr;
    int* idx = nullptr;
    long data_rows = 0;
};

namespace {

// Tile counts of g over `splits` K-chunks, and the K-step it takes (128, 64 or 32: the
// deepest that divides K and the chunk).
int prepare(GemmArgs& g, int splits) {
    g.nbx = (g.N + kBN - 1) / kBN;
    g.nby = (g.M + kBM - 1) / kBM;
    g.tiles = g.nbx * g.nby * splits;
    if (splits == 1) g.k_chunk = g.K;
    if (g.K % 128 == 0 && g.k_chunk % 128 == 0) return 128;
    if (g.K % 64 == 0 && g.k_chunk % 64 == 0) return 64;
    return 32;
}

template <int EPI>
hipError_t gemm(hipStream_t st, GemmArgs g, int splits = 1) {
    const int bk = prepare(g, splits);
    const dim3 grid(g.nbx, g.nby, splits);
    if (bk == 128)
        hipLaunchKernelGGL((gemm_kernel<EPI, 128>), grid, dim3(256), 0, st, g);
    else if (bk == 64)
        hipLaunchKernelGGL((gemm_kernel<EPI, 64>), grid, dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((gemm_kernel<EPI, 32>), grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

template <int E1, int BK1, int E2>
void launch_pair2(hipStream_t st, const GemmArgs& g1, const GemmArgs& g2, int bk2) {
    const dim3 grid((unsigned)(g1.tiles + g2.tiles));
    if (bk2 == 128)
        hipLaunchKernelGGL((gemm_pair_kernel<E1, BK1, E2, 128>), grid, dim3(256), 0, st, g1, g2);
    else if (bk2 == 64)
        hipLaunchKernelGGL((gemm_pair_kernel<E1, BK1, E2, 64>), grid, dim3(256), 0, st, g1, g2);
    else
        hipLaunchKernelGGL((gemm_pair_kernel<E1, BK1, E2, 32>), grid, dim3(256), 0, st, g1, g2);
}

// g1 over splits1 K-chunks and g2 (one chunk) in one launch.
template <int E1, int E2>
hipError_t gemm_pair(hipStream_t st, GemmArgs g1, int splits1, GemmArgs g2) {
    const int bk1 = prepare(g1, splits1), bk2 = prepare(g2, 1);
    if (bk1 == 128)
        launch_pair2<E1, 128, E2>(st, g1, g2, bk2);
    else if (bk1 == 64)
        launch_pair2<E1, 64, E2>(st, g1, g2, bk2);
    else
        launch_pair2<E1, 32, E2>(st, g1, g2, bk2);
    return hipGetLastError();
}

void free_mlp(cronos_mlp_t* q) {
    std::vector<void*> ptrs = {q->p, q->m, q->v, q->grad, q->xin, q->x, q->xt, q->y, q->t, q->dy, q->dyt, q->part_w,
                               q->part, q->data_x, q->data_t, q->idx};
    for (int l = 0; l < 4; ++l) {
        ptrs.push_back(q->w[l]);
        ptrs.push_back(q->wt[l]);
    }
    for (int l = 0; l < 3; ++l) {
        ptrs.push_back(q->z[l]);
        ptrs.push_back(q->h[l]);
        ptrs.push_back(q->ht[l]);
        ptrs.push_back(q->dz[l]);
        ptrs.push_back(q->dzt[l]);
    }
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (q->own_stream && q->stream) (void)hipStreamDestroy(q->stream);
}

// Forward over `rows` (<= max_rows, padded to 64) rows already in q->x; with_loss: the output
// product's epilogue also forms the loss partials and dY from the targets in q->t.
cronos_status forward_dev(cronos_mlp_t* q, int rows, bool with_loss) {
    const int P = (rows + 63) / 64 * 64;
    const long R = q->max_rows;
    const bf16* in = q->x;
    for (int l = 0; l < 3; ++l) {
        GemmArgs g{};
        g.A = in;
        g.lda = q->wp[l];
        g.B = q->wt[l];
        g.ldb = q->wp[l];
        g.M = P;
        g.N = q->wp[l + 1];
        g.K = q->wp[l];
        g.n_real = q->sizes[l + 1];
        g.bias = q->p + q->off_b[l];
        g.Cf = q->z[l];
        g.ldcf = q->wp[l + 1];
        g.Cb = q->h[l];
        g.ldcb = q->wp[l + 1];
        g.Ct = q->ht[l];
        g.ldct = R;
        HIP_TRY(gemm<kFwdGelu>(q->stream, g));
        in = q->h[l];
    }
    GemmArgs g{};
    g.A = in;
    g.lda = q->wp[3];
    g.B = q->wt[3];
    g.ldb = q->wp[3];
    g.M = P;
    g.N = q->wp[4];
    g.K = q->wp[3];
    g.n_real = q->sizes[4];
    g.bias = q->p + q->off_b[3];
    g.Cf = q->y;
    g.ldcf = q->sizes[4];
    if (with_loss) {
        g.T = q->t;
        g.dY = q->dy;
        g.lddy = q->wp[4];
        g.dYt = q->dyt;
        g.lddyt = R;
        g.loss_part = q->part;
        g.rows = rows;
    }
    HIP_TRY(gemm<kLinear>(q->stream, g));
    return CRONOS_OK;
}

// Loss and gradients for `rows` rows whose inputs are in q->x / q->xt and targets in q->t.
// With more than one K-split the weight gradients stay as per-split partials (q->part_w,
// laid out like the parameters) for Adam to add, unless sum_grads asks for them in q->grad.
cronos_status backward_dev(cronos_mlp_t* q, int rows, bool sum_grads) {
    const int P = (rows + 63) / 64 * 64;
    const long R = q->max_rows;
    const int splits = (P + kSplitRows - 1) / kSplitRows;
    const bf16* dnext = q->dy;     // [P][wp[l+1]]
    const bf16* dnext_t = q->dyt;  // [sizes[l+1]][R]
    for (int l = 3; l >= 0; --l) {
        const int K = q->sizes[l], N = q->sizes[l + 1];
        // [dW_l; db_l] = [H_in^T; 1] dZ_l : (K + 1) x N, summed over the P rows
        GemmArgs g{};
        g.A = l ? q->ht[l - 1] : q->xt;
        g.lda = R;
        g.B = dnext_t;
        g.ldb = R;
        g.M = K + 1;
        g.N = N;
        g.K = P;
        g.k_chunk = kSplitRows;
        g.n_real = N;
        g.ldcf = N;
        if (splits == 1) {
            g.Cf = q->grad + q->off_w[l];
        } else {
            g.Cf = q->part_w + q->off_w[l];
            g.part_stride = q->n_params;
        }
        if (l == 0) HIP_TRY(gemm<kPartial>(q->stream, g, splits));
        if (l) {
            // dZ_{l-1} = (dZ_l W_l^T) * gelu'(Z_{l-1}) : (P x wp[l+1]) (wp[l+1] x wp[l])
            GemmArgs d{};
            d.A = dnext;
            d.lda = q->wp[l + 1];
            d.B = q->w[l];
            d.ldb = q->wp[l + 1];
            d.M = P;
            d.N = q->wp[l];
            d.K = q->wp[l + 1];
            d.n_real = K;
            d.Cb = q->dz[l - 1];
            d.ldcb = q->wp[l];
            d.Ct = q->dzt[l - 1];
            d.ldct = R;
            d.Z = q->z[l - 1];
            d.ldz = q->wp[l];
            // both read dZ_l only: one launch for the pair
            HIP_TRY((gemm_pair<kPartial, kBwdGelu>(q->stream, g, splits, d)));
            dnext = q->dz[l - 1];
            dnext_t = q->dzt[l - 1];
        }
    }
    q->grad_splits = splits;
    if (splits > 1 && sum_grads) {
        hipLaunchKernelGGL(splitk_sum_kernel, dim3((unsigned)((q->n_params + 255) / 256)), dim3(256), 0, q->stream,
                           q->part_w, q->n_params, splits, q->grad, q->n_params);
        HIP_TRY(hipGetLastError());
        q->grad_splits = 1;
    }
    return CRONOS_OK;
}

// Rows of the minibatch from device arrays (idx == nullptr: the first `rows` rows in order).
cronos_status gather_rows(cronos_mlp_t* q, const float* X, const float* T, const int* idx, int rows) {
    const int P = (rows + 63) / 64 * 64;
    hipLaunchKernelGGL(gather_kernel, dim3(P), dim3(128), 0, q->stream, X, T, idx, q->x, (long)q->wp[0], q->xt,
                       (long)q->max_rows, q->t, rows, P, q->sizes[0], q->sizes[4]);
    HIP_TRY(hipGetLastError());
    return CRONOS_OK;
}

cronos_status upload_rows(cronos_mlp_t* q, const float* x, const float* t, int rows) {
    const int n_in = q->sizes[0], n_out = q->sizes[4];
    HIP_TRY(hipMemcpyAsync(q->xin, x, (size_t)rows * n_in * sizeof(float), hipMemcpyHostToDevice, q->stream));
    // targets: the loss reads rows below `rows` only
    if (t) HIP_TRY(hipMemcpyAsync(q->t, t, (size_t)rows * n_out * sizeof(float), hipMemcpyHostToDevice, q->stream));
    return gather_rows(q, q->xin, nullptr, nullptr, rows);
}

cronos_status adam_dev(cronos_mlp_t* q, double lr, double b1, double b2, double eps) {
    q->step += 1;
    const float c1 = (float)(1.0 - std::pow(b1, q->step)), c2 = (float)(1.0 - std::pow(b2, q->step));
    const bool parts = q->grad_splits > 1;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((q->n_params + 255) / 256)), dim3(256), 0, q->stream, q->p, q->m,
                       q->v, parts ? q->part_w : q->grad, parts ? q->grad_splits : 1, q->n_params, q->smap,
                       q->n_params, (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
    HIP_TRY(hipGetLastError());
    return CRONOS_OK;
}

double loss_from_parts(cronos_mlp_t* q, int rows, cronos_status* st) {
    const int nb = (rows + 63) / 64;   // one partial per 64-row tile of the output product
    std::vector<double> h(nb);
    *st = CRONOS_OK;
    if (hipMemcpyAsync(h.data(), q->part, nb * sizeof(double), hipMemcpyDeviceToHost, q->stream) != hipSuccess ||
        hipStreamSynchronize(q->stream) != hipSuccess) {
        *st = fail(CRONOS_EDEVICE, "mlp: loss read-back failed");
        return 0.0;
    }
    double s = 0.0;
    for (double v : h) s += v;
    return s / ((double)rows * q->sizes[4]);
}

}  // namespace

extern "C" cronos_status cronos_mlp_create(const int32_t* sizes, const double* params, int32_t max_rows, int32_t device,
                                           void* stream, cronos_mlp* out) {
    cronos::clear_error();
    if (!sizes || !params || !out || max_rows < 1) return fail(CRONOS_EINVAL, "mlp_create: bad arguments");
    *out = nullptr;
    for (int l = 0; l < 5; ++l)
        if (sizes[l] < 1 || sizes[l] > 4096) return fail(CRONOS_EINVAL, "mlp_create: layer width out of range");
    if (max_rows > (1 << 20)) return fail(CRONOS_EINVAL, "mlp_create: max_rows above 2^20");
    auto* q = new (std::nothrow) cronos_mlp_t;
    if (!q) return fail(CRONOS_ENOMEM, "mlp_create: out of memory");
    for (int l = 0; l < 5; ++l) {
        q->sizes[l] = sizes[l];
        q->wp[l] = pad_width(sizes[l]);
    }
    q->max_rows = (max_rows + 63) / 64 * 64;
    q->device = device;
    long off = 0;
    for (int l = 0; l < 4; ++l) {
        q->off_w[l] = off;
        off += (long)sizes[l] * sizes[l + 1];
        q->off_b[l] = off;
        off += sizes[l + 1];
    }
    q->n_params = off;
    auto st = [&]() -> cronos_status {
        HIP_TRY(hipSetDevice(device));
        if (stream) {
            q->stream = (hipStream_t)stream;
        } else {
            HIP_TRY(hipStreamCreateWithFlags(&q->stream, hipStreamNonBlocking));
            q->own_stream = true;
        }
        const long n = q->n_params, R = q->max_rows;
        auto dmalloc = [&](auto** ptr, size_t count) -> hipError_t {
            return hipMalloc((void**)ptr, std::max<size_t>(count, 1) * sizeof(**ptr));
        };
        HIP_TRY(dmalloc(&q->p, n));
        HIP_TRY(dmalloc(&q->m, n));
        HIP_TRY(dmalloc(&q->v, n));
        HIP_TRY(dmalloc(&q->grad, n));
        for (int l = 0; l < 4; ++l) {
            const size_t cnt = (size_t)q->wp[l] * q->wp[l + 1];
            HIP_TRY(dmalloc(&q->w[l], cnt));
            HIP_TRY(dmalloc(&q->wt[l], cnt));
            HIP_TRY(hipMemsetAsync(q->w[l], 0, cnt * sizeof(bf16), q->stream));
            HIP_TRY(hipMemsetAsync(q->wt[l], 0, cnt * sizeof(bf16), q->stream));
            q->smap.off_w[l] = q->off_w[l];
            q->smap.off_b[l] = q->off_b[l];
            q->smap.K[l] = sizes[l];
            q->smap.N[l] = sizes[l + 1];
            q->smap.Kp[l] = q->wp[l];
            q->smap.Np[l] = q->wp[l + 1];
            q->smap.w[l] = q->w[l];
            q->smap.wt[l] = q->wt[l];
        }
        HIP_TRY(dmalloc(&q->xin, R * sizes[0]));
        HIP_TRY(dmalloc(&q->x, R * q->wp[0]));
        HIP_TRY(dmalloc(&q->xt, (sizes[0] + 1) * R));
        for (int l = 0; l < 3; ++l) {
            HIP_TRY(dmalloc(&q->z[l], R * q->wp[l + 1]));
            HIP_TRY(dmalloc(&q->h[l], R * q->wp[l + 1]));
            HIP_TRY(dmalloc(&q->ht[l], (sizes[l + 1] + 1) * R));
            HIP_TRY(dmalloc(&q->dz[l], R * q->wp[l + 1]));
            HIP_TRY(dmalloc(&q->dzt[l], sizes[l + 1] * R));
        }
        HIP_TRY(dmalloc(&q->y, R * sizes[4]));
        HIP_TRY(dmalloc(&q->t, R * sizes[4]));
        HIP_TRY(dmalloc(&q->dy, R * q->wp[4]));
        HIP_TRY(dmalloc(&q->dyt, sizes[4] * R));
        HIP_TRY(dmalloc(&q->part, (R * q->wp[4] + 255) / 256));
        // split-K partials of the weight gradients at max_rows rows, laid out like the parameters
        const int splits = (int)((R + kSplitRows - 1) / kSplitRows);
        if (splits > 1) HIP_TRY(dmalloc(&q->part_w, (size_t)splits * n));
        // the appended row of ones of every transposed layer input
        auto ones = [&](bf16* base, int row) -> hipError_t {
            hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, q->stream, base + (long)row * R, R,
                               1.0f);
            return hipGetLastError();
        };
        HIP_TRY(ones(q->xt, sizes[0]));
        for (int l = 0; l < 3; ++l) HIP_TRY(ones(q->ht[l], sizes[l + 1]));
        std::vector<float> hp(n), zero(n, 0.0f);
        for (long i = 0; i < n; ++i) hp[i] = (float)params[i];
        HIP_TRY(hipMemcpyAsync(q->p, hp.data(), n * sizeof(float), hipMemcpyHostToDevice, q->stream));
        HIP_TRY(hipMemcpyAsync(q->m, zero.data(), n * sizeof(float), hipMemcpyHostToDevice, q->stream));
        HIP_TRY(hipMemcpyAsync(q->v, zero.data(), n * sizeof(float), hipMemcpyHostToDevice, q->stream));
        HIP_TRY(hipMemcpyAsync(q->grad, zero.data(), n * sizeof(float), hipMemcpyHostToDevice, q->stream));
        hipLaunchKernelGGL(shadow_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, q->stream, q->p, q->smap, n);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(q->stream));
        return CRONOS_OK;
    }();
    if (st != CRONOS_OK) {
        free_mlp(q);
        delete q;
        return st;
    }
    *out = q;
    return CRONOS_OK;
}

extern "C" void cronos_mlp_destroy(cronos_mlp q) {
    if (!q) return;
    (void)hipSetDevice(q->device);
    (void)hipStreamSynchronize(q->stream);
    free_mlp(q);
    delete q;
}

extern "C" cronos_status cronos_mlp_get_params(cronos_mlp q, double* params) {
    if (!q || !params) return fail(CRONOS_EINVAL, "mlp_get_params: NULL argument");
    std::vector<float> hp(q->n_params);
    HIP_TRY(hipSetDevice(q->device));
    HIP_TRY(hipMemcpyAsync(hp.data(), q->p, q->n_params * sizeof(float), hipMemcpyDeviceToHost, q->stream));
    HIP_TRY(hipStreamSynchronize(q->stream));
    for (long i = 0; i < q->n_params; ++i) params[i] = hp[i];
    return CRONOS_OK;
}

extern "C" cronos_status cronos_mlp_forward(cronos_mlp q, const float* x, int64_t rows, float* y) {
    cronos::clear_error();
    if (!q || !x || !y || rows < 0) return fail(CRONOS_EINVAL, "mlp_forward: bad arguments");
    HIP_TRY(hipSetDevice(q->device));
    const int n_out = q->sizes[4];
    for (int64_t r0 = 0; r0 < rows; r0 += q->max_rows) {
        const int r = (int)std::min<int64_t>(q->max_rows, rows - r0);
        cronos_status st = upload_rows(q, x + r0 * q->sizes[0], nullptr, r);
        if (st != CRONOS_OK) return st;
        st = forward_dev(q, r, false);
        if (st != CRONOS_OK) return st;
        HIP_TRY(hipMemcpyAsync(y + r0 * n_out, q->y, (size_t)r * n_out * sizeof(float), hipMemcpyDeviceToHost, q->stream));
        HIP_TRY(hipStreamSynchronize(q->stream));
    }
    return CRONOS_OK;
}

extern "C" cronos_status cronos_mlp_loss_grad(cronos_mlp q, const float* x, const float* t, int32_t rows, double* loss,
                                              double* grads) {
    cronos::clear_error();
    if (!q || !x || !t || rows < 1 || rows > q->max_rows) return fail(CRONOS_EINVAL, "mlp_loss_grad: bad arguments");
    HIP_TRY(hipSetDevice(q->device));
    cronos_status st = upload_rows(q, x, t, rows);
    if (st == CRONOS_OK) st = forward_dev(q, rows, true);
    if (st == CRONOS_OK) st = backward_dev(q, rows, true);
    if (st != CRONOS_OK) return st;
    const double l = loss_from_parts(q, rows, &st);
    if (st != CRONOS_OK) return st;
    if (loss) *loss = l;
    if (grads) {
        std::vector<float> hg(q->n_params);
        HIP_TRY(hipMemcpyAsync(hg.data(), q->grad, q->n_params * sizeof(float), hipMemcpyDeviceToHost, q->stream));
        HIP_TRY(hipStreamSynchronize(q->stream));
        for (long i = 0; i < q->n_params; ++i) grads[i] = hg[i];
    }
    return CRONOS_OK;
}

extern "C" cronos_status cronos_mlp_adam(cronos_mlp q, double lr, double beta1, double beta2, double eps) {
    cronos::clear_error();
    if (!q) return fail(CRONOS_EINVAL, "mlp_adam: NULL handle");
    HIP_TRY(hipSetDevice(q->device));
    cronos_status st = adam_dev(q, lr, beta1, beta2, eps);
    if (st != CRONOS_OK) return st;
    HIP_TRY(hipStreamSynchronize(q->stream));
    return CRONOS_OK;
}

extern "C" cronos_status cronos_mlp_train(cronos_mlp q, const float* x, const float* t, int64_t rows, int32_t batch,
                                          int32_t epochs, double lr, double lr_final, uint64_t seed, double* epoch_loss) {
    cronos::clear_error();
    if (!q || !x || !t || rows < 1 || batch < 1 || batch > q->max_rows || epochs < 0 || !(lr >= 0.0) ||
        !(lr_final >= 0.0))
        return fail(CRONOS_EINVAL, "mlp_train: bad arguments");
    HIP_TRY(hipSetDevice(q->device));
    const int n_in = q->sizes[0], n_out = q->sizes[4];
    if (q->data_rows != rows) {
        if (q->data_x) (void)hipFree(q->data_x);
        if (q->data_t) (void)hipFree(q->data_t);
        if (q->idx) (void)hipFree(q->idx);
        q->data_x = nullptr;
        q->data_t = nullptr;
        q->idx = nullptr;
        q->data_rows = 0;
        HIP_TRY(hipMalloc((void**)&q->data_x, (size_t)rows * n_in * sizeof(float)));
        HIP_TRY(hipMalloc((void**)&q->data_t, (size_t)rows * n_out * sizeof(float)));
        HIP_TRY(hipMalloc((void**)&q->idx, (size_t)rows * sizeof(int)));
        q->data_rows = rows;
    }
    HIP_TRY(hipMemcpyAsync(q->data_x, x, (size_t)rows * n_in * sizeof(float), hipMemcpyHostToDevice, q->stream));
    HIP_TRY(hipMemcpyAsync(q->data_t, t, (size_t)rows * n_out * sizeof(float), hipMemcpyHostToDevice, q->stream));
    std::vector<int> perm(rows);
    // learning rate: cosine from lr to lr_final over all minibatch steps (constant if equal)
    const int64_t per_epoch = (rows + batch - 1) / batch, last = std::max<int64_t>(1, per_epoch * epochs - 1);
    int64_t step = 0;
    for (int e = 0; e < epochs; ++e) {
        // epoch order: Fisher-Yates driven by SplitMix64(seed, epoch, i)
        for (int64_t i = 0; i < rows; ++i) perm[i] = (int)i;
        for (int64_t i = rows - 1; i > 0; --i) {
            const uint64_t r = splitmix64(splitmix64(seed ^ (0x5851F42D4C957F2Dull * (uint64_t)(e + 1))) ^ (uint64_t)i);
            std::swap(perm[i], perm[(int64_t)(r % (uint64_t)(i + 1))]);
        }
        HIP_TRY(hipMemcpyAsync(q->idx, perm.data(), rows * sizeof(int), hipMemcpyHostToDevice, q->stream));
        double sum = 0.0;
        int64_t seen = 0;
        for (int64_t b0 = 0; b0 < rows; b0 += batch) {
            const int r = (int)std::min<int64_t>(batch, rows - b0);
            cronos_status st = gather_rows(q, q->data_x, q->data_t, q->idx + b0, r);
            if (st == CRONOS_OK) st = forward_dev(q, r, true);
            if (st == CRONOS_OK) st = backward_dev(q, r, false);
            const double lr_t = lr_final + 0.5 * (lr - lr_final) * (1.0 + std::cos(M_PI * (double)step++ / (double)last));
            if (st == CRONOS_OK) st = adam_dev(q, lr_t, 0.9, 0.999, 1e-8);
            if (st != CRONOS_OK) return st;
            if (e == epochs - 1) {
                const double l = loss_from_parts(q, r, &st);
                if (st != CRONOS_OK) return st;
                sum += l * r;
                seen += r;
            }
        }
        HIP_TRY(hipStreamSynchronize(q->stream));   // perm is rewritten next epoch
        if (e == epochs - 1 && epoch_loss) *epoch_loss = seen ? sum / seen : 0.0;
    }
    return CRONOS_OK;
}
