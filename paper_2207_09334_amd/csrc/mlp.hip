// Surrogate network on gfx950: a 4-layer perceptron (3 exact-erf GELU hidden layers, linear
// output) whose products run on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation; weights are kept as an FP32 master copy and a BF16 shadow; Adam in FP32.
//
// GEMM: C[M x N] = sum_k A(m, k) B(k, n) with strided A and B (so the forward product, the
// back-propagation through W^T and the weight gradient X^T dZ are one kernel).  A workgroup
// (4 wavefronts) computes a 64 x 64 tile, each wavefront a 32 x 32 quarter as 2 x 2 MFMA tiles
// of 16 x 16, stepping K by 32 through LDS.  Operand layouts of the 16x16x32 BF16 MFMA: lane l
// supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j = 0..7, and receives
// C[4 (l / 16) + r][l % 16], r = 0..3.
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

constexpr int kTile = 64, kK = 32, kPad = 8;

enum Epilogue { kFwdGelu = 0, kLinear = 1, kBwdGelu = 2, kPlain = 3 };

struct GemmArgs {
    const bf16* A;
    long sam, sak;        // A(m, k) = A[m * sam + k * sak]
    const bf16* B;
    long sbk, sbn;        // B(k, n) = B[k * sbk + n * sbn]
    int M, N, K;
    const float* bias;    // [N] (forward epilogues)
    float* Cf;            // FP32 output, row-major M x N
    bf16* Cb;             // BF16 output, row-major M x N
    const float* Z;       // pre-activation, row-major M x N (backward GELU)
};

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

template <int EPI>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) bf16 As[kTile][kK + kPad];
    __shared__ __attribute__((aligned(16))) bf16 Bs[kTile][kK + kPad];   // [n][k]
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = t >> 2, lk = (t & 3) * 8;   // this thread's row and k-offset in the LDS tiles
    for (int kb = 0; kb < g.K; kb += kK) {
        {
            const int m = m0 + lr;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = kb + lk + j;
                As[lr][lk + j] = (m < g.M && k < g.K) ? g.A[(long)m * g.sam + (long)k * g.sak] : (bf16)0.0f;
            }
            const int n = n0 + lr;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = kb + lk + j;
                Bs[lr][lk + j] = (n < g.N && k < g.K) ? g.B[(long)k * g.sbk + (long)n * g.sbn] : (bf16)0.0f;
            }
        }
        __syncthreads();
        const int r16 = lane & 15, k8 = (lane >> 4) * 8;
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + i * 16 + r16][k8]);
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + j * 16 + r16][k8]);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[i][j][r];
                const long o = (long)m * g.N + n;
                if (EPI == kFwdGelu) {
                    const float z = v + g.bias[n];
                    g.Cf[o] = z;
                    g.Cb[o] = (bf16)gelu(z);
                } else if (EPI == kLinear) {
                    g.Cf[o] = v + g.bias[n];
                } else if (EPI == kBwdGelu) {
                    g.Cb[o] = (bf16)(v * gelu_grad(g.Z[o]));
                } else {
                    g.Cf[o] = v;
                }
            }
}

// dY = 2 (Y - T) / (rows * n_out) as BF16 (zero on padding rows) and per-block loss partials.
__global__ void __launch_bounds__(256) loss_kernel(const float* Y, const float* T, bf16* dY, double* part, int rows,
                                                   int padded_rows, int n_out) {
    __shared__ double red[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (i < padded_rows * n_out) {
        const int r = i / n_out;
        float d = 0.0f;
        if (r < rows) {
            d = Y[i] - T[i];
            l = (double)d * (double)d;
        }
        dY[i] = (bf16)(2.0f * d / (float)(rows * n_out));
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Column sums of a BF16 matrix (bias gradients), one thread per column, rows in order.
__global__ void colsum_kernel(const bf16* D, float* out, int rows, int cols) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.0f;
    for (int r = 0; r < rows; ++r) s += (float)D[(long)r * cols + c];
    out[c] = s;
}

// Adam on the FP32 master copy; refreshes the BF16 shadow of the weight entries.
__global__ void adam_kernel(float* p, float* m, float* v, const float* grad, bf16* shadow, const int* is_weight,
                            long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (is_weight[i]) shadow[i] = (bf16)pi;
}

__global__ void to_bf16_kernel(const float* src, bf16* dst, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (bf16)src[i];
}

// Minibatch gather: X_b[r] = bf16(X[idx[r]]), T_b[r] = T[idx[r]]; zero beyond `rows`.
__global__ void gather_kernel(const float* X, const float* T, const int* idx, bf16* Xb, float* Tb, int rows,
                              int padded_rows, int n_in, int n_out) {
    const int r = blockIdx.x;
    if (r >= padded_rows) return;
    const long src = r < rows ? (long)idx[r] : -1;
    for (int c = threadIdx.x; c < n_in; c += blockDim.x) Xb[(long)r * n_in + c] = src >= 0 ? (bf16)X[src * n_in + c] : (bf16)0.0f;
    for (int c = threadIdx.x; c < n_out; c += blockDim.x) Tb[(long)r * n_out + c] = src >= 0 ? T[src * n_out + c] : 0.0f;
}

uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

using cronos::fail;

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(CRONOS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct cronos_mlp_t {
    int sizes[5];
    int max_rows = 0;      // padded to a multiple of 64
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    long n_params = 0;
    long off_w[4], off_b[4];
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    bf16* shadow = nullptr;
    int* is_weight = nullptr;
    int step = 0;
    // activations for max_rows
    bf16* x = nullptr;                 // [rows][sizes[0]]
    float* z[3] = {nullptr, nullptr, nullptr};
    bf16* h[3] = {nullptr, nullptr, nullptr};
    float* y = nullptr;
    float* t = nullptr;
    bf16* dy = nullptr;
    bf16* dz[3] = {nullptr, nullptr, nullptr};
    double* part = nullptr;
    // training data
    float* data_x = nullptr;
    float* data_t = nullptr;
    int* idx = nullptr;
    long data_rows = 0;
};

namespace {

template <int EPI>
hipError_t gemm(hipStream_t st, const bf16* A, long sam, long sak, const bf16* B, long sbk, long sbn, int M, int N, int K,
                const float* bias, float* Cf, bf16* Cb, const float* Z) {
    GemmArgs g{A, sam, sak, B, sbk, sbn, M, N, K, bias, Cf, Cb, Z};
    dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile);
    hipLaunchKernelGGL(gemm_kernel<EPI>, grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

void free_mlp(cronos_mlp_t* q) {
    void* ptrs[] = {q->p, q->m, q->v, q->grad, q->shadow, q->is_weight, q->x, q->z[0], q->z[1], q->z[2], q->h[0],
                    q->h[1], q->h[2], q->y, q->t, q->dy, q->dz[0], q->dz[1], q->dz[2], q->part, q->data_x, q->data_t,
                    q->idx};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (q->own_stream && q->stream) (void)hipStreamDestroy(q->stream);
}

// Forward over `rows` (<= max_rows, padded to 64) rows already in q->x.
cronos_status forward_dev(cronos_mlp_t* q, int rows) {
    const int P = (rows + 63) / 64 * 64;
    const bf16* in = q->x;
    for (int l = 0; l < 3; ++l) {
        const int K = q->sizes[l], N = q->sizes[l + 1];
        HIP_TRY(gemm<kFwdGelu>(q->stream, in, K, 1, q->shadow + q->off_w[l], N, 1, P, N, K, q->p + q->off_b[l], q->z[l],
                               q->h[l], nullptr));
        in = q->h[l];
    }
    const int K = q->sizes[3], N = q->sizes[4];
    HIP_TRY(gemm<kLinear>(q->stream, in, K, 1, q->shadow + q->off_w[3], N, 1, P, N, K, q->p + q->off_b[3], q->y, nullptr,
                          nullptr));
    return CRONOS_OK;
}

// Loss and gradients for `rows` rows whose inputs are in q->x and targets in q->t.
cronos_status backward_dev(cronos_mlp_t* q, int rows) {
    const int P = (rows + 63) / 64 * 64;
    const int n_out = q->sizes[4];
    const int nel = P * n_out;
    hipLaunchKernelGGL(loss_kernel, dim3((nel + 255) / 256), dim3(256), 0, q->stream, q->y, q->t, q->dy, q->part, rows, P,
                       n_out);
    HIP_TRY(hipGetLastError());
    const bf16* dnext = q->dy;
    for (int l = 3; l >= 0; --l) {
        const int K = q->sizes[l], N = q->sizes[l + 1];
        const bf16* hin = l ? q->h[l - 1] : q->x;
        // dW_l = H_in^T dZ_l : (K x P) (P x N)
        HIP_TRY(gemm<kPlain>(q->stream, hin, 1, K, dnext, N, 1, K, N, P, nullptr, q->grad + q->off_w[l], nullptr, nullptr));
        hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, q->stream, dnext, q->grad + q->off_b[l], P, N);
        HIP_TRY(hipGetLastError());
        if (l) {
            // dZ_{l-1} = (dZ_l W_l^T) * gelu'(Z_{l-1}) : (P x N) (N x K)
            HIP_TRY(gemm<kBwdGelu>(q->stream, dnext, N, 1, q->shadow + q->off_w[l], 1, N, P, K, N, nullptr, nullptr,
                                   q->dz[l - 1], q->z[l - 1]));
            dnext = q->dz[l - 1];
        }
    }
    return CRONOS_OK;
}

cronos_status upload_rows(cronos_mlp_t* q, const float* x, const float* t, int rows) {
    const int n_in = q->sizes[0], n_out = q->sizes[4];
    const int P = (rows + 63) / 64 * 64;
    std::vector<bf16> hx((size_t)P * n_in, (bf16)0.0f);
    for (long i = 0; i < (long)rows * n_in; ++i) hx[i] = (bf16)x[i];
    HIP_TRY(hipMemcpyAsync(q->x, hx.data(), hx.size() * sizeof(bf16), hipMemcpyHostToDevice, q->stream));
    if (t) {
        std::vector<float> ht((size_t)P * n_out, 0.0f);
        std::memcpy(ht.data(), t, (size_t)rows * n_out * sizeof(float));
        HIP_TRY(hipMemcpyAsync(q->t, ht.data(), ht.size() * sizeof(float), hipMemcpyHostToDevice, q->stream));
    }
    HIP_TRY(hipStreamSynchronize(q->stream));   // host staging buffers go out of scope
    return CRONOS_OK;
}

cronos_status adam_dev(cronos_mlp_t* q, double lr, double b1, double b2, double eps) {
    q->step += 1;
    const float c1 = (float)(1.0 - std::pow(b1, q->step)), c2 = (float)(1.0 - std::pow(b2, q->step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((q->n_params + 255) / 256)), dim3(256), 0, q->stream, q->p, q->m,
                       q->v, q->grad, q->shadow, q->is_weight, q->n_params, (float)lr, (float)b1, (float)b2, (float)eps,
                       c1, c2);
    HIP_TRY(hipGetLastError());
    return CRONOS_OK;
}

double loss_from_parts(cronos_mlp_t* q, int rows, cronos_status* st) {
    const int P = (rows + 63) / 64 * 64;
    const int nb = (P * q->sizes[4] + 255) / 256;
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
    auto* q = new (std::nothrow) cronos_mlp_t;
    if (!q) return fail(CRONOS_ENOMEM, "mlp_create: out of memory");
    for (int l = 0; l < 5; ++l) q->sizes[l] = sizes[l];
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
        HIP_TRY(hipMalloc((void**)&q->p, n * sizeof(float)));
        HIP_TRY(hipMalloc((void**)&q->m, n * sizeof(float)));
        HIP_TRY(hipMalloc((void**)&q->v, n * sizeof(float)));
        HIP_TRY(hipMalloc((void**)&q->grad, n * sizeof(float)));
        HIP_TRY(hipMalloc((void**)&q->shadow, n * sizeof(bf16)));
        HIP_TRY(hipMalloc((void**)&q->is_weight, n * sizeof(int)));
        HIP_TRY(hipMalloc((void**)&q->x, R * sizes[0] * sizeof(bf16)));
        for (int l = 0; l < 3; ++l) {
            HIP_TRY(hipMalloc((void**)&q->z[l], R * sizes[l + 1] * sizeof(float)));
            HIP_TRY(hipMalloc((void**)&q->h[l], R * sizes[l + 1] * sizeof(bf16)));
            HIP_TRY(hipMalloc((void**)&q->dz[l], R * sizes[l + 1] * sizeof(bf16)));
        }
        HIP_TRY(hipMalloc((void**)&q->y, R * sizes[4] * sizeof(float)));
        HIP_TRY(hipMalloc((void**)&q->t, R * sizes[4] * sizeof(float)));
        HIP_TRY(hipMalloc((void**)&q->dy, R * sizes[4] * sizeof(bf16)));
        HIP_TRY(hipMalloc((void**)&q->part, ((R * sizes[4] + 255) / 256) * sizeof(double)));
        std::vector<float> hp(n), zero(n, 0.0f);
        std::vector<int> iw(n, 0);
        for (long i = 0; i < n; ++i) hp[i] = (float)params[i];
        for (int l = 0; l < 4; ++l)
            for (long i = q->off_w[l]; i < q->off_b[l]; ++i) iw[i] = 1;
        HIP_TRY(hipMemcpy(q->p, hp.data(), n * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(q->m, zero.data(), n * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(q->v, zero.data(), n * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(q->grad, zero.data(), n * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(q->is_weight, iw.data(), n * sizeof(int), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, q->stream, q->p, q->shadow, n);
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
    std::vector<float> hy;
    for (int64_t r0 = 0; r0 < rows; r0 += q->max_rows) {
        const int r = (int)std::min<int64_t>(q->max_rows, rows - r0);
        cronos_status st = upload_rows(q, x + r0 * q->sizes[0], nullptr, r);
        if (st != CRONOS_OK) return st;
        st = forward_dev(q, r);
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
    if (st == CRONOS_OK) st = forward_dev(q, rows);
    if (st == CRONOS_OK) st = backward_dev(q, rows);
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
            const int P = (r + 63) / 64 * 64;
            hipLaunchKernelGGL(gather_kernel, dim3(P), dim3(128), 0, q->stream, q->data_x, q->data_t, q->idx + b0, q->x, q->t,
                               r, P, n_in, n_out);
            HIP_TRY(hipGetLastError());
            cronos_status st = forward_dev(q, r);
            if (st == CRONOS_OK) st = backward_dev(q, r);
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
