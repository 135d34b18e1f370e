// Natural frequencies of the linearised mass-spring system (section "Natural Frequency
// Analysis": the generalised eigenproblem K v = w^2 M v).  Lanczos iterations on the
// symmetric operator A = M^-1/2 K M^-1/2 run on the device in FP64; the host takes the
// eigenvalues of the tridiagonal matrix they build (see cronos_natural_frequencies).
//
// K is the tangent stiffness of the Hookean springs of eq. (2) at the current positions:
// for a spring with unit direction n, length l and (actuated) rest length l0 its 3x3 block is
// k [n n^T + (1 - l0 / l)(I - n n^T)], entering the two diagonal blocks with + and the two
// off-diagonal blocks with -, so that df = -K dx; a mass below the contact plane adds the
// penalty stiffness k_g to its z diagonal.  Fixed masses are removed (their M^-1/2 is 0).
//
// Layout: the step's explicit incidence form (per-lane slices of (LDS slot, k, L0) with
// halo indices), one workgroup per block of masses whose positions and M^-1/2 q (with the
// halo's) are staged in LDS first; every sum is reduced in a fixed order, so a run is
// bitwise repeatable.
#include "kernels.h"

#include <mutex>
#include <vector>

// Workspace of cronos_natural_frequencies_noalloc (each GPU holds its own copy).  Host code
// never uses this name as an address: modes_scratch looks the device address up.
static __device__ __align__(256) double scratch[cronos::kModesScratchDoubles];

namespace cronos {
namespace {

constexpr int kMaxWaves = 16;
constexpr size_t kModesMaxLds = 150 * 1024;   // dynamic LDS of the staged apply kernel (of 160 KiB)
// workgroups of the vector kernels of an iteration: each workgroup first sums the previous
// kernel's partials, so fewer of them (each thread taking several masses) cost fewer sums
constexpr int kModesVecGroups = 512;

__device__ __forceinline__ double wave_add(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup: wavefront sums, then added in wavefront order by one lane.
__device__ double workgroup_sum(double v, double* red) {
    v = wave_add(v);
    const int t = (int)threadIdx.x, nw = ((int)blockDim.x + 63) >> 6;
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w];
        red[kMaxWaves] = s;
    }
    __syncthreads();
    const double s = red[kMaxWaves];
    __syncthreads();
    return s;
}

// Sum of part[0..count) in a fixed order (the same in every workgroup).
__device__ double sum_parts(const double* __restrict__ part, int count, double* red) {
    double a = 0.0;
    for (int q = (int)threadIdx.x; q < count; q += (int)blockDim.x) a += part[q];
    return workgroup_sum(a, red);
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// M^-1/2 per mass and a random start vector (zero on fixed masses); partial squared norms;
// zeros in q_prev (the Lanczos vector before the first, cleared here by a kernel rather than a
// memset node so that the sequence stays a plain kernel chain).
__global__ void __launch_bounds__(256) modes_init_kernel(const float4* __restrict__ x, const float* __restrict__ mass,
                                                         double* __restrict__ ism, double* __restrict__ w,
                                                         double* __restrict__ q_prev, double* __restrict__ part, int n,
                                                         unsigned long long seed) {
    __shared__ double red[kMaxWaves + 1];
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    double nn = 0.0;
    if (i < n) {
        const bool free_mass = x[i].w != 0.0f;
        ism[i] = free_mass ? 1.0 / sqrt((double)mass[i]) : 0.0;
        for (int c = 0; c < 3; ++c) {
            const unsigned long long h = mix64(seed + 0x9e3779b97f4a7c15ull * (unsigned long long)(3 * (long long)i + c + 1));
            const double u = free_mass ? (double)(h >> 11) * 0x1.0p-53 - 0.5 : 0.0;
            w[3 * i + c] = u;
            q_prev[3 * i + c] = 0.0;
            nn += u * u;
        }
    }
    const double s = workgroup_sum(nn, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

struct ApplyArgs {
    const float4* __restrict__ x;
    const double* __restrict__ ism;
    const int32_t* __restrict__ slice_ptr;
    const uint16_t* __restrict__ nbr;
    const float2* __restrict__ kl;
    const uint16_t* __restrict__ grp;
    const float* __restrict__ factor;
    const int32_t* __restrict__ halo_ptr;
    const int32_t* __restrict__ halo_idx;
    const uint16_t* __restrict__ lane_mass;
    int n, block, lds_slots;
    int ground;
    float ground_z, ground_k;
};

// 1/sqrt(s) to FP64 accuracy: the hardware estimate refined by two Newton steps
// y <- y + y (1 - s y^2) / 2 (each roughly doubles the correct bits), far cheaper than a
// correctly rounded square root followed by a division.
__device__ __forceinline__ double rsqrt_fp64(double s) {
    double y = __builtin_amdgcn_rsq(s);
    for (int it = 0; it < 2; ++it) {
        const double e = __builtin_fma(-(s * y), y, 1.0);
        y = __builtin_fma(0.5 * y, e, y);
    }
    return y;
}

// Contribution of spring (i, j) to (K u)_i: k [n n^T + (1 - l0/l)(I - n n^T)] (u_i - u_j).
__device__ __forceinline__ void spring_hessian(float4 xi, float4 xj, double u0, double u1, double u2, double v0,
                                               double v1, double v2, double kk, double l0, double& k0, double& k1,
                                               double& k2) {
    const double dx = (double)xj.x - (double)xi.x, dy = (double)xj.y - (double)xi.y, dz = (double)xj.z - (double)xi.z;
    const double il = rsqrt_fp64(dx * dx + dy * dy + dz * dz);
    const double nx = dx * il, ny = dy * il, nz = dz * il;
    const double d0 = u0 - v0, d1 = u1 - v1, d2 = u2 - v2;
    const double nd = nx * d0 + ny * d1 + nz * d2;
    const double g = 1.0 - l0 * il;
    k0 += kk * (nd * nx + g * (d0 - nd * nx));
    k1 += kk * (nd * ny + g * (d1 - nd * ny));
    k2 += kk * (nd * nz + g * (d2 - nd * nz));
}

// y = A q with the workgroup's masses and halo staged in LDS: positions (float4) and
// u = M^-1/2 q (FP64) per slot, so the incidence loop reads no global memory but its entries.
__global__ void __launch_bounds__(1024) modes_apply_lds_kernel(ApplyArgs a, const double* __restrict__ q,
                                                               double* __restrict__ y, double* __restrict__ part) {
    extern __shared__ float4 sx[];                       // [lds_slots] positions
    double* su = reinterpret_cast<double*>(sx + a.lds_slots);   // [lds_slots][3] u
    __shared__ double red[kMaxWaves + 1];
    const int b = (int)blockIdx.x, t = (int)threadIdx.x;
    const int base = b * a.block;
    const int h0 = a.halo_ptr[b], slots = a.block + (a.halo_ptr[b + 1] - h0);
    for (int sl = t; sl < slots; sl += (int)blockDim.x) {
        const int m = sl < a.block ? base + sl : a.halo_idx[h0 + sl - a.block];
        float4 xm = make_float4(0.f, 0.f, 0.f, 0.f);
        double u0 = 0.0, u1 = 0.0, u2 = 0.0;
        if (m < a.n) {
            xm = a.x[m];
            const double sm = a.ism[m];
            u0 = sm * q[3 * m];
            u1 = sm * q[3 * m + 1];
            u2 = sm * q[3 * m + 2];
        }
        sx[sl] = xm;
        su[3 * sl] = u0;
        su[3 * sl + 1] = u1;
        su[3 * sl + 2] = u2;
    }
    __syncthreads();
    const int own = a.lane_mass[base + t];
    const int i = base + own;
    double dot = 0.0;
    if (i < a.n) {
        const float4 xi = sx[own];
        const double u0 = su[3 * own], u1 = su[3 * own + 1], u2 = su[3 * own + 2];
        double k0 = 0.0, k1 = 0.0, k2 = 0.0;
        const int s = (base + t) >> 6, lane = t & 63;
        const int e0 = a.slice_ptr[s];
        const int width = (a.slice_ptr[s + 1] - e0) >> 6;
        for (int r = 0, e = e0 + lane; r < width; ++r, e += 64) {
            const int slot = a.nbr[e];
            if (slot == own) continue;  // padding
            const float2 c = a.kl[e];
            double l0 = (double)c.y;
            if (a.grp) l0 *= (double)a.factor[a.grp[e]];
            spring_hessian(xi, sx[slot], u0, u1, u2, su[3 * slot], su[3 * slot + 1], su[3 * slot + 2], (double)c.x,
                           l0, k0, k1, k2);
        }
        if (a.ground && xi.z < a.ground_z) k2 += (double)a.ground_k * u2;
        const double si = a.ism[i];
        const double y0 = si * k0, y1 = si * k1, y2 = si * k2;
        y[3 * i] = y0;
        y[3 * i + 1] = y1;
        y[3 * i + 2] = y2;
        dot = q[3 * i] * y0 + q[3 * i + 1] * y1 + q[3 * i + 2] * y2;
    }
    const double sum = workgroup_sum(dot, red);
    if (t == 0) part[b] = sum;
}

// y = A q for a full box in the structured-box layout (one 512-mass workgroup per aligned
// 8 x 8 x 8 Morton cube, every mass linked to its 26 grid neighbours, as the step's
// structured-box form): the cube and its one-node halo are staged as a 10 x 10 x 10 tile of
// positions and u = M^-1/2 q, each neighbour sits at a fixed tile offset, k comes from the
// table per (boundary class, direction) and L0 per direction kind, so no incidence data is
// read.  Halo cells outside the box hold a far position and u = 0 with k = 0: no contribution.
struct GridApplyArgs {
    const float4* __restrict__ x;
    const double* __restrict__ ism;
    const int32_t* __restrict__ halo;   // [nblk][488] new index of each halo cell, -1 outside
    const int4* __restrict__ org;       // [nblk] grid coordinates of the block's first node
    const float* __restrict__ kcls;     // [27][26] k per (boundary class, direction)
    const uint32_t* __restrict__ tab;   // [512] lane's tile cell | lx << 10 | ly << 13 | lz << 16,
                                        // then [488] tile cell of each halo slot
    int nx, ny, nz;
    float l0[3];                        // rest length per direction kind (1, 2, 3 non-zero offsets)
    int ground;
    float ground_z, ground_k;
};

constexpr int kTilePitch = 10, kTileCells = 1000, kTileHalo = 488, kTileMasses = 512;

__global__ void __launch_bounds__(kTileMasses) modes_apply_grid_kernel(GridApplyArgs a, const double* __restrict__ q,
                                                                       double* __restrict__ y,
                                                                       double* __restrict__ part) {
    __shared__ float4 tx[kTileCells];
    __shared__ double tu[3 * kTileCells];
    __shared__ float kc[27 * 26];
    __shared__ double red[kMaxWaves + 1];
    const int b = (int)blockIdx.x, t = (int)threadIdx.x;
    const int i = b * kTileMasses + t;   // the box holds whole cubes: i < n
    const uint32_t info = a.tab[t];
    const int cell = (int)(info & 1023u);
    {
        const double sm = a.ism[i];
        tx[cell] = a.x[i];
        tu[3 * cell + 0] = sm * q[3 * i + 0];
        tu[3 * cell + 1] = sm * q[3 * i + 1];
        tu[3 * cell + 2] = sm * q[3 * i + 2];
    }
    for (int h = t; h < kTileHalo; h += kTileMasses) {
        const int g = a.halo[(long)b * kTileHalo + h];
        const int c = (int)a.tab[kTileMasses + h];
        float4 xm = make_float4(1e18f, 1e18f, 1e18f, 0.0f);
        double u0 = 0.0, u1 = 0.0, u2 = 0.0;
        if (g >= 0) {
            const double sm = a.ism[g];
            xm = a.x[g];
            u0 = sm * q[3 * g + 0];
            u1 = sm * q[3 * g + 1];
            u2 = sm * q[3 * g + 2];
        }
        tx[c] = xm;
        tu[3 * c + 0] = u0;
        tu[3 * c + 1] = u1;
        tu[3 * c + 2] = u2;
    }
    for (int r = t; r < 27 * 26; r += kTileMasses) kc[r] = a.kcls[r];
    const int4 o = a.org[b];
    const int gx = o.x + (int)((info >> 10) & 7u), gy = o.y + (int)((info >> 13) & 7u), gz = o.z + (int)((info >> 16) & 7u);
    const int cls = (gx == 0 ? 0 : gx == a.nx - 1 ? 2 : 1) + 3 * (gy == 0 ? 0 : gy == a.ny - 1 ? 2 : 1) +
                    9 * (gz == 0 ? 0 : gz == a.nz - 1 ? 2 : 1);
    __syncthreads();
    const float4 xi = tx[cell];
    const double u0 = tu[3 * cell + 0], u1 = tu[3 * cell + 1], u2 = tu[3 * cell + 2];
    double k0 = 0.0, k1 = 0.0, k2 = 0.0;
#pragma unroll
    for (int d = 0; d < 26; ++d) {
        const int e = d < 13 ? d : d + 1;   // the 3 x 3 x 3 stencil without its centre, (dz, dy, dx) order
        const int ox = e % 3 - 1, oy = (e / 3) % 3 - 1, oz = e / 9 - 1;
        const int kind = (ox != 0) + (oy != 0) + (oz != 0) - 1;
        const int nc = cell + (oz * kTilePitch + oy) * kTilePitch + ox;
        spring_hessian(xi, tx[nc], u0, u1, u2, tu[3 * nc], tu[3 * nc + 1], tu[3 * nc + 2], (double)kc[26 * cls + d],
                       (double)a.l0[kind], k0, k1, k2);
    }
    if (a.ground && xi.z < a.ground_z) k2 += (double)a.ground_k * u2;
    const double si = a.ism[i];
    const double y0 = si * k0, y1 = si * k1, y2 = si * k2;
    y[3 * i] = y0;
    y[3 * i + 1] = y1;
    y[3 * i + 2] = y2;
    const double dot = q[3 * i] * y0 + q[3 * i + 1] * y1 + q[3 * i + 2] * y2;
    const double sum = workgroup_sum(dot, red);
    if (t == 0) part[b] = sum;
}

// y = A q for the masses of workgroup-block b, and the block's part of q . y; neighbours read
// from global memory (used when the staged form's LDS would not fit).
__global__ void __launch_bounds__(1024) modes_apply_kernel(ApplyArgs a, const double* __restrict__ q,
                                                           double* __restrict__ y, double* __restrict__ part) {
    __shared__ double red[kMaxWaves + 1];
    const int b = (int)blockIdx.x, t = (int)threadIdx.x;
    const int base = b * a.block;
    const int i = base + a.lane_mass[base + t];
    double dot = 0.0;
    if (i < a.n) {
        const float4 xi = a.x[i];
        const double si = a.ism[i];
        const double u0 = si * q[3 * i], u1 = si * q[3 * i + 1], u2 = si * q[3 * i + 2];
        double k0 = 0.0, k1 = 0.0, k2 = 0.0;
        const int s = (base + t) >> 6, lane = t & 63;
        const int e0 = a.slice_ptr[s];
        const int width = (a.slice_ptr[s + 1] - e0) >> 6;
        const int h0 = a.halo_ptr[b];
        for (int r = 0, e = e0 + lane; r < width; ++r, e += 64) {
            const int slot = a.nbr[e];
            const int j = slot < a.block ? base + slot : a.halo_idx[h0 + slot - a.block];
            if (j == i) continue;  // padding
            const float2 c = a.kl[e];
            double l0 = (double)c.y;
            if (a.grp) l0 *= (double)a.factor[a.grp[e]];
            const double sj = a.ism[j];
            spring_hessian(xi, a.x[j], u0, u1, u2, sj * q[3 * j], sj * q[3 * j + 1], sj * q[3 * j + 2], (double)c.x,
                           l0, k0, k1, k2);
        }
        if (a.ground && xi.z < a.ground_z) k2 += (double)a.ground_k * u2;
        const double y0 = si * k0, y1 = si * k1, y2 = si * k2;
        y[3 * i] = y0;
        y[3 * i + 1] = y1;
        y[3 * i + 2] = y2;
        dot = q[3 * i] * y0 + q[3 * i + 1] * y1 + q[3 * i + 2] * y2;
    }
    const double sum = workgroup_sum(dot, red);
    if (t == 0) part[b] = sum;
}

// alpha_k = q . y (from the apply kernel's parts); w = y - alpha_k q - beta_k q_prev written
// over q_prev; partial squared norms of w.
__global__ void __launch_bounds__(256) modes_update_kernel(const double* __restrict__ apart, int n_apart,
                                                           const double* __restrict__ y, const double* __restrict__ q,
                                                           double* __restrict__ qw, double* __restrict__ alpha,
                                                           const double* __restrict__ beta, int k,
                                                           double* __restrict__ part, int n) {
    __shared__ double red[kMaxWaves + 1];
    const double al = sum_parts(apart, n_apart, red);
    const double bp = k > 0 ? beta[k - 1] : 0.0;
    double nn = 0.0;
    for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += (int)(gridDim.x * blockDim.x)) {
        for (int c = 0; c < 3; ++c) {
            const double w = y[3 * i + c] - al * q[3 * i + c] - bp * qw[3 * i + c];
            qw[3 * i + c] = w;
            nn += w * w;
        }
    }
    const double s = workgroup_sum(nn, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha[k] = al;
}

// beta = |w| (from the parts); w /= beta in place; beta stored at beta[k] when k >= 0.
__global__ void __launch_bounds__(256) modes_scale_kernel(const double* __restrict__ part, int n_part,
                                                          double* __restrict__ w, double* __restrict__ beta, int k,
                                                          int n) {
    __shared__ double red[kMaxWaves + 1];
    const double b = sqrt(sum_parts(part, n_part, red));
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += (int)(gridDim.x * blockDim.x))
        for (int c = 0; c < 3; ++c) w[3 * i + c] *= inv;
    if (k >= 0 && blockIdx.x == 0 && threadIdx.x == 0) beta[k] = b;
}

}  // namespace

hipError_t launch_modes_init(const DeviceArrays& d, int cur, ModesBuffers& m, unsigned long long seed, hipStream_t st) {
    const int n = (int)d.n, g = (n + 255) / 256;
    hipLaunchKernelGGL(modes_init_kernel, dim3(g), dim3(256), 0, st, d.x[cur], d.mass, m.ism, m.q[1], m.q[0], m.part_u,
                       n, seed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(modes_scale_kernel, dim3(g), dim3(256), 0, st, m.part_u, g, m.q[1], m.beta, -1, n);
    return hipGetLastError();
}

hipError_t launch_modes_iteration(const DeviceArrays& d, int cur, const StepParams& p, ModesBuffers& m, int k,
                                  hipStream_t st) {
    const int n = (int)d.n, g = (n + 255) / 256;
    double* q = m.q[(k + 1) & 1];   // q_k (the start vector q_0 sits in q[1])
    double* qw = m.q[k & 1];        // q_{k-1} in, q_{k+1} out
    ApplyArgs a{d.x[cur], m.ism, d.slice_ptr, d.nbr, d.kl, d.grp, d.factor, d.halo_ptr, d.halo_idx, d.lane_mass,
                n, d.block, d.lds_slots, p.ground, p.ground_z, p.ground_k};
    const size_t lds = (size_t)d.lds_slots * (sizeof(float4) + 3 * sizeof(double));
    if (d.grid) {
        GridApplyArgs ga{d.x[cur], m.ism, d.grid_halo, d.grid_org, d.grid_k, d.grid_tab,
                         d.grid_dim[0], d.grid_dim[1], d.grid_dim[2], {d.grid_l0[0], d.grid_l0[1], d.grid_l0[2]},
                         p.ground, p.ground_z, p.ground_k};
        hipLaunchKernelGGL(modes_apply_grid_kernel, dim3((unsigned)d.nblk), dim3(kTileMasses), 0, st, ga, q, m.y,
                           m.part_a);
    } else if (lds <= kModesMaxLds)
        hipLaunchKernelGGL(modes_apply_lds_kernel, dim3((unsigned)d.nblk), dim3(d.block), lds, st, a, q, m.y, m.part_a);
    else
        hipLaunchKernelGGL(modes_apply_kernel, dim3((unsigned)d.nblk), dim3(d.block), 0, st, a, q, m.y, m.part_a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int gv = std::min(g, kModesVecGroups);   // part_u holds g >= gv partials
    hipLaunchKernelGGL(modes_update_kernel, dim3(gv), dim3(256), 0, st, m.part_a, (int)d.nblk, m.y, q, qw, m.alpha,
                       m.beta, k, m.part_u, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(modes_scale_kernel, dim3(gv), dim3(256), 0, st, m.part_u, gv, qw, m.beta, k, n);
    return hipGetLastError();
}

hipError_t modes_scratch(int device, double** ptr) {
    static std::mutex mu;
    static std::vector<double*> addr;   // per device ordinal
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<double*>(p);
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace cronos
