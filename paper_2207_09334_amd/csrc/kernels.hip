// Device kernels of the mass-spring step for gfx950 (CDNA4, wave64).
//
// One time step is one launch of `step_kernel` (plus a one-workgroup launch that tabulates
// the actuation factors when springs are actuated).  It fuses what Algorithm 1 splits into
// a spring pass and a mass pass: every lane owns one mass, walks that mass's incidence list
// in a fixed order and sums the eq. (2) spring forces itself, so no force is ever written
// twice and no atomic is needed; the sum is bitwise reproducible run to run.
//
// Memory: positions are float4 (x, y, z, 1/m) so one 16-byte load fetches a neighbour; a
// workgroup first copies its own masses and its halo (the neighbours outside the workgroup)
// into LDS, then every incidence reads its neighbour from LDS through a 16-bit slot index.
// The incidence stream (slot, k, L0) is laid out column-major per 64-mass slice, so each
// wavefront's loads are contiguous.  Workgroups are spread so that each of the 8 XCDs gets a
// contiguous range of the Morton order (their halos then overlap within one L2).
//
// Precision: FP32 state and FP32 accumulation.  The elongation |d| - L0 of a nearly relaxed
// spring is a difference of nearly equal numbers; it is computed as (|d|^2 - L0^2)/(|d| + L0)
// with |d|^2 - L0^2 formed from error-free products (FMA) and error-free sums (Knuth's
// TwoSum), so its error is a few ulps of the elongation itself, not of L0.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cronos {

namespace {

__device__ __forceinline__ int logical_block(int nblk) {
    const int per = (nblk + 7) >> 3;
    return (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
}

// Error-free sum (Knuth): s + e == a + b exactly.
__device__ __forceinline__ float two_sum(float a, float b, float& e) {
    float s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
    return s;
}

// Residual of a floating-point subtraction: returns e with (a - b) == s + e exactly, where
// s = fl(a - b) (Knuth's TwoSum applied to a and -b).
__device__ __forceinline__ float sub_residual(float a, float b, float s) {
    const float bb = s - a;
    return (a - (s - bb)) - (b + bb);
}

// Hooke force of eq. (2) on mass i from one spring to a neighbour at (xj, yj, zj),
// accumulated into f; a zero-length spring contributes zero.
// EXACT: d = xj - xi is exact whenever the two coordinates are within a factor of two of
// each other (Sterbenz); near a coordinate plane it is not, and for a nearly relaxed spring
// that one-ulp error in d would be a large fraction of the elongation.  With EXACT the
// subtraction residuals r are folded into |d|^2 - L0^2 (as 2 d r), so the elongation is that
// of the stored positions whatever their magnitude.
template <bool EXACT>
__device__ __forceinline__ void hooke(float xi, float yi, float zi, float xj, float yj, float zj,
                                      float k, float l0, float& fx, float& fy, float& fz) {
    const float dx = xj - xi, dy = yj - yi, dz = zj - zi;
    const float px = dx * dx, py = dy * dy, pz = dz * dz;
    const float ex = __builtin_fmaf(dx, dx, -px);
    const float ey = __builtin_fmaf(dy, dy, -py);
    const float ez = __builtin_fmaf(dz, dz, -pz);
    const float q = l0 * l0;
    const float eq = __builtin_fmaf(l0, l0, -q);
    float e1, e2;
    const float s1 = two_sum(px, py, e1);
    const float s2 = two_sum(s1, pz, e2);
    // |d|^2 - L0^2 = (s2 - q) + (e1 + e2 + ex + ey + ez - eq); s2 - q is exact near rest
    float lo = ((e1 + e2) + (ex + ey)) + (ez - eq);
    if (EXACT) {
        const float rx = sub_residual(xj, xi, dx);
        const float ry = sub_residual(yj, yi, dy);
        const float rz = sub_residual(zj, zi, dz);
        lo = __builtin_fmaf(dx + dx, rx, lo);
        lo = __builtin_fmaf(dy + dy, ry, lo);
        lo = __builtin_fmaf(dz + dz, rz, lo);
    }
    const float diff = (s2 - q) + lo;
    const float len = __builtin_amdgcn_sqrtf(s2);
    const float den = (len + l0) * len;
    // computed unconditionally and then selected, so a zero length (padding entries) costs
    // no branch; the NaN of 0 * rcp(0) is discarded by the select
    float fac = k * diff * __builtin_amdgcn_rcpf(den);
    fac = len > 0.0f ? fac : 0.0f;
    fx = __builtin_fmaf(fac, dx, fx);
    fy = __builtin_fmaf(fac, dy, fy);
    fz = __builtin_fmaf(fac, dz, fz);
}

// Stage the workgroup's own positions and its halo in LDS.  Returns this lane's position.
__device__ __forceinline__ float4 stage_positions(float4* __restrict__ sx, const float4* __restrict__ xin,
                                                  const int32_t* __restrict__ halo_ptr,
                                                  const int32_t* __restrict__ halo_idx, int b, int base,
                                                  int n, int block) {
    const int t = threadIdx.x;
    const int i = base + t;
    float4 xi = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < n) xi = xin[i];
    sx[t] = xi;
    const int h0 = halo_ptr[b], h1 = halo_ptr[b + 1];
    for (int h = h0 + t; h < h1; h += block) sx[block + (h - h0)] = xin[halo_idx[h]];
    __syncthreads();
    return xi;
}

// Sum of the spring forces on this lane's mass over its slice entries.  The slice (and so the
// trip count) is uniform across the wavefront; entries are fetched in batches of kBatch so
// that several loads are in flight before the first is consumed.
constexpr int kBatch = 4;

template <bool ACT, bool EXACT>
__device__ __forceinline__ void gather(const float4* __restrict__ sx, float4 xi, int s, int nslice,
                                       const int32_t* __restrict__ slice_ptr,
                                       const uint16_t* __restrict__ nbr, const float2* __restrict__ kl,
                                       const uint16_t* __restrict__ grp, const float* __restrict__ factor,
                                       float& fx, float& fy, float& fz) {
    fx = fy = fz = 0.0f;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s >= nslice) return;
    const int lane = threadIdx.x & 63;
    const int e0 = __builtin_amdgcn_readfirstlane(slice_ptr[s]);
    const int w = __builtin_amdgcn_readfirstlane((slice_ptr[s + 1] - e0) >> 6);
    const uint16_t* pn = nbr + e0 + lane;
    const float2* pk = kl + e0 + lane;
    const uint16_t* pg = ACT ? grp + e0 + lane : nullptr;
    int r = 0;
    for (; r + kBatch <= w; r += kBatch) {
        int slot[kBatch];
        float2 c[kBatch];
        float f[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            slot[u] = pn[(r + u) * 64];
            c[u] = pk[(r + u) * 64];
            if (ACT) f[u] = factor[pg[(r + u) * 64]];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const float4 xj = sx[slot[u]];
            const float l0 = ACT ? c[u].y * f[u] : c[u].y;
            hooke<EXACT>(xi.x, xi.y, xi.z, xj.x, xj.y, xj.z, c[u].x, l0, fx, fy, fz);
        }
    }
    for (; r < w; ++r) {
        const int slot = pn[r * 64];
        const float2 c = pk[r * 64];
        const float l0 = ACT ? c.y * factor[pg[r * 64]] : c.y;
        const float4 xj = sx[slot];
        hooke<EXACT>(xi.x, xi.y, xi.z, xj.x, xj.y, xj.z, c.x, l0, fx, fy, fz);
    }
}

template <bool ACT, bool GROUND, bool FEXT, bool EXACT>
__global__ void __launch_bounds__(1024)
step_kernel(const float4* __restrict__ xin, const float* __restrict__ vin, float4* __restrict__ xout,
            float* __restrict__ vout, const int32_t* __restrict__ slice_ptr, const uint16_t* __restrict__ nbr,
            const float2* __restrict__ kl, const uint16_t* __restrict__ grp,
            const int32_t* __restrict__ halo_ptr, const int32_t* __restrict__ halo_idx,
            const float* __restrict__ factor, const float* __restrict__ fext, int n, int nblk, int nslice,
            int block, StepParams p) {
    extern __shared__ float4 sx[];
    const int b = logical_block(nblk);
    if (b >= nblk) return;
    const int base = b * block;
    const float4 xi = stage_positions(sx, xin, halo_ptr, halo_idx, b, base, n, block);
    float fx, fy, fz;
    gather<ACT, EXACT>(sx, xi, (base + (int)threadIdx.x) >> 6, nslice, slice_ptr, nbr, kl, grp, factor, fx, fy, fz);
    const int i = base + (int)threadIdx.x;
    if (i >= n) return;

    const float inv_m = xi.w;
    float vx = vin[3 * i + 0], vy = vin[3 * i + 1], vz = vin[3 * i + 2];
    float ax = __builtin_fmaf(fx, inv_m, p.gx);
    float ay = __builtin_fmaf(fy, inv_m, p.gy);
    float az = __builtin_fmaf(fz, inv_m, p.gz);
    if (FEXT) {
        ax = __builtin_fmaf(fext[3 * i + 0], inv_m, ax);
        ay = __builtin_fmaf(fext[3 * i + 1], inv_m, ay);
        az = __builtin_fmaf(fext[3 * i + 2], inv_m, az);
    }
    float fn = 0.0f;
    if (GROUND) {
        const float pen = p.ground_z - xi.z;
        fn = pen > 0.0f ? p.ground_k * pen : 0.0f;
        az = __builtin_fmaf(fn, inv_m, az);
    }
    vx = __builtin_fmaf(p.dt, ax, vx);
    vy = __builtin_fmaf(p.dt, ay, vy);
    vz = __builtin_fmaf(p.dt, az, vz);
    if (GROUND && fn > 0.0f) {
        // Coulomb clamp: the tangential speed loses mu F_n dt / m, or stops
        const float c = p.ground_mu * fn * p.dt * inv_m;
        const float sp = __builtin_sqrtf(vx * vx + vy * vy);
        const float sc = sp > c ? (sp - c) / sp : 0.0f;
        vx *= sc;
        vy *= sc;
    }
    vx *= p.damp;
    vy *= p.damp;
    vz *= p.damp;
    float nx = __builtin_fmaf(p.dt, vx, xi.x);
    float ny = __builtin_fmaf(p.dt, vy, xi.y);
    float nz = __builtin_fmaf(p.dt, vz, xi.z);
    if (inv_m == 0.0f) {  // fixed mass
        nx = xi.x;
        ny = xi.y;
        nz = xi.z;
        vx = vy = vz = 0.0f;
    }
    xout[i] = make_float4(nx, ny, nz, inv_m);
    vout[3 * i + 0] = vx;
    vout[3 * i + 1] = vy;
    vout[3 * i + 2] = vz;
}

// Total force of eq. (2) + contact normal at the current state (same gather as the step).
template <bool ACT>
__global__ void __launch_bounds__(1024)
forces_kernel(const float4* __restrict__ xin, const float* __restrict__ mass, const int32_t* __restrict__ slice_ptr,
              const uint16_t* __restrict__ nbr, const float2* __restrict__ kl, const uint16_t* __restrict__ grp,
              const int32_t* __restrict__ halo_ptr, const int32_t* __restrict__ halo_idx,
              const float* __restrict__ factor, const float* __restrict__ fext, float* __restrict__ fout, int n,
              int nblk, int nslice, int block, StepParams p) {
    extern __shared__ float4 sx[];
    const int b = logical_block(nblk);
    if (b >= nblk) return;
    const int base = b * block;
    const float4 xi = stage_positions(sx, xin, halo_ptr, halo_idx, b, base, n, block);
    float fx, fy, fz;
    gather<ACT, true>(sx, xi, (base + (int)threadIdx.x) >> 6, nslice, slice_ptr, nbr, kl, grp, factor, fx, fy, fz);
    const int i = base + (int)threadIdx.x;
    if (i >= n) return;
    const float m = mass[i];
    fx = __builtin_fmaf(m, p.gx, fx);
    fy = __builtin_fmaf(m, p.gy, fy);
    fz = __builtin_fmaf(m, p.gz, fz);
    if (fext) {
        fx += fext[3 * i + 0];
        fy += fext[3 * i + 1];
        fz += fext[3 * i + 2];
    }
    if (p.ground) {
        const float pen = p.ground_z - xi.z;
        if (pen > 0.0f) fz += p.ground_k * pen;
    }
    fout[3 * i + 0] = fx;
    fout[3 * i + 1] = fy;
    fout[3 * i + 2] = fz;
}

// Actuation table at t_n = n dt for the device step counter n: factor[g] = 1 + A_g sin(w t_n
// + phi_g) evaluated in FP64 and rounded once to FP32; factor[n_factor] = 1 (passive springs).
// With `advance`, the counter moves to n + 1 (the step that follows consumes the table).
// Launched as ONE workgroup, so the counter update cannot race with its reads.
__global__ void __launch_bounds__(1024)
actuation_kernel(const double* __restrict__ phase, const double* __restrict__ amp, double omega, double dt,
                 long long* __restrict__ step_ctr, float* __restrict__ factor, int n_factor, int advance) {
    const long long n = *step_ctr;
    const double t = (double)n * dt;
    for (int g = threadIdx.x; g < n_factor; g += blockDim.x)
        factor[g] = (float)(1.0 + amp[g] * sin(omega * t + phase[g]));
    if (threadIdx.x == 0) factor[n_factor] = 1.0f;
    __syncthreads();
    if (advance && threadIdx.x == 0) *step_ctr = n + 1;
}

// ---------------------------------------------------------------- FP64 diagnostics

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// One workgroup per chunk = (workgroup-block b, masses [m0, m1) of one body).  Every term is
// widened to FP64, reduced across the wavefront with cross-lane shuffles, then across the
// workgroup's wavefronts in a fixed order.  Spring energy is counted at the lower endpoint.
template <bool ACT>
__global__ void __launch_bounds__(1024)
diag_chunk_kernel(const float4* __restrict__ xin, const float* __restrict__ vin, const float* __restrict__ mass,
                  const int32_t* __restrict__ slice_ptr, const uint16_t* __restrict__ nbr,
                  const float2* __restrict__ kl, const uint16_t* __restrict__ grp,
                  const int32_t* __restrict__ halo_ptr, const int32_t* __restrict__ halo_idx,
                  const float* __restrict__ factor, const int4* __restrict__ chunks, double* __restrict__ part,
                  int n, int nslice, int block, StepParams p) {
    extern __shared__ float4 sx[];
    __shared__ double red[16][kDiagFields];
    const int4 ch = chunks[blockIdx.x];
    const int b = ch.x, base = b * block;
    const float4 xi = stage_positions(sx, xin, halo_ptr, halo_idx, b, base, n, block);
    const int t = threadIdx.x;
    const int i = base + t;
    const bool mine = i >= ch.y && i < ch.z;
    // fields: 0 ke, 1 pe_spring, 2 pe_grav, 3 pe_contact, 4-6 momentum, 7-9 sum m x,
    //         10 mass, 11-13 bbox max, 14-16 bbox min, 17 non-finite count
    double acc[18];
    for (int f = 0; f < 11; ++f) acc[f] = 0.0;
    acc[11] = acc[12] = acc[13] = -1e300;
    acc[14] = acc[15] = acc[16] = 1e300;
    acc[17] = 0.0;
    if (mine) {
        const double m = mass[i];
        const double x = xi.x, y = xi.y, z = xi.z;
        const double vx = vin[3 * i], vy = vin[3 * i + 1], vz = vin[3 * i + 2];
        acc[0] = 0.5 * m * (vx * vx + vy * vy + vz * vz);
        acc[2] = -m * ((double)p.gx * x + (double)p.gy * y + (double)p.gz * z);
        if (p.ground) {
            const double pen = (double)p.ground_z - z;
            if (pen > 0.0) acc[3] = 0.5 * (double)p.ground_k * pen * pen;
        }
        acc[4] = m * vx; acc[5] = m * vy; acc[6] = m * vz;
        acc[7] = m * x;  acc[8] = m * y;  acc[9] = m * z;
        acc[10] = m;
        acc[11] = x; acc[12] = y; acc[13] = z;
        acc[14] = x; acc[15] = y; acc[16] = z;
        const bool fin = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(vx) && isfinite(vy) && isfinite(vz);
        acc[17] = fin ? 0.0 : 1.0;
        // spring energy of springs whose other end has a larger index
        const int s = i >> 6;
        if (s < nslice) {
            const int lane = t & 63;
            const int e0 = slice_ptr[s];
            const int w = (slice_ptr[s + 1] - e0) >> 6;
            const int h0 = halo_ptr[b];
            int e = e0 + lane;
            double es = 0.0;
            for (int r = 0; r < w; ++r, e += 64) {
                const int slot = nbr[e];
                const int j = slot < block ? base + slot : halo_idx[h0 + slot - block];
                if (j <= i) continue;
                const float2 c = kl[e];
                double l0 = (double)c.y;
                if (ACT) l0 *= (double)factor[grp[e]];
                const float4 xj = sx[slot];
                const double dx = (double)xj.x - x, dy = (double)xj.y - y, dz = (double)xj.z - z;
                const double dl = sqrt(dx * dx + dy * dy + dz * dz) - l0;
                es += 0.5 * (double)c.x * dl * dl;
            }
            acc[1] = es;
        }
    }
    const int wv = t >> 6, nw = (blockDim.x + 63) >> 6;
    double r[18];
    for (int f = 0; f < 11; ++f) r[f] = wave_sum(acc[f]);
    for (int f = 11; f < 14; ++f) r[f] = wave_max(acc[f]);
    for (int f = 14; f < 17; ++f) r[f] = wave_min(acc[f]);
    r[17] = wave_sum(acc[17]);
    if ((t & 63) == 0)
        for (int f = 0; f < 18; ++f) red[wv][f] = r[f];
    __syncthreads();
    if (t == 0) {
        double o[18];
        for (int f = 0; f < 18; ++f) o[f] = red[0][f];
        for (int w2 = 1; w2 < nw; ++w2) {
            for (int f = 0; f < 11; ++f) o[f] += red[w2][f];
            for (int f = 11; f < 14; ++f) o[f] = fmax(o[f], red[w2][f]);
            for (int f = 14; f < 17; ++f) o[f] = fmin(o[f], red[w2][f]);
            o[17] += red[w2][17];
        }
        double* out = part + (size_t)blockIdx.x * kDiagFields;
        for (int f = 0; f < 18; ++f) out[f] = o[f];
    }
}

// Per body: sum its chunk partials in chunk order (fixed, independent of launch shape).
__global__ void diag_body_kernel(const double* __restrict__ part, const int32_t* __restrict__ body_chunk,
                                 double* __restrict__ out, int nb) {
    const int bdy = blockIdx.x * blockDim.x + threadIdx.x;
    if (bdy >= nb) return;
    double o[18];
    for (int f = 0; f < 18; ++f) o[f] = (f >= 11 && f < 14) ? -1e300 : (f >= 14 && f < 17 ? 1e300 : 0.0);
    for (int c = body_chunk[bdy]; c < body_chunk[bdy + 1]; ++c) {
        const double* q = part + (size_t)c * kDiagFields;
        for (int f = 0; f < 11; ++f) o[f] += q[f];
        for (int f = 11; f < 14; ++f) o[f] = fmax(o[f], q[f]);
        for (int f = 14; f < 17; ++f) o[f] = fmin(o[f], q[f]);
        o[17] += q[17];
    }
    double* d = out + (size_t)bdy * kDiagFields;
    for (int f = 0; f < 18; ++f) d[f] = o[f];
}

inline int grid_for(int64_t nblk) { return (int)(((nblk + 7) / 8) * 8); }

}  // namespace

hipError_t launch_step(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st) {
    const int nslice = (int)((d.n + 63) / 64);
    const size_t lds = (size_t)d.lds_slots * sizeof(float4);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid_for(d.nblk)), dim3(d.block), lds, st, d.x[cur], d.v[cur], d.x[cur ^ 1],
                           d.v[cur ^ 1], d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.factor, d.fext,
                           (int)d.n, (int)d.nblk, nslice, d.block, p);
    };
    const int key = (d.grp ? 8 : 0) | (p.ground ? 4 : 0) | (d.fext ? 2 : 0) | (p.exact ? 1 : 0);
    switch (key) {
        case 0: go(step_kernel<false, false, false, false>); break;
        case 1: go(step_kernel<false, false, false, true>); break;
        case 2: go(step_kernel<false, false, true, false>); break;
        case 3: go(step_kernel<false, false, true, true>); break;
        case 4: go(step_kernel<false, true, false, false>); break;
        case 5: go(step_kernel<false, true, false, true>); break;
        case 6: go(step_kernel<false, true, true, false>); break;
        case 7: go(step_kernel<false, true, true, true>); break;
        case 8: go(step_kernel<true, false, false, false>); break;
        case 9: go(step_kernel<true, false, false, true>); break;
        case 10: go(step_kernel<true, false, true, false>); break;
        case 11: go(step_kernel<true, false, true, true>); break;
        case 12: go(step_kernel<true, true, false, false>); break;
        case 13: go(step_kernel<true, true, false, true>); break;
        case 14: go(step_kernel<true, true, true, false>); break;
        default: go(step_kernel<true, true, true, true>); break;
    }
    return hipGetLastError();
}

hipError_t launch_actuation(const DeviceArrays& d, double omega, double dt, int advance, hipStream_t st) {
    hipLaunchKernelGGL(actuation_kernel, dim3(1), dim3(1024), 0, st, d.phase, d.amp, omega, dt, d.step_ctr, d.factor,
                       d.n_factor, advance);
    return hipGetLastError();
}

hipError_t launch_forces(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st) {
    const int nslice = (int)((d.n + 63) / 64);
    const size_t lds = (size_t)d.lds_slots * sizeof(float4);
    if (d.grp)
        hipLaunchKernelGGL(forces_kernel<true>, dim3(grid_for(d.nblk)), dim3(d.block), lds, st, d.x[cur], d.mass,
                           d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.factor, d.fext, d.fout, (int)d.n,
                           (int)d.nblk, nslice, d.block, p);
    else
        hipLaunchKernelGGL(forces_kernel<false>, dim3(grid_for(d.nblk)), dim3(d.block), lds, st, d.x[cur], d.mass,
                           d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.factor, d.fext, d.fout, (int)d.n,
                           (int)d.nblk, nslice, d.block, p);
    return hipGetLastError();
}

hipError_t launch_diagnostics(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st) {
    const int nslice = (int)((d.n + 63) / 64);
    const size_t lds = (size_t)d.lds_slots * sizeof(float4);
    if (d.grp)
        hipLaunchKernelGGL(diag_chunk_kernel<true>, dim3(d.n_chunks), dim3(d.block), lds, st, d.x[cur], d.v[cur],
                           d.mass, d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.factor, d.chunks,
                           d.chunk_part, (int)d.n, nslice, d.block, p);
    else
        hipLaunchKernelGGL(diag_chunk_kernel<false>, dim3(d.n_chunks), dim3(d.block), lds, st, d.x[cur], d.v[cur],
                           d.mass, d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.factor, d.chunks,
                           d.chunk_part, (int)d.n, nslice, d.block, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_body_kernel, dim3((d.nb + 63) / 64), dim3(64), 0, st, d.chunk_part, d.body_chunk,
                       d.body_out, d.nb);
    return hipGetLastError();
}

}  // namespace cronos
