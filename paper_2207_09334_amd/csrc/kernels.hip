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

#include <algorithm>

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

// Stage the workgroup's masses (in mass order) and its halo in LDS; returns the block-relative
// index of the mass this lane owns (lanes take the block's masses by decreasing degree).
__device__ __forceinline__ int stage_positions(float4* __restrict__ sx, const float4* __restrict__ xin,
                                               const int32_t* __restrict__ halo_ptr,
                                               const int32_t* __restrict__ halo_idx,
                                               const uint16_t* __restrict__ lane_mass, int b, int base, int n,
                                               int block) {
    const int t = threadIdx.x;
    const int own = lane_mass[base + t];
    float4 xt = make_float4(0.f, 0.f, 0.f, 0.f);
    if (base + t < n) xt = xin[base + t];
    sx[t] = xt;
    const int h0 = halo_ptr[b], h1 = halo_ptr[b + 1];
    for (int h = h0 + t; h < h1; h += block) sx[block + (h - h0)] = xin[halo_idx[h]];
    __syncthreads();
    return own;
}

// Sum of the spring forces on this lane's mass over its slice entries.  The slice (and so the
// trip count) is uniform across the wavefront; entries are fetched in batches of BATCH so
// that several loads are in flight before the first is consumed.
template <bool ACT, bool EXACT, int BATCH>
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
    for (; r + BATCH <= w; r += BATCH) {
        int slot[BATCH];
        float2 c[BATCH];
        float f[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            slot[u] = pn[(r + u) * 64];
            c[u] = pk[(r + u) * 64];
            if (ACT) f[u] = factor[pg[(r + u) * 64]];
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
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

// The same sum over the compact entry stream: one 32-bit word per entry holding the LDS slot
// (low 16 bits) and the index of the spring's (k, L0) pair in the simulation's parameter
// table (high 16 bits), the table being staged in LDS (st).
template <bool ACT, bool EXACT, int BATCH>
__device__ __forceinline__ void gather_table(const float4* __restrict__ sx, const float2* __restrict__ st, float4 xi,
                                             int s, int nslice, const int32_t* __restrict__ slice_ptr,
                                             const uint32_t* __restrict__ packed, const uint16_t* __restrict__ grp,
                                             const float* __restrict__ factor, float& fx, float& fy, float& fz) {
    fx = fy = fz = 0.0f;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s >= nslice) return;
    const int lane = threadIdx.x & 63;
    const int e0 = __builtin_amdgcn_readfirstlane(slice_ptr[s]);
    const int w = __builtin_amdgcn_readfirstlane((slice_ptr[s + 1] - e0) >> 6);
    const uint32_t* pp = packed + e0 + lane;
    const uint16_t* pg = ACT ? grp + e0 + lane : nullptr;
    int r = 0;
    for (; r + BATCH <= w; r += BATCH) {
        uint32_t q[BATCH];
        float f[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            q[u] = pp[(r + u) * 64];
            if (ACT) f[u] = factor[pg[(r + u) * 64]];
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const float4 xj = sx[q[u] & 0xFFFFu];
            const float2 c = st[q[u] >> 16];
            const float l0 = ACT ? c.y * f[u] : c.y;
            hooke<EXACT>(xi.x, xi.y, xi.z, xj.x, xj.y, xj.z, c.x, l0, fx, fy, fz);
        }
    }
    for (; r < w; ++r) {
        const uint32_t q = pp[r * 64];
        const float2 c = st[q >> 16];
        const float l0 = ACT ? c.y * factor[pg[r * 64]] : c.y;
        const float4 xj = sx[q & 0xFFFFu];
        hooke<EXACT>(xi.x, xi.y, xi.z, xj.x, xj.y, xj.z, c.x, l0, fx, fy, fz);
    }
}

struct StepArgs {
    const float4* __restrict__ xin;
    const float* __restrict__ vin;
    float4* __restrict__ xout;
    float* __restrict__ vout;
    const int32_t* __restrict__ slice_ptr;
    const uint16_t* __restrict__ nbr;
    const float2* __restrict__ kl;
    const uint16_t* __restrict__ grp;
    const int32_t* __restrict__ halo_ptr;
    const int32_t* __restrict__ halo_idx;
    const uint16_t* __restrict__ lane_mass;
    const float* __restrict__ factor;
    const float* __restrict__ fext;
    float* __restrict__ vstar_out;   // optional: velocity before friction and damping (adjoint recompute)
    const uint32_t* __restrict__ packed;   // compact entries (slot | table index << 16), or null
    const float2* __restrict__ table;      // (k, L0) pairs of the compact entries
    int n, nblk, nslice, block, n_table, lds_slots;
};

// One time step of the masses of workgroup-block b: gather, body forces, contact, friction,
// damping, symplectic Euler, fixed masses.
template <bool ACT, bool EXACT, int BATCH, bool TABLE>
__device__ __forceinline__ void step_block(float4* __restrict__ sx, const StepArgs& a, const StepParams& p, int b) {
    const int base = b * a.block;
    float2* st = reinterpret_cast<float2*>(sx + a.lds_slots);
    if (TABLE)
        for (int q = threadIdx.x; q < a.n_table; q += a.block) st[q] = a.table[q];
    const int own = stage_positions(sx, a.xin, a.halo_ptr, a.halo_idx, a.lane_mass, b, base, a.n, a.block);
    const float4 xi = sx[own];
    float fx, fy, fz;
    // Coordinates at least `safe` away from zero make every difference with a neighbour closer
    // than safe/2 exact (Sterbenz), and a spring longer than that is far from rest, where a
    // one-ulp error in d is negligible; such wavefronts skip the residual terms.
    bool plain = !EXACT;
    if (EXACT) {
        const float m = fminf(fminf(fabsf(xi.x), fabsf(xi.y)), fabsf(xi.z));
        plain = __builtin_amdgcn_ballot_w64(!(m >= p.safe)) == 0;
    }
    const int s = (base + (int)threadIdx.x) >> 6;
    if (TABLE) {
        if (plain) gather_table<ACT, false, BATCH>(sx, st, xi, s, a.nslice, a.slice_ptr, a.packed, a.grp, a.factor, fx, fy, fz);
        else gather_table<ACT, true, BATCH>(sx, st, xi, s, a.nslice, a.slice_ptr, a.packed, a.grp, a.factor, fx, fy, fz);
    } else {
        if (plain) gather<ACT, false, BATCH>(sx, xi, s, a.nslice, a.slice_ptr, a.nbr, a.kl, a.grp, a.factor, fx, fy, fz);
        else gather<ACT, true, BATCH>(sx, xi, s, a.nslice, a.slice_ptr, a.nbr, a.kl, a.grp, a.factor, fx, fy, fz);
    }
    const int i = base + own;
    if (i >= a.n) return;

    const float inv_m = xi.w;
    float vx = a.vin[3 * i + 0], vy = a.vin[3 * i + 1], vz = a.vin[3 * i + 2];
    float ax = __builtin_fmaf(fx, inv_m, p.gx);
    float ay = __builtin_fmaf(fy, inv_m, p.gy);
    float az = __builtin_fmaf(fz, inv_m, p.gz);
    if (a.fext) {
        ax = __builtin_fmaf(a.fext[3 * i + 0], inv_m, ax);
        ay = __builtin_fmaf(a.fext[3 * i + 1], inv_m, ay);
        az = __builtin_fmaf(a.fext[3 * i + 2], inv_m, az);
    }
    float fn = 0.0f;
    if (p.ground) {
        const float pen = p.ground_z - xi.z;
        fn = pen > 0.0f ? p.ground_k * pen : 0.0f;
        az = __builtin_fmaf(fn, inv_m, az);
    }
    vx = __builtin_fmaf(p.dt, ax, vx);
    vy = __builtin_fmaf(p.dt, ay, vy);
    vz = __builtin_fmaf(p.dt, az, vz);
    if (a.vstar_out) {
        a.vstar_out[3 * i + 0] = vx;
        a.vstar_out[3 * i + 1] = vy;
        a.vstar_out[3 * i + 2] = vz;
    }
    if (fn > 0.0f) {
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
    a.xout[i] = make_float4(nx, ny, nz, inv_m);
    a.vout[3 * i + 0] = vx;
    a.vout[3 * i + 1] = vy;
    a.vout[3 * i + 2] = vz;
}

// One workgroup per block.
template <bool ACT, bool EXACT, int BATCH, bool TABLE>
__global__ void __launch_bounds__(1024) step_kernel(StepArgs a, StepParams p) {
    extern __shared__ float4 sx[];
    const int b = logical_block(a.nblk);
    if (b >= a.nblk) return;
    step_block<ACT, EXACT, BATCH, TABLE>(sx, a, p, b);
}

// Persistent form: a fixed grid (a multiple of 8 workgroups) walks the blocks; workgroup w runs
// on XCD w % 8 and takes that XCD's contiguous eighth of the blocks in strides.
template <bool ACT, bool EXACT, int BATCH, bool TABLE>
__global__ void __launch_bounds__(1024) step_persistent(StepArgs a, StepParams p) {
    extern __shared__ float4 sx[];
    const int per = (a.nblk + 7) >> 3;
    const int xcd = (int)(blockIdx.x & 7u);
    const int stride = (int)(gridDim.x >> 3);
    for (int j = (int)(blockIdx.x >> 3); j < per; j += stride) {
        const int b = xcd * per + j;
        if (b >= a.nblk) break;
        step_block<ACT, EXACT, BATCH, TABLE>(sx, a, p, b);
        __syncthreads();  // LDS is restaged for the next block
    }
}

// Total force of eq. (2) + contact normal at the current state (same gather as the step).
template <bool ACT>
__global__ void __launch_bounds__(1024)
forces_kernel(const float4* __restrict__ xin, const float* __restrict__ mass, const int32_t* __restrict__ slice_ptr,
              const uint16_t* __restrict__ nbr, const float2* __restrict__ kl, const uint16_t* __restrict__ grp,
              const int32_t* __restrict__ halo_ptr, const int32_t* __restrict__ halo_idx,
              const uint16_t* __restrict__ lane_mass, const float* __restrict__ factor,
              const float* __restrict__ fext, float* __restrict__ fout, int n, int nblk, int nslice, int block,
              StepParams p) {
    extern __shared__ float4 sx[];
    const int b = logical_block(nblk);
    if (b >= nblk) return;
    const int base = b * block;
    const int own = stage_positions(sx, xin, halo_ptr, halo_idx, lane_mass, b, base, n, block);
    const float4 xi = sx[own];
    float fx, fy, fz;
    // the same choice of difference as the step, so this is the force the step integrates
    const float mc = fminf(fminf(fabsf(xi.x), fabsf(xi.y)), fabsf(xi.z));
    const bool plain = !p.exact || __builtin_amdgcn_ballot_w64(!(mc >= p.safe)) == 0;
    const int s = (base + (int)threadIdx.x) >> 6;
    if (plain) gather<ACT, false, 4>(sx, xi, s, nslice, slice_ptr, nbr, kl, grp, factor, fx, fy, fz);
    else gather<ACT, true, 4>(sx, xi, s, nslice, slice_ptr, nbr, kl, grp, factor, fx, fy, fz);
    const int i = base + own;
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
                 long long* __restrict__ step_ctr, float* __restrict__ factor, int n_factor, int advance,
                 long long n_explicit) {
    const long long n = n_explicit >= 0 ? n_explicit : *step_ctr;
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
                  const uint16_t* __restrict__ lane_mass, const float* __restrict__ factor,
                  const int4* __restrict__ chunks, double* __restrict__ part, int n, int nslice, int block,
                  StepParams p) {
    extern __shared__ float4 sx[];
    __shared__ double red[16][kDiagFields];
    const int4 ch = chunks[blockIdx.x];
    const int b = ch.x, base = b * block;
    const int own = stage_positions(sx, xin, halo_ptr, halo_idx, lane_mass, b, base, n, block);
    const float4 xi = sx[own];
    const int t = threadIdx.x;
    const int i = base + own;
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
        const double x = (double)xi.x + p.ox, y = (double)xi.y + p.oy, z = (double)xi.z + p.oz;
        const double vx = vin[3 * i], vy = vin[3 * i + 1], vz = vin[3 * i + 2];
        acc[0] = 0.5 * m * (vx * vx + vy * vy + vz * vz);
        acc[2] = -m * ((double)p.gx * x + (double)p.gy * y + (double)p.gz * z);
        if (p.ground) {
            const double pen = (double)p.ground_z - (double)xi.z;   // both in device coordinates
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
        const int s = (base + t) >> 6;
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
                const double dx = (double)xj.x - (double)xi.x, dy = (double)xj.y - (double)xi.y,
                             dz = (double)xj.z - (double)xi.z;
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

// ---------------------------------------------------------------- adjoint of one step
//
// For the loss L = sum_i w_i . x_i(T), with (x_bar', v_bar') the adjoints of the outputs of
// step n, the reverse of the step is (see the step above, in reverse order):
//   v'_bar_tot = v_bar' + dt x_bar'          (x' = x + dt v')
//   v**_bar    = (1 - d) v'_bar_tot          (damping)
//   v*_bar     = J^T v**_bar                 (friction clamp: J = I - (c/|v_t|)(I - u u^T) on
//                                             the tangential part when sliding, 0 when stuck)
//   c_bar      = -u . v**_bar_t,  c = mu k_g (z_g - z) dt / m  ->  z_bar += c_bar (-mu k_g dt / m)
//   w          = dt v*_bar / m               (adjoint of the force on the mass)
//   x_bar      = x_bar' - k_g w_z (contact) + sum_springs K_s (w_j - w_i)
//   K_s        = k [n n^T + (delta / l)(I - n n^T)]
//   theta_bar += (dL0/dtheta) k n . (w_j - w_i)   (actuated springs)
// Fixed masses (1/m = 0) have w = 0 and v_bar = 0.  adj_local computes everything but the
// spring sum; adj_gather adds the spring sum with the same LDS-staged incidence walk as the
// step, and accumulates each actuated spring's sensitivity in FP64, half from each end.

__global__ void __launch_bounds__(256)
adj_local_kernel(const float4* __restrict__ x, const float* __restrict__ vstar, const float* __restrict__ xb1,
                 const float* __restrict__ vb1, float4* __restrict__ w, float* __restrict__ vb0,
                 float* __restrict__ xbl, int n, StepParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 xi = x[i];
    const float inv_m = xi.w;
    const float tx = __builtin_fmaf(p.dt, xb1[3 * i + 0], vb1[3 * i + 0]);
    const float ty = __builtin_fmaf(p.dt, xb1[3 * i + 1], vb1[3 * i + 1]);
    const float tz = __builtin_fmaf(p.dt, xb1[3 * i + 2], vb1[3 * i + 2]);
    float gx = p.damp * tx, gy = p.damp * ty, gz = p.damp * tz;
    float zb = 0.0f;
    float wz_contact = 0.0f;
    if (inv_m == 0.0f) {
        w[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        vb0[3 * i + 0] = vb0[3 * i + 1] = vb0[3 * i + 2] = 0.0f;
        xbl[3 * i + 0] = xb1[3 * i + 0];
        xbl[3 * i + 1] = xb1[3 * i + 1];
        xbl[3 * i + 2] = xb1[3 * i + 2];
        return;
    }
    const float pen = p.ground ? p.ground_z - xi.z : 0.0f;
    const bool touching = pen > 0.0f;
    if (touching) {
        const float fn = p.ground_k * pen;
        const float c = p.ground_mu * fn * p.dt * inv_m;
        const float vx = vstar[3 * i + 0], vy = vstar[3 * i + 1];
        const float sp = __builtin_sqrtf(vx * vx + vy * vy);
        if (sp > c) {
            const float ux = vx / sp, uy = vy / sp;
            const float ug = ux * gx + uy * gy;
            const float r = c / sp;
            gx = gx - r * (gx - ux * ug);
            gy = gy - r * (gy - uy * ug);
            zb = -ug * (-p.ground_mu * p.ground_k * p.dt * inv_m);
        } else {
            gx = gy = 0.0f;
        }
    }
    const float wx = p.dt * gx * inv_m, wy = p.dt * gy * inv_m, wz = p.dt * gz * inv_m;
    if (touching) wz_contact = -p.ground_k * wz;
    w[i] = make_float4(wx, wy, wz, 0.0f);
    vb0[3 * i + 0] = gx;
    vb0[3 * i + 1] = gy;
    vb0[3 * i + 2] = gz;
    xbl[3 * i + 0] = xb1[3 * i + 0];
    xbl[3 * i + 1] = xb1[3 * i + 1];
    xbl[3 * i + 2] = xb1[3 * i + 2] + wz_contact + zb;
}

template <bool ACT>
__global__ void __launch_bounds__(1024)
adj_gather_kernel(const float4* __restrict__ x, const float4* __restrict__ w, const float* __restrict__ xbl,
                  float* __restrict__ xb0, const int32_t* __restrict__ slice_ptr, const uint16_t* __restrict__ nbr,
                  const float2* __restrict__ kl, const uint16_t* __restrict__ grp,
                  const int32_t* __restrict__ halo_ptr, const int32_t* __restrict__ halo_idx,
                  const uint16_t* __restrict__ lane_mass, const float* __restrict__ factor,
                  double2* __restrict__ sens, int n_factor, double cos_t, double sin_t, int n, int nblk, int nslice,
                  int block, int lds_slots) {
    extern __shared__ float4 sx[];
    float4* sw = sx + lds_slots;
    const int b = logical_block(nblk);
    if (b >= nblk) return;
    const int base = b * block;
    const int t = threadIdx.x;
    {
        float4 wt = make_float4(0.f, 0.f, 0.f, 0.f);
        if (base + t < n) wt = w[base + t];
        sw[t] = wt;
        const int h0 = halo_ptr[b], h1 = halo_ptr[b + 1];
        for (int h = h0 + t; h < h1; h += block) sw[block + (h - h0)] = w[halo_idx[h]];
    }
    const int own = stage_positions(sx, x, halo_ptr, halo_idx, lane_mass, b, base, n, block);
    const float4 xi = sx[own];
    const float4 wi = sw[own];
    float ax = 0.f, ay = 0.f, az = 0.f;
    const int s = __builtin_amdgcn_readfirstlane((base + t) >> 6);
    if (s < nslice) {
        const int lane = t & 63;
        const int e0 = __builtin_amdgcn_readfirstlane(slice_ptr[s]);
        const int wdt = __builtin_amdgcn_readfirstlane((slice_ptr[s + 1] - e0) >> 6);
        for (int r = 0; r < wdt; ++r) {
            const int e = e0 + r * 64 + lane;
            const int slot = nbr[e];
            const float2 c = kl[e];
            const int g = ACT ? (int)grp[e] : n_factor;
            const float l0 = ACT ? c.y * factor[g] : c.y;
            const float4 xj = sx[slot];
            const float4 wj = sw[slot];
            const float dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
            const float len2 = dx * dx + dy * dy + dz * dz;
            if (len2 > 0.0f) {
                const float len = __builtin_sqrtf(len2);
                const float il = 1.0f / len;
                const float nx = dx * il, ny = dy * il, nz = dz * il;
                const float dwx = wj.x - wi.x, dwy = wj.y - wi.y, dwz = wj.z - wi.z;
                const float ndw = nx * dwx + ny * dwy + nz * dwz;
                const float tr = 1.0f - l0 * il;        // delta / l
                const float k = c.x;
                ax += k * (nx * ndw + tr * (dwx - nx * ndw));
                ay += k * (ny * ndw + tr * (dwy - ny * ndw));
                az += k * (nz * ndw + tr * (dwz - nz * ndw));
                if (ACT && g < n_factor) {
                    const double q = 0.5 * (double)c.y * (double)k * (double)ndw;
                    double2 acc = sens[e];
                    acc.x += cos_t * q;
                    acc.y += sin_t * q;
                    sens[e] = acc;
                }
            }
        }
    }
    const int i = base + own;
    if (i >= n) return;
    xb0[3 * i + 0] = xbl[3 * i + 0] + ax;
    xb0[3 * i + 1] = xbl[3 * i + 1] + ay;
    xb0[3 * i + 2] = xbl[3 * i + 2] + az;
}

inline int grid_for(int64_t nblk) { return (int)(((nblk + 7) / 8) * 8); }

}  // namespace

hipError_t launch_step(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st) {
    return launch_step_io(d, d.x[cur], d.v[cur], d.x[cur ^ 1], d.v[cur ^ 1], nullptr, p, st);
}

hipError_t launch_step_io(const DeviceArrays& d, const float4* xin, const float* vin, float4* xout, float* vout,
                          float* vstar, const StepParams& p, hipStream_t st) {
    const bool table = d.packed != nullptr;
    StepArgs a{xin, vin, xout, vout, d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx,
               d.lane_mass, d.factor, d.fext, vstar, d.packed, d.table, (int)d.n, (int)d.nblk, (int)d.nslice, d.block,
               d.n_table, d.lds_slots};
    const size_t lds = (size_t)d.lds_slots * sizeof(float4) + (table ? (size_t)d.n_table * sizeof(float2) : 0);
    const bool persistent = d.persistent_groups > 0;
    const dim3 grid(persistent ? (unsigned)d.persistent_groups : (unsigned)grid_for(d.nblk));
    auto go = [&](auto normal, auto pers) {
        if (persistent) hipLaunchKernelGGL(pers, grid, dim3(d.block), lds, st, a, p);
        else hipLaunchKernelGGL(normal, grid, dim3(d.block), lds, st, a, p);
    };
#define CRONOS_GO(A, E, B, T) go(step_kernel<A, E, B, T>, step_persistent<A, E, B, T>)
#define CRONOS_GO_T(A, E, B) (table ? CRONOS_GO(A, E, B, true) : CRONOS_GO(A, E, B, false))
    const bool act = d.grp != nullptr, ex = p.exact != 0;
    if (d.batch == 8) {
        if (act) ex ? CRONOS_GO_T(true, true, 8) : CRONOS_GO_T(true, false, 8);
        else ex ? CRONOS_GO_T(false, true, 8) : CRONOS_GO_T(false, false, 8);
    } else if (d.batch == 2) {
        if (act) ex ? CRONOS_GO_T(true, true, 2) : CRONOS_GO_T(true, false, 2);
        else ex ? CRONOS_GO_T(false, true, 2) : CRONOS_GO_T(false, false, 2);
    } else {
        if (act) ex ? CRONOS_GO_T(true, true, 4) : CRONOS_GO_T(true, false, 4);
        else ex ? CRONOS_GO_T(false, true, 4) : CRONOS_GO_T(false, false, 4);
    }
#undef CRONOS_GO_T
#undef CRONOS_GO
    return hipGetLastError();
}

hipError_t persistent_grid(const DeviceArrays& d, int exact, int* grid) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const bool table = d.packed != nullptr;
    const size_t lds = (size_t)d.lds_slots * sizeof(float4) + (table ? (size_t)d.n_table * sizeof(float2) : 0);
    const void* k = d.grp ? (exact ? (const void*)step_persistent<true, true, 4, true> : (const void*)step_persistent<true, false, 4, true>)
                          : (exact ? (const void*)step_persistent<false, true, 4, true> : (const void*)step_persistent<false, false, 4, true>);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, d.block, lds);
    if (e != hipSuccess) return e;
    int g = std::max(1, per_cu) * cus;
    g = (g + 7) / 8 * 8;
    *grid = (int)std::min<int64_t>(g, grid_for(d.nblk));
    return hipSuccess;
}

hipError_t launch_actuation(const DeviceArrays& d, double omega, double dt, int advance, hipStream_t st,
                            long long n_explicit) {
    hipLaunchKernelGGL(actuation_kernel, dim3(1), dim3(1024), 0, st, d.phase, d.amp, omega, dt, d.step_ctr, d.factor,
                       d.n_factor, n_explicit >= 0 ? 0 : advance, n_explicit);
    return hipGetLastError();
}

hipError_t launch_forces(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st) {
    const int nslice = (int)d.nslice;
    const size_t lds = (size_t)d.lds_slots * sizeof(float4);
    if (d.grp)
        hipLaunchKernelGGL(forces_kernel<true>, dim3(grid_for(d.nblk)), dim3(d.block), lds, st, d.x[cur], d.mass,
                           d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.lane_mass, d.factor, d.fext,
                           d.fout, (int)d.n, (int)d.nblk, nslice, d.block, p);
    else
        hipLaunchKernelGGL(forces_kernel<false>, dim3(grid_for(d.nblk)), dim3(d.block), lds, st, d.x[cur], d.mass,
                           d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.lane_mass, d.factor, d.fext,
                           d.fout, (int)d.n, (int)d.nblk, nslice, d.block, p);
    return hipGetLastError();
}

hipError_t launch_diagnostics(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st) {
    const int nslice = (int)d.nslice;
    const size_t lds = (size_t)d.lds_slots * sizeof(float4);
    if (d.grp)
        hipLaunchKernelGGL(diag_chunk_kernel<true>, dim3(d.n_chunks), dim3(d.block), lds, st, d.x[cur], d.v[cur],
                           d.mass, d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.lane_mass, d.factor,
                           d.chunks, d.chunk_part, (int)d.n, nslice, d.block, p);
    else
        hipLaunchKernelGGL(diag_chunk_kernel<false>, dim3(d.n_chunks), dim3(d.block), lds, st, d.x[cur], d.v[cur],
                           d.mass, d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.lane_mass, d.factor,
                           d.chunks, d.chunk_part, (int)d.n, nslice, d.block, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_body_kernel, dim3((d.nb + 63) / 64), dim3(64), 0, st, d.chunk_part, d.body_chunk,
                       d.body_out, d.nb);
    return hipGetLastError();
}

hipError_t launch_adj_local(const DeviceArrays& d, const float4* x, const float* vstar, const float* xb1,
                            const float* vb1, float4* w, float* vb0, float* xbl, const StepParams& p, hipStream_t st) {
    hipLaunchKernelGGL(adj_local_kernel, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, st, x, vstar, xb1, vb1, w,
                       vb0, xbl, (int)d.n, p);
    return hipGetLastError();
}

hipError_t launch_adj_gather(const DeviceArrays& d, const float4* x, const float4* w, const float* xbl, float* xb0,
                             double2* sens, double cos_t, double sin_t, hipStream_t st) {
    const size_t lds = 2 * (size_t)d.lds_slots * sizeof(float4);
    if (d.grp)
        hipLaunchKernelGGL(adj_gather_kernel<true>, dim3(grid_for(d.nblk)), dim3(d.block), lds, st, x, w, xbl, xb0,
                           d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.lane_mass, d.factor, sens,
                           d.n_factor, cos_t, sin_t, (int)d.n, (int)d.nblk, (int)d.nslice, d.block, d.lds_slots);
    else
        hipLaunchKernelGGL(adj_gather_kernel<false>, dim3(grid_for(d.nblk)), dim3(d.block), lds, st, x, w, xbl, xb0,
                           d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx, d.lane_mass, d.factor, sens,
                           d.n_factor, cos_t, sin_t, (int)d.n, (int)d.nblk, (int)d.nslice, d.block, d.lds_slots);
    return hipGetLastError();
}

}  // namespace cronos
