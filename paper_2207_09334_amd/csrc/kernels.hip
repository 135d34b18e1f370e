// Device kernels of the mass-spring step for gfx950 (CDNA4, wave64).
//
// One time step is one launch of `step_kernel` (actuated bodies in the compact table forms
// compute their actuation factors inside it; the explicit form takes a separate actuation
// launch).  It fuses what Algorithm 1 splits into a spring pass and a mass pass: every lane
// owns one mass (or 2 or 4 lanes share one, `step_lanes_kernel`), walks that mass's incidence
// list in a fixed order and sums the eq. (2) spring forces itself, so no force is ever written
// twice and no atomic is needed; the sum is bitwise reproducible run to run.
//
// Memory: positions are float4 (x, y, z, 1/m) so one 16-byte load fetches a neighbour; a
// workgroup first copies its own masses and its halo (the neighbours outside the workgroup)
// into LDS, then every incidence reads its neighbour from LDS.  The incidence stream is laid
// out column-major per 64-mass slice, so each wavefront's loads are contiguous; in the compact
// forms an entry is one 16-bit word (passive bodies: neighbour slot and index into the LDS
// table of distinct (k, L0) pairs) or one 32-bit word (also the actuation factor).
// Workgroups are spread so that each of the 8 XCDs gets a contiguous range of the Morton
// order (their halos then overlap within one L2).  A workgroup's lanes take its masses in
// order of decreasing degree; where the step streams from HBM (actuated 32-bit form beyond the
// Infinity Cache) a variant reads the velocities and writes the new state through LDS in mass
// order instead of where each lane's mass lies.
//
// A full box of masses linked to all 26 grid neighbours takes `step_grid_kernel` instead: one
// 512-thread workgroup per aligned 8 x 8 x 8 cube stages the cube and its one-node halo as a
// 10 x 10 x 10 tile and reads each neighbour at a fixed tile offset, with no incidence data.
//
// Precision: FP32 state and FP32 accumulation.  The elongation |d| - L0 of a nearly relaxed
// spring is a difference of nearly equal numbers; it is computed as (|d|^2 - L0^2)/(|d| + L0)
// with |d|^2 - L0^2 formed in FP64 from the FP32 differences (exact squares, L0^2 held
// exactly), so its error is about an ulp of the elongation itself, not of L0.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace cronos {

namespace {

__device__ __forceinline__ int logical_block(int nblk) {
    const int per = (nblk + 7) >> 3;
    return (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
}

// Coordinate-difference modes of the spring arithmetic (see hooke_fac).
enum : int { kPlain = 0, kExactZ = 1, kExactAll = 2 };

// Scalar factor of the Hooke force of eq. (2) for the spring from (xi, yi, zi) to (xj, yj, zj):
// the force on the first end is fac * d with d = xj - xi; a zero-length spring gives 0 (its d
// is 0 and fac stays finite).  Every step below is unchanged, bit for bit, when d changes sign,
// so both ends of a spring see the same factor.
//
// Elongation: |d| - L0 = (|d|^2 - L0^2) / (|d| + L0).  The numerator is formed in FP64 from the
// FP32 differences: the square of a 24-bit value is exact in 53 bits, L0^2 (q) is held exactly,
// so near rest the cancellation in |d|^2 - L0^2 loses nothing that matters (the error is
// ~1e-16 of L0^2, against FP32's ~6e-8).  On this chip an FP64 FMA takes the issue slot of an
// FP32 one, so five FP64 operations replace the twenty-odd FP32 ones of an error-free FP32
// formulation.
// EX: d = xj - xi is exact in FP32 whenever the two coordinates are within a factor of two of
// each other (Sterbenz); near a coordinate plane it is not, and for a nearly relaxed spring
// that one-ulp error in d would be a large fraction of the elongation.  kExactAll takes the
// differences in FP64 (exact for any two FP32 values of similar scale), so the elongation is
// that of the stored positions whatever their magnitude; kExactZ does so for z only, for
// wavefronts near the z = 0 plane alone (the contact plane); kPlain widens the FP32 ones.
template <int EX>
__device__ __forceinline__ float hooke_fac(float xi, float yi, float zi, float xj, float yj, float zj, float k,
                                           float l0, double q, float& dx, float& dy, float& dz) {
    dx = xj - xi;
    dy = yj - yi;
    dz = zj - zi;
    double ex = dx, ey = dy, ez = dz;
    if (EX == kExactAll) {
        ex = (double)xj - (double)xi;
        ey = (double)yj - (double)yi;
    }
    if (EX != kPlain) ez = (double)zj - (double)zi;
    const double s = __builtin_fma(ex, ex, __builtin_fma(ey, ey, ez * ez));
    const float diff = (float)(s - q);
    const float s2 = (float)s;
    const float len = __builtin_amdgcn_sqrtf(s2);
    // |d| (|d| + L0) = s2 + L0 |d| to within an ulp; the floor keeps a zero-length spring's
    // factor finite (its force fac * d is then exactly 0) and is far below any real spring's
    const float den = __builtin_fmaxf(__builtin_fmaf(l0, len, s2), 1e-30f);
    return k * diff * __builtin_amdgcn_rcpf(den);
}

// The same with L0^2 formed here (exact in FP64).
template <int EX>
__device__ __forceinline__ float hooke_fac(float xi, float yi, float zi, float xj, float yj, float zj, float k,
                                           float l0, float& dx, float& dy, float& dz) {
    return hooke_fac<EX>(xi, yi, zi, xj, yj, zj, k, l0, (double)l0 * (double)l0, dx, dy, dz);
}

// Hooke force of eq. (2) on mass i from one spring to a neighbour at (xj, yj, zj),
// accumulated into f.
template <int EX>
__device__ __forceinline__ void hooke(float xi, float yi, float zi, float xj, float yj, float zj,
                                      float k, float l0, float& fx, float& fy, float& fz) {
    float dx, dy, dz;
    const float fac = hooke_fac<EX>(xi, yi, zi, xj, yj, zj, k, l0, dx, dy, dz);
    fx = __builtin_fmaf(fac, dx, fx);
    fy = __builtin_fmaf(fac, dy, fy);
    fz = __builtin_fmaf(fac, dz, fz);
}

// L0^2 of a parameter-table entry c = (k, L0, L0^2 as an FP64 value in its last two words).
__device__ __forceinline__ double table_l0sq(float4 c) {
    const unsigned long long bits =
        ((unsigned long long)__float_as_uint(c.w) << 32) | (unsigned long long)__float_as_uint(c.z);
    return __longlong_as_double((long long)bits);
}

// The same with a parameter-table entry c = (k, L0, L0^2 in FP64); an actuated spring scales L0
// by its factor g and squares it here.
template <bool ACT, int EX>
__device__ __forceinline__ float hooke_fac_tab(float4 xi, float4 xj, float4 c, float g, float& dx, float& dy,
                                               float& dz) {
    if (ACT) return hooke_fac<EX>(xi.x, xi.y, xi.z, xj.x, xj.y, xj.z, c.x, c.y * g, dx, dy, dz);
    return hooke_fac<EX>(xi.x, xi.y, xi.z, xj.x, xj.y, xj.z, c.x, c.y, table_l0sq(c), dx, dy, dz);
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
template <bool ACT, int EX, int BATCH>
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
            hooke<EX>(xi.x, xi.y, xi.z, xj.x, xj.y, xj.z, c[u].x, l0, fx, fy, fz);
        }
    }
    for (; r < w; ++r) {
        const int slot = pn[r * 64];
        const float2 c = pk[r * 64];
        const float l0 = ACT ? c.y * factor[pg[r * 64]] : c.y;
        const float4 xj = sx[slot];
        hooke<EX>(xi.x, xi.y, xi.z, xj.x, xj.y, xj.z, c.x, l0, fx, fy, fz);
    }
}

// LDS read at a byte address.  The step kernels declare no static LDS, so their dynamic LDS
// (positions first) starts at address 0 (checked on the host) and an entry word can carry
// ready-made byte addresses.
typedef float lds_vec4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 lds_f4(uint32_t byte) {
    const lds_vec4 v = *(const __attribute__((address_space(3))) lds_vec4*)(size_t)byte;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float lds_f1(uint32_t byte) {
    return *(const __attribute__((address_space(3))) float*)(size_t)byte;
}

// The same sum over the compact entry stream: one 32-bit word per entry and the parameter
// table of the simulation's distinct (k, L0) pairs staged in LDS at byte address T (a
// multiple of 8192, so "| T" adds it).
//   passive simulations: neighbour slot << 19 | pair index << 4, so the neighbour's byte
//     address is q >> 15 and the pair's is (q & 0x1FF0) | T;
//   actuated simulations: neighbour slot (bits 0-12) | pair index (bits 13-21) | index of
//     the spring's actuation factor in the workgroup's slice of the factor table, staged in
//     LDS at sf (bits 22-31, 0 = passive).
constexpr uint32_t kSlotBits = 13, kTypeBits = 9;

template <bool ACT>
__device__ __forceinline__ void decode_entry(uint32_t q, uint32_t tbase, uint32_t& xa, uint32_t& ca, uint32_t& g) {
    if (ACT) {
        xa = (q & ((1u << kSlotBits) - 1u)) << 4;
        ca = ((q >> (kSlotBits - 4)) & (((1u << kTypeBits) - 1u) << 4)) | tbase;
        g = q >> (kSlotBits + kTypeBits);
    } else {
        xa = q >> 15;
        ca = (q & (((1u << kTypeBits) - 1u) << 4)) | tbase;
        g = 0;
    }
}

template <bool ACT, int EX, int BATCH>
__device__ __forceinline__ void gather_table(uint32_t tbase, const float* __restrict__ sf, float4 xi, int s,
                                             int nslice, const int32_t* __restrict__ slice_ptr,
                                             const uint32_t* __restrict__ packed, float& fx, float& fy, float& fz) {
    fx = fy = fz = 0.0f;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s >= nslice) return;
    const int lane = threadIdx.x & 63;
    const int e0 = __builtin_amdgcn_readfirstlane(slice_ptr[s]);
    const int w = __builtin_amdgcn_readfirstlane((slice_ptr[s + 1] - e0) >> 6);
    const uint32_t* pp = packed + e0 + lane;
    auto one = [&](uint32_t q) {
        uint32_t xa, ca, gi;
        decode_entry<ACT>(q, tbase, xa, ca, gi);
        const float4 xj = lds_f4(xa);
        const float4 c = lds_f4(ca);
        const float g = ACT ? sf[gi] : 1.0f;
        float dx, dy, dz;
        const float fac = hooke_fac_tab<ACT, EX>(xi, xj, c, g, dx, dy, dz);
        fx = __builtin_fmaf(fac, dx, fx);
        fy = __builtin_fmaf(fac, dy, fy);
        fz = __builtin_fmaf(fac, dz, fz);
    };
    int r = 0;
    for (; r + BATCH <= w; r += BATCH) {
        uint32_t q[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) q[u] = pp[(r + u) * 64];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) one(q[u]);
    }
    for (; r < w; ++r) one(pp[r * 64]);
}

// The same sum over 16-bit entries (passive simulations whose LDS slots and (k, L0) pairs fit
// together in 16 bits): neighbour slot << tb | pair index.  Half the entry stream of the
// 32-bit form, which is most of what a step reads from HBM.
template <int EX, int BATCH>
__device__ __forceinline__ void gather_narrow(uint32_t tbase, float4 xi, int s, int nslice,
                                              const int32_t* __restrict__ slice_ptr,
                                              const uint16_t* __restrict__ narrow, int tb, float& fx, float& fy,
                                              float& fz) {
    fx = fy = fz = 0.0f;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s >= nslice) return;
    const int lane = threadIdx.x & 63;
    const int e0 = __builtin_amdgcn_readfirstlane(slice_ptr[s]);
    const int w = __builtin_amdgcn_readfirstlane((slice_ptr[s + 1] - e0) >> 6);
    const uint16_t* pp = narrow + e0 + lane;
    const uint32_t tmask = (1u << tb) - 1u;
    auto one = [&](uint32_t q) {
        const float4 xj = lds_f4((q >> tb) << 4);
        const float4 c = lds_f4(((q & tmask) << 4) | tbase);
        float dx, dy, dz;
        const float fac = hooke_fac_tab<false, EX>(xi, xj, c, 1.0f, dx, dy, dz);
        fx = __builtin_fmaf(fac, dx, fx);
        fy = __builtin_fmaf(fac, dy, fy);
        fz = __builtin_fmaf(fac, dz, fz);
    };
    int r = 0;
    for (; r + BATCH <= w; r += BATCH) {
        uint32_t q[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) q[u] = pp[(r + u) * 64];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) one(q[u]);
    }
    for (; r < w; ++r) one(pp[r * 64]);
}

// Split form of the same sum, in two passes over the workgroup's LDS.
// Spring pass: every spring with an end among the workgroup's masses is evaluated once (a
// spring between two of them is shared; one to a halo mass is evaluated here and again by
// the workgroup that owns the other end), its force factor stored in LDS (sfac).  Record
// word: LDS slot of the first end (bits 0-9, always a workgroup mass), LDS slot of the other
// end (bits 10-22), (k, L0) pair index (bits 23-31); actuated springs carry their local
// factor index in a parallel 16-bit stream.
constexpr uint32_t kRecA = 10, kRecB = 13;

template <bool ACT, bool EXACT, int BATCH>
__device__ __forceinline__ void spring_pass(const float4* __restrict__ sx, uint32_t tbase,
                                            const float* __restrict__ sf, float* __restrict__ sfac,
                                            const uint32_t* __restrict__ rec, const uint16_t* __restrict__ rgrp,
                                            int n_sp, int block, float safe) {
    const int lane = threadIdx.x & 63;
    const int w0 = (int)(threadIdx.x & ~63u);
    if (threadIdx.x == 0) sfac[n_sp] = 0.0f;  // the factor of the padding entries
    for (int j0 = __builtin_amdgcn_readfirstlane(w0); j0 < n_sp; j0 += BATCH * block) {
        uint32_t r[BATCH];
        float g[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {  // lanes past the end re-read the last record
            const int j = min(j0 + u * block + lane, n_sp - 1);
            r[u] = rec[j];
            if (ACT) g[u] = sf[rgrp[j]];
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int j = j0 + u * block + lane;
            const float4 xa = lds_f4((r[u] << 4) & (((1u << kRecA) - 1u) << 4));
            const float4 xb = lds_f4((r[u] >> (kRecA - 4)) & (((1u << kRecB) - 1u) << 4));
            const float4 c = lds_f4(((r[u] >> (kRecA + kRecB)) << 4) | tbase);
            bool plain = !EXACT;
            if (EXACT) {
                const float m = fminf(fminf(fabsf(xa.x), fabsf(xa.y)), fabsf(xa.z));
                plain = __builtin_amdgcn_ballot_w64(j < n_sp && !(m >= safe)) == 0;
            }
            float dx, dy, dz, fac;
            if (plain) fac = hooke_fac_tab<ACT, kPlain>(xa, xb, c, ACT ? g[u] : 1.0f, dx, dy, dz);
            else fac = hooke_fac_tab<ACT, kExactAll>(xa, xb, c, ACT ? g[u] : 1.0f, dx, dy, dz);
            if (j < n_sp) sfac[j] = fac;
        }
    }
}

// Gather pass: each lane walks its mass's entries in the usual order; an entry holds the
// neighbour's LDS slot (bits 0-12) and the index of the spring's factor in sfac (bits 13-31).
// Its arithmetic is light, so the entry loads would sit exposed: the first kPre entries of
// the slice are loaded (`prefetch_entries`) before the spring pass and consumed after it.
constexpr int kPre = 16;

struct SliceEntries {
    const uint32_t* pp;  // this lane's first entry
    int w;               // entries per lane (uniform over the wavefront)
    uint32_t pre[kPre];
};

__device__ __forceinline__ void prefetch_entries(SliceEntries& se, int s, int nslice,
                                                 const int32_t* __restrict__ slice_ptr,
                                                 const uint32_t* __restrict__ packed) {
    s = __builtin_amdgcn_readfirstlane(s);
    se.w = 0;
    se.pp = packed;
    if (s >= nslice) return;
    const int e0 = __builtin_amdgcn_readfirstlane(slice_ptr[s]);
    se.w = __builtin_amdgcn_readfirstlane((slice_ptr[s + 1] - e0) >> 6);
    se.pp = packed + e0 + (threadIdx.x & 63);
#pragma unroll
    for (int u = 0; u < kPre; ++u)
        if (u < se.w) se.pre[u] = se.pp[u * 64];
}

template <int BATCH>
__device__ __forceinline__ void gather_split(uint32_t fbase, float4 xi, const SliceEntries& se, float& fx, float& fy,
                                             float& fz) {
    fx = fy = fz = 0.0f;
    auto one = [&](uint32_t q) {
        const float4 xj = lds_f4((q & ((1u << kSlotBits) - 1u)) << 4);
        const float fac = lds_f1(((q >> kSlotBits) << 2) + fbase);
        fx = __builtin_fmaf(fac, xj.x - xi.x, fx);
        fy = __builtin_fmaf(fac, xj.y - xi.y, fy);
        fz = __builtin_fmaf(fac, xj.z - xi.z, fz);
    };
#pragma unroll
    for (int u = 0; u < kPre; ++u)
        if (u < se.w) one(se.pre[u]);
    int r = kPre;
    for (; r + BATCH <= se.w; r += BATCH) {
        uint32_t q[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) q[u] = se.pp[(r + u) * 64];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) one(q[u]);
    }
    for (; r < se.w; ++r) one(se.pp[r * 64]);
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
    const uint32_t* __restrict__ packed;   // compact entries (see gather_table), or null
    const uint16_t* __restrict__ narrow;   // 16-bit compact entries (see gather_narrow), or null
    const float4* __restrict__ table;      // (k, L0, L0^2 in FP64) of the compact entries
    const int2* __restrict__ blk_groups;   // per workgroup: first factor index and count
    const uint32_t* __restrict__ sp_rec;   // split form: spring records, workgroup after workgroup
    const uint16_t* __restrict__ sp_grp;   // split form: local actuation factor index per record
    const int32_t* __restrict__ sp_ptr;    // split form: first record of each workgroup
    int n, nblk, nslice, block, n_table, lds_slots, max_local_groups;
    int narrow_tb;                         // pair-index bits of the 16-bit entries
    // fused actuation (actuated table forms): each workgroup computes its factors for step
    // n = *step_in from phase and amp; one thread stores n + 1 to *step_out (the other slot of
    // the counter pair, so no workgroup of this launch reads it)
    int fuse;
    const float* __restrict__ phase;
    const float* __restrict__ amp;
    const long long* step_in;
    long long* step_out;
    unsigned long long cycles;
};

// Difference mode of a wavefront (uniform across it).  A coordinate at least `safe` away from
// zero makes its difference with any neighbour closer than safe/2 exact (Sterbenz), and a
// spring longer than that is far from rest, where a one-ulp error in d is negligible; so an
// axis needs the residual terms only if some mass of the wavefront is nearer its plane.
__device__ __forceinline__ int difference_mode(float4 xi, float safe) {
    const bool nx = __builtin_amdgcn_ballot_w64(!(fabsf(xi.x) >= safe)) != 0;
    const bool ny = __builtin_amdgcn_ballot_w64(!(fabsf(xi.y) >= safe)) != 0;
    const bool nz = __builtin_amdgcn_ballot_w64(!(fabsf(xi.z) >= safe)) != 0;
    return (nx || ny) ? kExactAll : nz ? kExactZ : kPlain;
}

// The exact-difference loop holds more live values per entry; it loads half as far ahead so
// that it does not raise the kernel's register count (and cut its occupancy).
template <int BATCH>
constexpr int kExactBatch = BATCH > 2 ? BATCH / 2 : BATCH;

// Per-launch arguments of the resident form (see step_resident).
struct ResidentArgs {
    const float* __restrict__ phase;
    const float* __restrict__ amp;
    unsigned long long cycles;
    const long long* step_in;   // step index of the input state (one slot of the counter pair)
    long long* step_out;        // receives the index after the launch (the other slot)
    int steps;
    float dtv0;
    int staged;                 // compact entries copied into LDS after the factors (0: none)
};

// Step modes: explicit (k, L0) per entry, compact entries with the parameter table, split.
enum : int { kExplicit = 0, kTable = 1, kSplit = 2, kNarrow = 3 };

// Elapsed fraction of an actuation period at step n, frac(n f dt), formed exactly in 64-bit
// fixed point (n * cycles wraps modulo 2^64), and the factor 1 + A sin(2 pi u + phi).
__device__ __forceinline__ float period_fraction(long long n, unsigned long long cycles) {
    const unsigned long long frac = (unsigned long long)n * cycles;
    return (float)(unsigned)(frac >> 32) * 0x1p-32f;
}
__device__ __forceinline__ float actuation_factor(float amp, float phase, float u) {
    return __builtin_fmaf(amp, sinf(__builtin_fmaf(6.28318531f, u, phase)), 1.0f);
}

// Body forces, contact, friction, damping and the symplectic Euler update of one mass with
// spring force f: v* = v + dtv a (v* is stored to vstar when given), Coulomb clamp, damping,
// x' = x + dt v'; a fixed mass (1/m = 0) keeps x and gets v' = 0.  dtv is dt except in
// Verlet's first step (dt / 2).
__device__ __forceinline__ void integrate(const StepParams& p, float dtv, float4 xi, float fx, float fy, float fz,
                                          const float* __restrict__ fext, float& vx, float& vy, float& vz,
                                          float4& xo, float* __restrict__ vstar) {
    const float inv_m = xi.w;
    float ax = __builtin_fmaf(fx, inv_m, p.gx);
    float ay = __builtin_fmaf(fy, inv_m, p.gy);
    float az = __builtin_fmaf(fz, inv_m, p.gz);
    if (fext) {
        ax = __builtin_fmaf(fext[0], inv_m, ax);
        ay = __builtin_fmaf(fext[1], inv_m, ay);
        az = __builtin_fmaf(fext[2], inv_m, az);
    }
    float fn = 0.0f;
    if (p.ground) {
        const float pen = p.ground_z - xi.z;
        fn = pen > 0.0f ? p.ground_k * pen : 0.0f;
        az = __builtin_fmaf(fn, inv_m, az);
    }
    vx = __builtin_fmaf(dtv, ax, vx);
    vy = __builtin_fmaf(dtv, ay, vy);
    vz = __builtin_fmaf(dtv, az, vz);
    if (vstar) {
        vstar[0] = vx;
        vstar[1] = vy;
        vstar[2] = vz;
    }
    if (fn > 0.0f) {
        // Coulomb clamp: the tangential speed loses mu F_n dtv / m, or stops
        const float c = p.ground_mu * fn * dtv * inv_m;
        const float sp = __builtin_sqrtf(vx * vx + vy * vy);
        const float sc = sp > c ? (sp - c) / sp : 0.0f;
        vx *= sc;
        vy *= sc;
    }
    vx *= p.damp;
    vy *= p.damp;
    vz *= p.damp;
    xo = make_float4(__builtin_fmaf(p.dt, vx, xi.x), __builtin_fmaf(p.dt, vy, xi.y), __builtin_fmaf(p.dt, vz, xi.z),
                     inv_m);
    if (inv_m == 0.0f) {  // fixed mass
        xo = xi;
        vx = vy = vz = 0.0f;
    }
}

// One time step of the masses of workgroup-block b: gather, body forces, contact, friction,
// damping, symplectic Euler, fixed masses.
template <bool ACT, bool EXACT, int BATCH, int MODE, bool STAGE = false>
__device__ __forceinline__ void step_block(float4* __restrict__ sx, const StepArgs& a, const StepParams& p, int b,
                                           long long n_step) {
    constexpr bool TABLE = MODE != kExplicit;
    const int base = b * a.block;
    const uint32_t tbase = table_base(a.lds_slots);
    float4* st = reinterpret_cast<float4*>(reinterpret_cast<char*>(sx) + tbase);
    float* sf = reinterpret_cast<float*>(st + a.n_table);
    float* sfac = sf + a.max_local_groups + 1;
    if (TABLE) {
        for (int q = threadIdx.x; q < a.n_table; q += a.block) st[q] = a.table[q];
        if (ACT) {
            const int2 bg = a.blk_groups[b];
            if (a.fuse) {   // the same formula as actuation_kernel, for this workgroup's factors only
                const float u = period_fraction(n_step, a.cycles);
                for (int q = threadIdx.x; q <= bg.y; q += a.block)
                    sf[q] = q ? actuation_factor(a.amp[bg.x + q - 1], a.phase[bg.x + q - 1], u) : 1.0f;
            } else {
                for (int q = threadIdx.x; q <= bg.y; q += a.block) sf[q] = q ? a.factor[bg.x + q - 1] : 1.0f;
            }
        }
    }
    // velocities read in mass order (one contiguous run), handed to each mass's lane through LDS below
    float vt0 = 0.0f, vt1 = 0.0f, vt2 = 0.0f;
    if (STAGE && base + (int)threadIdx.x < a.n) {
        const long q = 3 * (long)(base + (int)threadIdx.x);
        vt0 = a.vin[q + 0];
        vt1 = a.vin[q + 1];
        vt2 = a.vin[q + 2];
    }
    const int own = stage_positions(sx, a.xin, a.halo_ptr, a.halo_idx, a.lane_mass, b, base, a.n, a.block);
    const float4 xi = sx[own];
    float fx, fy, fz;
    const int s = (base + (int)threadIdx.x) >> 6;
    if (MODE == kSplit) {
        SliceEntries se;
        prefetch_entries(se, s, a.nslice, a.slice_ptr, a.packed);
        const int r0 = a.sp_ptr[b];
        spring_pass<ACT, EXACT, BATCH>(sx, tbase, sf, sfac, a.sp_rec + r0, ACT ? a.sp_grp + r0 : nullptr,
                                       a.sp_ptr[b + 1] - r0, a.block, p.safe);
        __syncthreads();
        gather_split<BATCH>(tbase + (uint32_t)(reinterpret_cast<char*>(sfac) - reinterpret_cast<char*>(st)), xi, se,
                            fx, fy, fz);
    } else {
        const int mode = EXACT ? difference_mode(xi, p.safe) : kPlain;
        if (MODE == kNarrow) {   // passive only (the host never picks it for actuation)
            if (mode == kPlain)
                gather_narrow<kPlain, BATCH>(tbase, xi, s, a.nslice, a.slice_ptr, a.narrow, a.narrow_tb, fx, fy, fz);
            else if (mode == kExactZ)
                gather_narrow<kExactZ, BATCH>(tbase, xi, s, a.nslice, a.slice_ptr, a.narrow, a.narrow_tb, fx, fy, fz);
            else
                gather_narrow<kExactAll, kExactBatch<BATCH>>(tbase, xi, s, a.nslice, a.slice_ptr, a.narrow, a.narrow_tb,
                                                             fx, fy, fz);
        } else if (TABLE) {
            if (mode == kPlain) gather_table<ACT, kPlain, BATCH>(tbase, sf, xi, s, a.nslice, a.slice_ptr, a.packed, fx, fy, fz);
            else if (mode == kExactZ)
                gather_table<ACT, kExactZ, BATCH>(tbase, sf, xi, s, a.nslice, a.slice_ptr, a.packed, fx, fy, fz);
            else gather_table<ACT, kExactAll, kExactBatch<BATCH>>(tbase, sf, xi, s, a.nslice, a.slice_ptr, a.packed, fx, fy, fz);
        } else {
            if (mode == kPlain) gather<ACT, kPlain, BATCH>(sx, xi, s, a.nslice, a.slice_ptr, a.nbr, a.kl, a.grp, a.factor, fx, fy, fz);
            else if (mode == kExactZ)
                gather<ACT, kExactZ, BATCH>(sx, xi, s, a.nslice, a.slice_ptr, a.nbr, a.kl, a.grp, a.factor, fx, fy, fz);
            else gather<ACT, kExactAll, kExactBatch<BATCH>>(sx, xi, s, a.nslice, a.slice_ptr, a.nbr, a.kl, a.grp, a.factor, fx, fy, fz);
        }
    }
    const int i = base + own;
    if (!STAGE) {
        if (i >= a.n) return;
        float vx = a.vin[3 * i + 0], vy = a.vin[3 * i + 1], vz = a.vin[3 * i + 2];
        float4 xo;
        integrate(p, p.dtv, xi, fx, fy, fz, a.fext ? a.fext + 3 * i : nullptr, vx, vy, vz, xo,
                  a.vstar_out ? a.vstar_out + 3 * i : nullptr);
        a.xout[i] = xo;
        a.vout[3 * i + 0] = vx;
        a.vout[3 * i + 1] = vy;
        a.vout[3 * i + 2] = vz;
        return;
    }
    // The lane->mass map scatters a wavefront's masses over the block, and scattered 16- and
    // 12-byte accesses reach HBM as partly used lines: velocities come in (loaded above in
    // mass order) and the new state goes out through LDS (the staged positions and tables
    // are no longer read), one contiguous run per array.  The launch provides 40 bytes of LDS
    // per mass for it.  Two more barriers: a memory-bound system gains (the actuated
    // population: 317 -> 298 us per step), a compute-bound one loses (the 16-bit-entry
    // cantilever: 18.5 -> 20.6 us), so only the actuated 32-bit table form has the staged
    // variant, taken where the step's bytes exceed the Infinity Cache.
    __syncthreads();
    float4* ox = sx;
    float* ov = reinterpret_cast<float*>(sx + a.block);
    float* ovin = ov + 3 * a.block;
    ovin[3 * threadIdx.x + 0] = vt0;
    ovin[3 * threadIdx.x + 1] = vt1;
    ovin[3 * threadIdx.x + 2] = vt2;
    __syncthreads();
    float vx = 0.0f, vy = 0.0f, vz = 0.0f;
    float4 xo;
    if (i < a.n) {
        vx = ovin[3 * own + 0];
        vy = ovin[3 * own + 1];
        vz = ovin[3 * own + 2];
        integrate(p, p.dtv, xi, fx, fy, fz, a.fext ? a.fext + 3 * i : nullptr, vx, vy, vz, xo,
                  a.vstar_out ? a.vstar_out + 3 * i : nullptr);
    }
    if (i < a.n) {
        ox[own] = xo;
        ov[3 * own + 0] = vx;
        ov[3 * own + 1] = vy;
        ov[3 * own + 2] = vz;
    }
    __syncthreads();
    const int cnt = min(a.block, a.n - base);
    for (int q = threadIdx.x; q < cnt; q += a.block) a.xout[base + q] = ox[q];
    for (int q = threadIdx.x; q < 3 * cnt; q += a.block) a.vout[3 * (long)base + q] = ov[q];
}

// A fused-actuation launch hands the next one its step index through the other slot of the
// counter pair (the next launch reads that slot; the kernel boundary orders the two).
__device__ __forceinline__ void advance_step(const StepArgs& a, long long n_step) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.step_out = n_step + 1;
}

template <bool ACT, bool EXACT, int BATCH, int MODE, bool STAGE = false>
__global__ void __launch_bounds__(1024) step_kernel(StepArgs a, StepParams p) {
    extern __shared__ float4 sx[];
    constexpr bool FUSABLE = ACT && MODE != kExplicit;
    const int b = logical_block(a.nblk);
    const long long n_step = FUSABLE && a.fuse ? *a.step_in : 0;
    if (FUSABLE && a.fuse) advance_step(a, n_step);
    if (b < a.nblk) step_block<ACT, EXACT, BATCH, MODE, STAGE>(sx, a, p, b, n_step);
}

// Several lanes per mass (LPM = 2 or 4; compact table forms): lane j of a mass's group walks its
// incidence rows j, j + LPM, ... and the groups' partial sums are combined by a fixed pairing
// of cross-lane exchanges (the same value in every lane of the group).  More wavefronts for
// the same masses, each with a shorter dependent chain: for bodies too small to fill the chip.
// The sum is grouped differently from the one-lane form, so the two agree to rounding only.
template <bool ACT, int EX, int LPM, bool NARROW>
__device__ __forceinline__ void gather_lanes(uint32_t tbase, const float* __restrict__ sf, float4 xi, int s, int sub,
                                             int nslice, const int32_t* __restrict__ slice_ptr,
                                             const uint32_t* __restrict__ packed, const uint16_t* __restrict__ narrow,
                                             int tb, float& fx, float& fy, float& fz) {
    fx = fy = fz = 0.0f;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s < nslice) {
        const int lane = ((int)threadIdx.x / LPM) & 63;
        const int e0 = __builtin_amdgcn_readfirstlane(slice_ptr[s]);
        const int w = __builtin_amdgcn_readfirstlane((slice_ptr[s + 1] - e0) >> 6);
        const int rows = (w + LPM - 1) / LPM;
        const uint32_t tmask = (1u << tb) - 1u;
        auto one = [&](uint32_t q) {
            uint32_t xa, ca, gi = 0;
            if (NARROW) {
                xa = (q >> tb) << 4;
                ca = ((q & tmask) << 4) | tbase;
            } else {
                decode_entry<ACT>(q, tbase, xa, ca, gi);
            }
            const float4 xj = lds_f4(xa);
            const float4 c = lds_f4(ca);
            const float g = ACT ? sf[gi] : 1.0f;
            float dx, dy, dz;
            const float fac = hooke_fac_tab<ACT, EX>(xi, xj, c, g, dx, dy, dz);
            fx = __builtin_fmaf(fac, dx, fx);
            fy = __builtin_fmaf(fac, dy, fy);
            fz = __builtin_fmaf(fac, dz, fz);
        };
        constexpr int B = 2;
        for (int k = 0; k < rows; k += B) {
            uint32_t q[B];
            bool ok[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int r = (k + u) * LPM + sub;
                ok[u] = r < w;
                const int e = e0 + r * 64 + lane;
                q[u] = ok[u] ? (NARROW ? (uint32_t)narrow[e] : packed[e]) : 0u;
            }
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (ok[u]) one(q[u]);
        }
    }
#pragma unroll
    for (int o = 1; o < LPM; o <<= 1) {
        fx += __shfl_xor(fx, o, 64);
        fy += __shfl_xor(fy, o, 64);
        fz += __shfl_xor(fz, o, 64);
    }
}

// One step with LPM lanes per mass: a workgroup of block * LPM threads stages its block's
// positions and halo, thread t serves mass lane t / LPM; the first lane of each mass
// integrates.  Compact table forms (32- or 16-bit entries), one workgroup per block.
template <bool ACT, bool EXACT, int LPM, bool NARROW>
__global__ void __launch_bounds__(1024) step_lanes_kernel(StepArgs a, StepParams p) {
    extern __shared__ float4 sx[];
    const int b = logical_block(a.nblk);
    const long long n_step = ACT && a.fuse ? *a.step_in : 0;
    if (ACT && a.fuse) advance_step(a, n_step);
    if (b >= a.nblk) return;
    const int t = (int)threadIdx.x, nt = (int)blockDim.x;
    const int m = t / LPM, sub = t % LPM;
    const int base = b * a.block;
    const uint32_t tbase = table_base(a.lds_slots);
    float4* st = reinterpret_cast<float4*>(reinterpret_cast<char*>(sx) + tbase);
    float* sf = reinterpret_cast<float*>(st + a.n_table);
    for (int q = t; q < a.n_table; q += nt) st[q] = a.table[q];
    if (ACT) {
        const int2 bg = a.blk_groups[b];
        if (a.fuse) {
            const float u = period_fraction(n_step, a.cycles);
            for (int q = t; q <= bg.y; q += nt)
                sf[q] = q ? actuation_factor(a.amp[bg.x + q - 1], a.phase[bg.x + q - 1], u) : 1.0f;
        } else {
            for (int q = t; q <= bg.y; q += nt) sf[q] = q ? a.factor[bg.x + q - 1] : 1.0f;
        }
    }
    for (int q = t; q < a.block; q += nt) sx[q] = base + q < a.n ? a.xin[base + q] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int h0 = a.halo_ptr[b], h1 = a.halo_ptr[b + 1];
    for (int h = h0 + t; h < h1; h += nt) sx[a.block + (h - h0)] = a.xin[a.halo_idx[h]];
    __syncthreads();
    const int own = a.lane_mass[base + m];
    const float4 xi = sx[own];
    const int s = (base + m) >> 6;
    float fx, fy, fz;
    const int mode = EXACT ? difference_mode(xi, p.safe) : kPlain;
    if (mode == kPlain)
        gather_lanes<ACT, kPlain, LPM, NARROW>(tbase, sf, xi, s, sub, a.nslice, a.slice_ptr, a.packed, a.narrow,
                                               a.narrow_tb, fx, fy, fz);
    else if (mode == kExactZ)
        gather_lanes<ACT, kExactZ, LPM, NARROW>(tbase, sf, xi, s, sub, a.nslice, a.slice_ptr, a.packed, a.narrow,
                                                a.narrow_tb, fx, fy, fz);
    else
        gather_lanes<ACT, kExactAll, LPM, NARROW>(tbase, sf, xi, s, sub, a.nslice, a.slice_ptr, a.packed, a.narrow,
                                                  a.narrow_tb, fx, fy, fz);
    const int i = base + own;
    if (sub != 0 || i >= a.n) return;
    float vx = a.vin[3 * i + 0], vy = a.vin[3 * i + 1], vz = a.vin[3 * i + 2];
    float4 xo;
    integrate(p, p.dtv, xi, fx, fy, fz, a.fext ? a.fext + 3 * i : nullptr, vx, vy, vz, xo,
              a.vstar_out ? a.vstar_out + 3 * i : nullptr);
    a.xout[i] = xo;
    a.vout[3 * i + 0] = vx;
    a.vout[3 * i + 1] = vy;
    a.vout[3 * i + 2] = vz;
}

// Persistent form: a fixed grid (a multiple of 8 workgroups) walks the blocks; workgroup w runs
// on XCD w % 8 and takes that XCD's contiguous eighth of the blocks in strides.
template <bool ACT, bool EXACT, int BATCH, int MODE, bool STAGE = false>
__global__ void __launch_bounds__(1024) step_persistent(StepArgs a, StepParams p) {
    extern __shared__ float4 sx[];
    const int per = (a.nblk + 7) >> 3;
    const int xcd = (int)(blockIdx.x & 7u);
    const int stride = (int)(gridDim.x >> 3);
    constexpr bool FUSABLE = ACT && MODE != kExplicit;
    const long long n_step = FUSABLE && a.fuse ? *a.step_in : 0;
    if (FUSABLE && a.fuse) advance_step(a, n_step);
    for (int j = (int)(blockIdx.x >> 3); j < per; j += stride) {
        const int b = xcd * per + j;
        if (b >= a.nblk) break;
        step_block<ACT, EXACT, BATCH, MODE, STAGE>(sx, a, p, b, n_step);
        __syncthreads();  // LDS is restaged for the next block
    }
}

// Resident form for a system that fits one workgroup (at most 1024 masses, one block, the
// compact table form): K steps in one launch.  Positions stay in LDS, velocities in
// registers; each step computes its actuation factors in place (the same formula as
// actuation_kernel), gathers, integrates, and after a barrier overwrites the positions.  The
// device step counter advances by K.  The first step kicks for dtv0 (Verlet's dt / 2).
// STAGED: the compact entries are copied into LDS once (r.staged of them, after the factors),
// so no step waits on a memory load.
template <bool ACT, bool EXACT, int BATCH, bool STAGED>
__global__ void __launch_bounds__(1024) step_resident(StepArgs a, StepParams p, ResidentArgs r) {
    extern __shared__ float4 sx[];
    const uint32_t tbase = table_base(a.lds_slots);
    float4* st = reinterpret_cast<float4*>(reinterpret_cast<char*>(sx) + tbase);
    float* sf = reinterpret_cast<float*>(st + a.n_table);
    const int t = (int)threadIdx.x;
    for (int q = t; q < a.n_table; q += a.block) st[q] = a.table[q];
    const uint32_t* pk = a.packed;
    if (STAGED) {
        uint32_t* se = reinterpret_cast<uint32_t*>(sf + a.max_local_groups + 1);
        for (int q = t; q < r.staged; q += a.block) se[q] = a.packed[q];
        pk = se;
    }
    sx[t] = t < a.n ? a.xin[t] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int own = a.lane_mass[t];
    const bool live = own < a.n;
    float vx = 0.f, vy = 0.f, vz = 0.f;
    if (live) {
        vx = a.vin[3 * own + 0];
        vy = a.vin[3 * own + 1];
        vz = a.vin[3 * own + 2];
    }
    const long long n0 = *r.step_in;
    const int2 bg = ACT ? a.blk_groups[0] : make_int2(0, 0);
    const float* fext = a.fext && live ? a.fext + 3 * own : nullptr;
    const int s = t >> 6;
    float4 xo = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k = 0; k < r.steps; ++k) {
        if (ACT) {
            const float u = period_fraction(n0 + k, r.cycles);
            for (int q = t; q <= bg.y; q += a.block)
                sf[q] = q ? actuation_factor(r.amp[bg.x + q - 1], r.phase[bg.x + q - 1], u) : 1.0f;
        }
        __syncthreads();  // positions of step k and its factors are in LDS
        const float4 xi = sx[own];
        float fx, fy, fz;
        const int mode = EXACT ? difference_mode(xi, p.safe) : kPlain;
        if (mode == kPlain) gather_table<ACT, kPlain, BATCH>(tbase, sf, xi, s, a.nslice, a.slice_ptr, pk, fx, fy, fz);
        else if (mode == kExactZ) gather_table<ACT, kExactZ, BATCH>(tbase, sf, xi, s, a.nslice, a.slice_ptr, pk, fx, fy, fz);
        else gather_table<ACT, kExactAll, kExactBatch<BATCH>>(tbase, sf, xi, s, a.nslice, a.slice_ptr, pk, fx, fy, fz);
        integrate(p, k == 0 ? r.dtv0 : p.dtv, xi, fx, fy, fz, fext, vx, vy, vz, xo, nullptr);
        __syncthreads();  // every lane has read step k's positions
        if (live) sx[own] = xo;
    }
    if (live) {
        a.xout[own] = xo;
        a.vout[3 * own + 0] = vx;
        a.vout[3 * own + 1] = vy;
        a.vout[3 * own + 2] = vz;
    }
    if (t == 0) *r.step_out = n0 + r.steps;
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
    const int mode = p.exact ? difference_mode(xi, p.safe) : kPlain;
    const int s = (base + (int)threadIdx.x) >> 6;
    if (mode == kPlain) gather<ACT, kPlain, 4>(sx, xi, s, nslice, slice_ptr, nbr, kl, grp, factor, fx, fy, fz);
    else if (mode == kExactZ) gather<ACT, kExactZ, 4>(sx, xi, s, nslice, slice_ptr, nbr, kl, grp, factor, fx, fy, fz);
    else gather<ACT, kExactAll, 4>(sx, xi, s, nslice, slice_ptr, nbr, kl, grp, factor, fx, fy, fz);
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

// Actuation factors 1 + A_g sin(2 pi f t_n + phi_g) of eq. (2)'s rest lengths at step n, one per
// (body, group), FP32.  The elapsed fraction of a period, frac(n f dt), is formed exactly in
// 64-bit fixed point (n * cycles wraps modulo 2^64), so the phase stays accurate to ~1e-7 rad
// however many steps have been taken.  The step index is n_explicit, or (n_explicit < 0) the
// device counter *step_in; with `advance`, one thread stores n + 1 to *step_out, the other
// slot of the counter pair, which the next launch reads.
__global__ void __launch_bounds__(256)
actuation_kernel(const float* __restrict__ phase, const float* __restrict__ amp, unsigned long long cycles,
                 const long long* step_in, long long* step_out, float* __restrict__ factor, int n_factor, int advance,
                 long long n_explicit) {
    const long long n = n_explicit >= 0 ? n_explicit : *step_in;
    const float u = period_fraction(n, cycles);
    const int g = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g < n_factor) factor[g] = actuation_factor(amp[g], phase[g], u);
    else if (g == n_factor) factor[g] = 1.0f;
    if (advance && blockIdx.x == 0 && threadIdx.x == 0) *step_out = n + 1;
}

// The factors of steps n0, n0 + 1, ..., n0 + gridDim.y - 1 (one per blockIdx.y), row k at
// out + k * stride: the same formula as actuation_kernel, for a recomputed segment at once.
__global__ void __launch_bounds__(256)
actuation_steps_kernel(const float* __restrict__ phase, const float* __restrict__ amp, unsigned long long cycles,
                       long long n0, float* __restrict__ out, int n_factor, long long stride) {
    const int k = (int)blockIdx.y;
    const float u = period_fraction(n0 + k, cycles);
    const int g = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    float* f = out + (size_t)k * (size_t)stride;
    if (g < n_factor) f[g] = actuation_factor(amp[g], phase[g], u);
    else if (g == n_factor) f[g] = 1.0f;
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

// adj_local for mass i, given its x_bar' (bx, by, bz) and v_bar' (vb1).
__device__ __forceinline__ void adj_local_one(int i, const float4* __restrict__ x, const float* __restrict__ vstar,
                                              float bx, float by, float bz, const float* __restrict__ vb1,
                                              float4* __restrict__ w, float* __restrict__ vb0,
                                              float* __restrict__ xbl, const StepParams& p) {
    const float4 xi = x[i];
    const float inv_m = xi.w;
    const float tx = __builtin_fmaf(p.dt, bx, vb1[3 * i + 0]);
    const float ty = __builtin_fmaf(p.dt, by, vb1[3 * i + 1]);
    const float tz = __builtin_fmaf(p.dt, bz, vb1[3 * i + 2]);
    float gx = p.damp * tx, gy = p.damp * ty, gz = p.damp * tz;
    float zb = 0.0f;
    float wz_contact = 0.0f;
    if (inv_m == 0.0f) {
        w[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        vb0[3 * i + 0] = vb0[3 * i + 1] = vb0[3 * i + 2] = 0.0f;
        xbl[3 * i + 0] = bx;
        xbl[3 * i + 1] = by;
        xbl[3 * i + 2] = bz;
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
    xbl[3 * i + 0] = bx;
    xbl[3 * i + 1] = by;
    xbl[3 * i + 2] = bz + wz_contact + zb;
}

__global__ void __launch_bounds__(256)
adj_local_kernel(const float4* __restrict__ x, const float* __restrict__ vstar, const float* __restrict__ xb1,
                 const float* __restrict__ vb1, float4* __restrict__ w, float* __restrict__ vb0,
                 float* __restrict__ xbl, int n, StepParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    adj_local_one(i, x, vstar, xb1[3 * i + 0], xb1[3 * i + 1], xb1[3 * i + 2], vb1, w, vb0, xbl, p);
}

// LPM lanes per mass (1, 2 or 4; the simulation's lanes per mass): with more than one, lane j
// of a mass takes its incidence rows j, j + LPM, ... and the partial sums are combined by the
// same fixed cross-lane pairing as the step's; each incidence's sensitivity is still
// accumulated by exactly one lane.  With nx.x set, the mass's x_bar then feeds adj_local of
// the step before (every input of which is the mass's own), so one launch per reversed step
// remains; nx.w and nx.xbl must not be the w and xbl this launch reads.
template <bool ACT, int LPM>
__global__ void __launch_bounds__(1024)
adj_gather_kernel(const float4* __restrict__ x, const float4* __restrict__ w, const float* __restrict__ xbl,
                  float* __restrict__ xb0, const int32_t* __restrict__ slice_ptr, const uint16_t* __restrict__ nbr,
                  const float2* __restrict__ kl, const uint16_t* __restrict__ grp,
                  const int32_t* __restrict__ halo_ptr, const int32_t* __restrict__ halo_idx,
                  const uint16_t* __restrict__ lane_mass, const float* __restrict__ factor,
                  double2* __restrict__ sens, int n_factor, double cos_t, double sin_t, int n, int nblk, int nslice,
                  int block, int lds_slots, int stage_factors, StepParams p, AdjNext nx) {
    extern __shared__ float4 sx[];
    float4* sw = sx + lds_slots;
    float* sfac = reinterpret_cast<float*>(sw + lds_slots);   // the factor table, when staged
    const int b = logical_block(nblk);
    if (b >= nblk) return;
    const int base = b * block;
    const int t = threadIdx.x, nt = (int)blockDim.x;
    const int m = t / LPM, sub = t % LPM;
    const float* fac = factor;
    if (ACT && stage_factors) {   // small tables: one LDS copy per workgroup, no dependent global load
        for (int q = t; q <= n_factor; q += nt) sfac[q] = factor[q];
        fac = sfac;   // visible after the barrier below
    }
    int own;
    if constexpr (LPM == 1) {
        float4 wt = make_float4(0.f, 0.f, 0.f, 0.f);
        if (base + t < n) wt = w[base + t];
        sw[t] = wt;
        const int h0 = halo_ptr[b], h1 = halo_ptr[b + 1];
        for (int h = h0 + t; h < h1; h += block) sw[block + (h - h0)] = w[halo_idx[h]];
        own = stage_positions(sx, x, halo_ptr, halo_idx, lane_mass, b, base, n, block);
    } else {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int q = t; q < block; q += nt) {
            sx[q] = base + q < n ? x[base + q] : z;
            sw[q] = base + q < n ? w[base + q] : z;
        }
        const int h0 = halo_ptr[b], h1 = halo_ptr[b + 1];
        for (int h = h0 + t; h < h1; h += nt) {
            const int j = halo_idx[h];
            sx[block + (h - h0)] = x[j];
            sw[block + (h - h0)] = w[j];
        }
        __syncthreads();
        own = lane_mass[base + m];
    }
    const float4 xi = sx[own];
    const float4 wi = sw[own];
    float ax = 0.f, ay = 0.f, az = 0.f;
    // one incidence: the spring's tangent stiffness applied to w_j - w_i, and (actuated) the
    // sensitivity of the loss to its rest length, accumulated in FP64
    auto one = [&](int e, int slot, float2 c, int g, float f, double2 acc) {
        const float l0 = ACT ? c.y * f : c.y;
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
                acc.x += cos_t * q;
                acc.y += sin_t * q;
                sens[e] = acc;
            }
        }
    };
    const int s = __builtin_amdgcn_readfirstlane((base + (LPM == 1 ? t : m)) >> 6);
    if (s < nslice) {
        const int lane = (LPM == 1 ? t : m) & 63;
        const int e0 = __builtin_amdgcn_readfirstlane(slice_ptr[s]);
        const int wdt = __builtin_amdgcn_readfirstlane((slice_ptr[s + 1] - e0) >> 6);
        constexpr int B = LPM == 1 ? 8 : 4;   // rows whose loads are in flight together
        // this lane's rows: sub, sub + LPM, ... (all rows when LPM == 1)
        const int rows = (wdt - sub + LPM - 1) / LPM;
        int k = 0;
        for (; k + B <= rows; k += B) {
            int slot[B], g[B];
            float2 c[B];
            float f[B];
            double2 acc[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int e = e0 + ((k + u) * LPM + sub) * 64 + lane;
                slot[u] = nbr[e];
                c[u] = kl[e];
                g[u] = ACT ? (int)grp[e] : n_factor;
                if (ACT) acc[u] = sens[e];
            }
#pragma unroll
            for (int u = 0; u < B; ++u) f[u] = ACT ? fac[g[u]] : 1.0f;
#pragma unroll
            for (int u = 0; u < B; ++u) one(e0 + ((k + u) * LPM + sub) * 64 + lane, slot[u], c[u], g[u], f[u], acc[u]);
        }
        for (; k < rows; ++k) {
            const int e = e0 + (k * LPM + sub) * 64 + lane;
            const int g = ACT ? (int)grp[e] : n_factor;
            one(e, nbr[e], kl[e], g, ACT ? fac[g] : 1.0f, ACT ? sens[e] : make_double2(0.0, 0.0));
        }
    }
#pragma unroll
    for (int o = 1; o < LPM; o <<= 1) {
        ax += __shfl_xor(ax, o, 64);
        ay += __shfl_xor(ay, o, 64);
        az += __shfl_xor(az, o, 64);
    }
    const int i = base + own;
    if (sub != 0 || i >= n) return;
    const float bx = xbl[3 * i + 0] + ax, by = xbl[3 * i + 1] + ay, bz = xbl[3 * i + 2] + az;
    xb0[3 * i + 0] = bx;
    xb0[3 * i + 1] = by;
    xb0[3 * i + 2] = bz;
    if (nx.x) adj_local_one(i, nx.x, nx.vstar, bx, by, bz, nx.vb1, nx.w, nx.vb0, nx.xbl, p);
}

// ---------------------------------------------------------------------------------------
// Structured-box form (the lattice of section "Generating a Lattice" filled out to a full
// box): every node of an nx x ny x nz grid is a mass, every pair of grid neighbours (the 26
// directions) is a spring, the rest length depends only on the kind of direction (edge, face
// diagonal, body diagonal), and the stiffness on the direction and on which faces of the box
// the mass lies on (27 boundary classes; interior masses: on the kind only).  The
// host detects this structure (cronos_create) and then no incidence data is read at all: a
// workgroup owns one aligned 8 x 8 x 8 cube of the Morton order (512 masses, 512 threads),
// stages it with a one-node halo as a 10 x 10 x 10 tile in LDS, and each lane visits its 26
// tile neighbours at fixed offsets.  Directions are summed in a fixed order (dz, dy, dx
// ascending), so the result is bitwise reproducible; it equals the other forms' CSR-order
// sum to rounding.  Halo cells outside the box hold a far-away position whose spring has
// k = 0, contributing exactly nothing.
constexpr int kGridEdge = 8, kGridPitch = 10, kGridCells = 1000, kGridHalo = 488, kGridThreads = 512;

struct GridArgs {
    const float4* __restrict__ xin;
    const float* __restrict__ vin;
    float4* __restrict__ xout;
    float* __restrict__ vout;
    float* __restrict__ vstar_out;
    const float* __restrict__ fext;
    const int32_t* __restrict__ halo;   // [nblk][kGridHalo] new index of each halo cell, -1 outside
    const int4* __restrict__ org;       // [nblk] grid coordinates of the block's first node
    const float* __restrict__ kcls;     // [27][26] k per (boundary class, direction)
    const uint32_t* __restrict__ tab;   // [512] lane's tile cell | lx << 10 | ly << 13 | lz << 16,
                                        // then [488] tile cell of each halo slot
    int nblk, nx, ny, nz;
    // per direction kind (edge, face diagonal, body diagonal: 1, 2 or 3 non-zero offsets)
    float kin[3];                       // k of interior masses (class 13)
    float l0[3];                        // rest length
    double q[3];                        // its square, exact in FP64
};

// Sum of the 26 spring forces of the lane's mass at tile cell `cell`.  INTERIOR: every mass of
// the wavefront is interior, so each direction's k is the same for all lanes.
template <int EX, bool INTERIOR>
__device__ __forceinline__ void gather_grid(const float4* __restrict__ tile, const float* __restrict__ kc, int cell,
                                            float4 xi, const GridArgs& a, float& fx, float& fy, float& fz) {
    fx = fy = fz = 0.0f;
#pragma unroll
    for (int d = 0; d < 26; ++d) {
        const int e = d < 13 ? d : d + 1;                 // skip the centre of the 3 x 3 x 3 stencil
        const int ox = e % 3 - 1, oy = (e / 3) % 3 - 1, oz = e / 9 - 1;
        const int kind = (ox != 0) + (oy != 0) + (oz != 0) - 1;
        const float4 xj = tile[cell + (oz * kGridPitch + oy) * kGridPitch + ox];
        const float k = INTERIOR ? a.kin[kind] : kc[d];
        float dx, dy, dz;
        const float fac = hooke_fac<EX>(xi.x, xi.y, xi.z, xj.x, xj.y, xj.z, k, a.l0[kind], a.q[kind], dx, dy, dz);
        fx = __builtin_fmaf(fac, dx, fx);
        fy = __builtin_fmaf(fac, dy, fy);
        fz = __builtin_fmaf(fac, dz, fz);
    }
}

template <bool EXACT>
__global__ void __launch_bounds__(kGridThreads) step_grid_kernel(GridArgs a, StepParams p) {
    __shared__ float4 tile[kGridCells];
    __shared__ float kcls[27 * 26];
    const int b = logical_block(a.nblk);
    if (b >= a.nblk) return;
    const int t = threadIdx.x;
    const int i = b * kGridThreads + t;
    const uint32_t lane_info = a.tab[t];      // the block's mass t: its tile cell and local x, y, z
    const int cell = (int)(lane_info & 1023u);
    const float4 xi = a.xin[i];
    tile[cell] = xi;
    for (int h = t; h < kGridHalo; h += kGridThreads) {
        const int g = a.halo[(long)b * kGridHalo + h];
        tile[a.tab[kGridThreads + h]] = g >= 0 ? a.xin[g] : make_float4(1e18f, 1e18f, 1e18f, 0.0f);
    }
    // a block that touches no face of the box holds only interior masses (class 13): it needs
    // neither the class of each mass nor the per-class k table
    const int4 o = a.org[b];
    const bool face = o.x == 0 || o.y == 0 || o.z == 0 || o.x + kGridEdge >= a.nx || o.y + kGridEdge >= a.ny ||
                      o.z + kGridEdge >= a.nz;
    int cls = 13;
    if (face) {
        for (int q = t; q < 27 * 26; q += kGridThreads) kcls[q] = a.kcls[q];
        const int gx = o.x + (int)((lane_info >> 10) & 7u), gy = o.y + (int)((lane_info >> 13) & 7u),
                  gz = o.z + (int)((lane_info >> 16) & 7u);
        cls = (gx == 0 ? 0 : gx == a.nx - 1 ? 2 : 1) + 3 * (gy == 0 ? 0 : gy == a.ny - 1 ? 2 : 1) +
              9 * (gz == 0 ? 0 : gz == a.nz - 1 ? 2 : 1);
    }
    __syncthreads();
    const float* kc = kcls + 26 * cls;
    const bool interior = __builtin_amdgcn_ballot_w64(cls != 13) == 0;
    const int mode = EXACT ? difference_mode(xi, p.safe) : kPlain;
    float fx, fy, fz;
    if (mode == kPlain) {
        if (interior) gather_grid<kPlain, true>(tile, kc, cell, xi, a, fx, fy, fz);
        else gather_grid<kPlain, false>(tile, kc, cell, xi, a, fx, fy, fz);
    } else if (mode == kExactZ) {
        if (interior) gather_grid<kExactZ, true>(tile, kc, cell, xi, a, fx, fy, fz);
        else gather_grid<kExactZ, false>(tile, kc, cell, xi, a, fx, fy, fz);
    } else {
        if (interior) gather_grid<kExactAll, true>(tile, kc, cell, xi, a, fx, fy, fz);
        else gather_grid<kExactAll, false>(tile, kc, cell, xi, a, fx, fy, fz);
    }
    float vx = a.vin[3 * i + 0], vy = a.vin[3 * i + 1], vz = a.vin[3 * i + 2];
    float4 xo;
    integrate(p, p.dtv, xi, fx, fy, fz, a.fext ? a.fext + 3 * i : nullptr, vx, vy, vz, xo,
              a.vstar_out ? a.vstar_out + 3 * i : nullptr);
    a.xout[i] = xo;
    a.vout[3 * i + 0] = vx;
    a.vout[3 * i + 1] = vy;
    a.vout[3 * i + 2] = vz;
}

inline int grid_for(int64_t nblk) { return (int)(((nblk + 7) / 8) * 8); }

constexpr int kAdjStagedFactors = 4096;

}  // namespace

hipError_t launch_step(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st) {
    return launch_step_io(d, d.x[cur], d.v[cur], d.x[cur ^ 1], d.v[cur ^ 1], nullptr, p, st, nullptr,
                          fused_actuation(d) ? 1 : 0, cur);
}

// Dynamic LDS of one step workgroup: positions, then (table and split modes) the parameter
// table and the workgroup's actuation factors, then (split mode) the spring factors.
hipError_t step_static_lds(size_t* bytes) {
    const void* ks[] = {(const void*)step_kernel<false, true, 4, kTable>, (const void*)step_kernel<true, true, 4, kTable>,
                        (const void*)step_persistent<false, true, 4, kTable>, (const void*)step_kernel<true, true, 4, kSplit>,
                        (const void*)step_persistent<true, false, 8, kSplit>,
                        (const void*)step_kernel<false, true, 4, kNarrow>,
                        (const void*)step_lanes_kernel<true, true, 4, false>,
                        (const void*)step_lanes_kernel<false, true, 2, true>,
                        (const void*)step_resident<false, true, 4, true>, (const void*)step_resident<true, true, 4, false>};
    *bytes = 0;
    for (const void* k : ks) {
        hipFuncAttributes at{};
        hipError_t e = hipFuncGetAttributes(&at, k);
        if (e != hipSuccess) return e;
        *bytes = std::max(*bytes, (size_t)at.sharedSizeBytes);
    }
    return hipSuccess;
}

size_t step_lds_bytes(const DeviceArrays& d) {
    size_t b = (size_t)d.lds_slots * sizeof(float4);
    if (d.packed || d.narrow)
        b = table_base(d.lds_slots) + (size_t)d.n_table * sizeof(float4) + (size_t)(d.max_local_groups + 1) * sizeof(float);
    if (d.sp_rec) b += (size_t)(d.max_sp + 1) * sizeof(float);
    return b;
}

// Dynamic LDS of a one-lane step launch: the staging above, and with stage_io room for the old
// velocities and the new state of the block's masses (a float4 and six floats each) that
// step_block passes through LDS in mass order.  (The several-lanes kernel keeps direct
// accesses: on the small systems it serves, the extra barriers cost more than the scattered
// lines.)
size_t step_launch_lds_bytes(const DeviceArrays& d) {
    if (!d.stage_io) return step_lds_bytes(d);
    return std::max(step_lds_bytes(d), (size_t)d.block * (sizeof(float4) + 6 * sizeof(float)));
}

bool fused_actuation(const DeviceArrays& d) { return d.grp != nullptr && (d.sp_rec || d.narrow || d.packed); }

hipError_t launch_step_io(const DeviceArrays& d, const float4* xin, const float* vin, float4* xout, float* vout,
                          float* vstar, const StepParams& p, hipStream_t st, const float* factor, int fuse,
                          int cur) {
    if (d.grid) {
        if (fuse) return hipErrorInvalidValue;
        GridArgs g{xin, vin, xout, vout, vstar, d.fext, d.grid_halo, d.grid_org, d.grid_k, d.grid_tab, (int)d.nblk,
                   d.grid_dim[0], d.grid_dim[1], d.grid_dim[2], {}, {}, {}};
        for (int q = 0; q < 3; ++q) {
            g.kin[q] = d.grid_kin[q];
            g.l0[q] = d.grid_l0[q];
            g.q[q] = (double)d.grid_l0[q] * (double)d.grid_l0[q];
        }
        const dim3 grid((unsigned)grid_for(d.nblk)), th(kGridThreads);
        if (p.exact) hipLaunchKernelGGL(step_grid_kernel<true>, grid, th, 0, st, g, p);
        else hipLaunchKernelGGL(step_grid_kernel<false>, grid, th, 0, st, g, p);
        return hipGetLastError();
    }
    const int mode = d.sp_rec ? kSplit : d.narrow ? kNarrow : d.packed ? kTable : kExplicit;
    if (fuse && !fused_actuation(d)) return hipErrorInvalidValue;
    StepArgs a{xin, vin, xout, vout, d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx,
               d.lane_mass, factor ? factor : d.factor, d.fext, vstar, d.packed, d.narrow, d.table, d.blk_groups, d.sp_rec, d.sp_grp,
               d.sp_ptr, (int)d.n, (int)d.nblk, (int)d.nslice, d.block, d.n_table, d.lds_slots, d.max_local_groups,
               d.narrow_tb, fuse, d.phase, d.amp, d.step_ctr + (cur & 1), d.step_ctr + ((cur & 1) ^ 1), p.cycles};
    const size_t lds = step_lds_bytes(d);
    if (d.lanes > 1 && (mode == kTable || mode == kNarrow)) {
        const bool act = d.grp != nullptr, ex = p.exact != 0, nar = mode == kNarrow && !act;
        const dim3 g((unsigned)grid_for(d.nblk)), th((unsigned)(d.block * d.lanes));
        auto go = [&](auto k) { hipLaunchKernelGGL(k, g, th, lds, st, a, p); };
        if (d.lanes == 2) {
            if (act) ex ? go(step_lanes_kernel<true, true, 2, false>) : go(step_lanes_kernel<true, false, 2, false>);
            else if (nar) ex ? go(step_lanes_kernel<false, true, 2, true>) : go(step_lanes_kernel<false, false, 2, true>);
            else ex ? go(step_lanes_kernel<false, true, 2, false>) : go(step_lanes_kernel<false, false, 2, false>);
        } else {
            if (act) ex ? go(step_lanes_kernel<true, true, 4, false>) : go(step_lanes_kernel<true, false, 4, false>);
            else if (nar) ex ? go(step_lanes_kernel<false, true, 4, true>) : go(step_lanes_kernel<false, false, 4, true>);
            else ex ? go(step_lanes_kernel<false, true, 4, false>) : go(step_lanes_kernel<false, false, 4, false>);
        }
        return hipGetLastError();
    }
    const bool persistent = d.persistent_groups > 0;
    const dim3 grid(persistent ? (unsigned)d.persistent_groups : (unsigned)grid_for(d.nblk));
    const size_t lds1 = step_launch_lds_bytes(d);
    auto go = [&](auto normal, auto pers) {
        if (persistent) hipLaunchKernelGGL(pers, grid, dim3(d.block), lds1, st, a, p);
        else hipLaunchKernelGGL(normal, grid, dim3(d.block), lds1, st, a, p);
    };
#define CRONOS_GO(A, E, B, M) go(step_kernel<A, E, B, M>, step_persistent<A, E, B, M>)
// (16-bit entries exist for passive simulations only: the actuated expansion maps them to kTable,
// which it never meets there)
#define CRONOS_GO_M(A, E, B)                                                                         \
    (mode == kSplit    ? CRONOS_GO(A, E, B, kSplit)                                                  \
     : mode == kNarrow ? CRONOS_GO(A, E, B, (A ? kTable : kNarrow))                                  \
     : mode == kTable  ? CRONOS_GO(A, E, B, kTable)                                                  \
                       : CRONOS_GO(A, E, B, kExplicit))
    const bool act = d.grp != nullptr, ex = p.exact != 0;
    if (d.stage_io && act && mode == kTable) {
#define CRONOS_GO_S(E, B) go(step_kernel<true, E, B, kTable, true>, step_persistent<true, E, B, kTable, true>)
        if (d.batch == 8) ex ? CRONOS_GO_S(true, 8) : CRONOS_GO_S(false, 8);
        else if (d.batch == 2) ex ? CRONOS_GO_S(true, 2) : CRONOS_GO_S(false, 2);
        else ex ? CRONOS_GO_S(true, 4) : CRONOS_GO_S(false, 4);
#undef CRONOS_GO_S
    } else if (d.batch == 8) {
        if (act) ex ? CRONOS_GO_M(true, true, 8) : CRONOS_GO_M(true, false, 8);
        else ex ? CRONOS_GO_M(false, true, 8) : CRONOS_GO_M(false, false, 8);
    } else if (d.batch == 2) {
        if (act) ex ? CRONOS_GO_M(true, true, 2) : CRONOS_GO_M(true, false, 2);
        else ex ? CRONOS_GO_M(false, true, 2) : CRONOS_GO_M(false, false, 2);
    } else {
        if (act) ex ? CRONOS_GO_M(true, true, 4) : CRONOS_GO_M(true, false, 4);
        else ex ? CRONOS_GO_M(false, true, 4) : CRONOS_GO_M(false, false, 4);
    }
#undef CRONOS_GO_M
#undef CRONOS_GO
    return hipGetLastError();
}

hipError_t launch_resident(const DeviceArrays& d, int cur, const StepParams& p, float dtv0, unsigned long long cycles,
                           int steps, hipStream_t st) {
    StepArgs a{d.x[cur], d.v[cur], d.x[cur ^ 1], d.v[cur ^ 1], d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx,
               d.lane_mass, d.factor, d.fext, nullptr, d.packed, d.narrow, d.table, d.blk_groups, d.sp_rec, d.sp_grp,
               d.sp_ptr, (int)d.n, (int)d.nblk, (int)d.nslice, d.block, d.n_table, d.lds_slots, d.max_local_groups,
               d.narrow_tb, 0, d.phase, d.amp, d.step_ctr + (cur & 1), d.step_ctr + ((cur & 1) ^ 1), cycles};
    ResidentArgs r{d.phase, d.amp, cycles, d.step_ctr + (cur & 1), d.step_ctr + ((cur & 1) ^ 1), steps, dtv0,
                   d.resident_staged};
    const size_t lds = step_lds_bytes(d) + (size_t)d.resident_staged * sizeof(uint32_t);
    const bool act = d.grp != nullptr, ex = p.exact != 0;
    auto go = [&](auto k) { hipLaunchKernelGGL(k, dim3(1), dim3(d.block), lds, st, a, p, r); };
    if (d.resident_staged) {
        if (act) ex ? go(step_resident<true, true, 4, true>) : go(step_resident<true, false, 4, true>);
        else ex ? go(step_resident<false, true, 4, true>) : go(step_resident<false, false, 4, true>);
    } else {
        if (act) ex ? go(step_resident<true, true, 4, false>) : go(step_resident<true, false, 4, false>);
        else ex ? go(step_resident<false, true, 4, false>) : go(step_resident<false, false, 4, false>);
    }
    return hipGetLastError();
}

hipError_t persistent_grid(const DeviceArrays& d, int exact, int* grid) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const void* k;
    if (d.sp_rec)
        k = d.grp ? (exact ? (const void*)step_persistent<true, true, 4, kSplit> : (const void*)step_persistent<true, false, 4, kSplit>)
                  : (exact ? (const void*)step_persistent<false, true, 4, kSplit> : (const void*)step_persistent<false, false, 4, kSplit>);
    else
        k = d.grp ? (exact ? (const void*)step_persistent<true, true, 4, kTable> : (const void*)step_persistent<true, false, 4, kTable>)
                  : (exact ? (const void*)step_persistent<false, true, 4, kTable> : (const void*)step_persistent<false, false, 4, kTable>);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, d.block, step_launch_lds_bytes(d));
    if (e != hipSuccess) return e;
    int g = std::max(1, per_cu) * cus;
    g = (g + 7) / 8 * 8;
    *grid = (int)std::min<int64_t>(g, grid_for(d.nblk));
    return hipSuccess;
}

hipError_t launch_actuation(const DeviceArrays& d, unsigned long long cycles, int advance, hipStream_t st,
                            long long n_explicit, float* out, int cur) {
    const unsigned grid = (unsigned)((d.n_factor + 1 + 255) / 256);
    hipLaunchKernelGGL(actuation_kernel, dim3(grid), dim3(256), 0, st, d.phase, d.amp, cycles, d.step_ctr + (cur & 1),
                       d.step_ctr + ((cur & 1) ^ 1), out ? out : d.factor, d.n_factor, n_explicit >= 0 ? 0 : advance,
                       n_explicit);
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

hipError_t launch_actuation_steps(const DeviceArrays& d, unsigned long long cycles, long long n0, int steps,
                                  float* out, long long stride, hipStream_t st) {
    const unsigned grid = (unsigned)((d.n_factor + 1 + 255) / 256);
    for (int k0 = 0; k0 < steps; k0 += 65535) {   // at most 65535 rows per launch (grid y)
        const int rows = std::min(steps - k0, 65535);
        hipLaunchKernelGGL(actuation_steps_kernel, dim3(grid, (unsigned)rows), dim3(256), 0, st, d.phase, d.amp, cycles,
                           n0 + k0, out + (size_t)k0 * (size_t)stride, d.n_factor, stride);
    }
    return hipGetLastError();
}

hipError_t launch_adj_gather(const DeviceArrays& d, const float4* x, const float4* w, const float* xbl, float* xb0,
                             double2* sens, double cos_t, double sin_t, hipStream_t st, const float* factor,
                             const StepParams& p, const AdjNext& next) {
    if (!factor) factor = d.factor;
    // the factor table goes to LDS when small (kAdjStagedFactors entries at most)
    const int stage = d.grp && d.n_factor + 1 <= kAdjStagedFactors ? 1 : 0;
    const size_t lds = 2 * (size_t)d.lds_slots * sizeof(float4) + (stage ? (size_t)(d.n_factor + 1) * sizeof(float) : 0);
    const int lanes = d.lanes == 2 || d.lanes == 4 ? d.lanes : 1;
    const dim3 g(grid_for(d.nblk)), th((unsigned)(d.block * lanes));
    auto go = [&](auto k) {
        hipLaunchKernelGGL(k, g, th, lds, st, x, w, xbl, xb0, d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr, d.halo_idx,
                           d.lane_mass, factor, sens, d.n_factor, cos_t, sin_t, (int)d.n, (int)d.nblk, (int)d.nslice,
                           d.block, d.lds_slots, stage, p, next);
    };
    if (d.grp) {
        if (lanes == 4) go(adj_gather_kernel<true, 4>);
        else if (lanes == 2) go(adj_gather_kernel<true, 2>);
        else go(adj_gather_kernel<true, 1>);
    } else {
        if (lanes == 4) go(adj_gather_kernel<false, 4>);
        else if (lanes == 2) go(adj_gather_kernel<false, 2>);
        else go(adj_gather_kernel<false, 1>);
    }
    return hipGetLastError();
}

namespace {

// One workgroup per actuation group: its entries' sums, each thread over a strided part of
// the group's entry list in order, then the fixed-order workgroup tree.
__global__ void __launch_bounds__(256) adj_group_sums_kernel(const double2* __restrict__ sens,
                                                             const int32_t* __restrict__ grp_ptr,
                                                             const int32_t* __restrict__ grp_entries,
                                                             double2* __restrict__ gsum) {
    __shared__ double2 red[256];
    const int g = blockIdx.x, t = threadIdx.x;
    double2 s = make_double2(0.0, 0.0);
    for (int q = grp_ptr[g] + t; q < grp_ptr[g + 1]; q += 256) {
        const double2 v = sens[grp_entries[q]];
        s.x += v.x;
        s.y += v.y;
    }
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            red[t].x += red[t + h].x;
            red[t].y += red[t + h].y;
        }
        __syncthreads();
    }
    if (t == 0) gsum[g] = red[0];
}

}  // namespace

hipError_t launch_adj_group_sums(const double2* sens, const int32_t* grp_ptr, const int32_t* grp_entries, int n_groups,
                                 double2* gsum, hipStream_t st) {
    if (n_groups < 1) return hipSuccess;
    hipLaunchKernelGGL(adj_group_sums_kernel, dim3(n_groups), dim3(256), 0, st, sens, grp_ptr, grp_entries, gsum);
    return hipGetLastError();
}

}  // namespace cronos
