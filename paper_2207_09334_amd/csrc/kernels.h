// Launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cronos {

struct StepParams {
    float dt;            // position update x' = x + dt v'
    float dtv;           // velocity kick v* = v + dtv f / m (dt; dt / 2 in Verlet's first step)
    float damp;          // 1 - d
    float gx, gy, gz;
    float ground_z, ground_k, ground_mu;
    int ground;          // contact plane on
    int exact;           // exact coordinate differences (see hooke in kernels.hip)
    float safe;          // a wavefront whose masses all have |x_c| >= safe on every axis takes
                         // the plain difference (Sterbenz-exact for springs shorter than safe/2)
    double ox, oy, oz;   // origin of the device coordinates: absolute x = device x + o
    unsigned long long cycles = 0;   // actuation: frac(f dt) * 2^64, the period fraction per step
};

// Device-resident layout and state of one simulation (all arrays in Morton order).
struct DeviceArrays {
    int64_t n = 0;          // masses
    int32_t block = 256;    // masses (= threads) per workgroup
    int64_t nblk = 0;
    int64_t nslice = 0;     // nblk * block / 64
    int32_t lds_slots = 0;  // block + largest halo
    int32_t batch = 4;      // incidence entries fetched per batch (2, 4 or 8)
    int32_t persistent_groups = 0;  // > 0: persistent grid of that many workgroups
    int32_t lanes = 1;              // lanes per mass (1, 2 or 4; more than 1 in the table forms only)
    int32_t stage_io = 0;           // one-lane forms: velocities in and new state out through LDS in mass order
    float4* x[2] = {nullptr, nullptr};   // (x, y, z, 1/m); 1/m = 0 marks a fixed mass
    float* v[2] = {nullptr, nullptr};    // [n][3]
    float* mass = nullptr;               // [n]
    float* fext = nullptr;               // [n][3] or null
    uint16_t* lane_mass = nullptr;       // [nblk*block] mass owned by each lane, block-relative
    int32_t* slice_ptr = nullptr;
    uint16_t* nbr = nullptr;
    float2* kl = nullptr;                // (k, L0) per entry
    uint32_t* packed = nullptr;          // compact 32-bit entries (or null)
    uint16_t* narrow = nullptr;          // compact 16-bit entries: slot << narrow_tb | pair index (or null)
    int32_t narrow_tb = 0;
    float4* table = nullptr;             // distinct (k, L0) pairs of the compact entries, as
                                         // (k, L0, L0^2 as an FP64 value in the last two words)
    int32_t n_table = 0;
    int2* blk_groups = nullptr;          // per workgroup (first factor index, count) of its actuated springs
    int32_t max_local_groups = 0;
    uint32_t* sp_rec = nullptr;          // split form (see the step kernel): spring records,
    uint16_t* sp_grp = nullptr;          //   their local actuation factor indices,
    int32_t* sp_ptr = nullptr;           //   per-workgroup record ranges
    int32_t max_sp = 0;                  //   and the largest record count of a workgroup
    int32_t resident = 0;                // one workgroup holds the system (see launch_resident)
    int32_t resident_staged = 0;         // entries the resident form copies into LDS (0: read from memory)
    uint16_t* grp = nullptr;             // per entry index into factor[], or null
    int32_t* halo_ptr = nullptr;
    int32_t* halo_idx = nullptr;
    // actuation
    int32_t n_factor = 0;                // bodies * groups (factor[n_factor] = 1 for passive)
    float* phase = nullptr;
    float* amp = nullptr;
    float* factor = nullptr;             // 1 + A sin(...) per (body, group), FP32
    long long* step_ctr = nullptr;       // [2] device step counter pair: slot cur holds the step
                                         // index of x[cur]; a launch reads slot cur, writes cur ^ 1
    // diagnostics
    int32_t n_chunks = 0;
    int32_t nb = 1;
    int4* chunks = nullptr;              // (block, first mass, end mass, body)
    int32_t* body_chunk = nullptr;       // [nb+1] chunk offsets of each body
    double* chunk_part = nullptr;        // [n_chunks][kDiagFields]
    double* body_out = nullptr;          // [nb][kDiagFields]
    float* fout = nullptr;               // [n][3] force output
    // structured-box form (see step_grid_kernel): blocks are aligned 8 x 8 x 8 cubes of a full box
    int32_t grid = 0;
    int32_t grid_dim[3] = {0, 0, 0};
    int32_t* grid_halo = nullptr;        // [nblk][488] new index of each halo cell of the block's tile, -1 outside
    int4* grid_org = nullptr;            // [nblk] grid coordinates of the block's first node
    float* grid_k = nullptr;             // [27][26] k per (boundary class, direction)
    uint32_t* grid_tab = nullptr;        // [512] lane's tile cell | lx << 10 | ly << 13 | lz << 16, then
                                         // [488] tile cell of each halo slot
    float grid_kin[3] = {};              // interior k per direction kind (1, 2, 3 non-zero offsets)
    float grid_l0[3] = {};               // rest length per direction kind
};

constexpr int kDiagFields = 20;  // ke, pe_s, pe_g, pe_c, p3, mx3, mass, min3, max3, nonfinite

// Byte address of the parameter table in a step workgroup's LDS: after the positions, rounded
// up to a multiple of 8192 so that OR-ing an in-table offset (< 8192) adds it.
__host__ __device__ inline uint32_t table_base(int lds_slots) { return ((uint32_t)lds_slots * 16u + 8191u) & ~8191u; }
// Static LDS of the step kernels (must be 0: entry words carry absolute LDS byte addresses).
hipError_t step_static_lds(size_t* bytes);

hipError_t launch_step(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st);
// The step with explicit buffers; vstar (optional) receives the velocity before friction/damping.
// factor (optional) replaces the simulation's actuation factor table.  fuse != 0 (actuated
// table forms only, see fused_actuation): the step computes its factors for the step index in
// counter slot cur itself and stores the next index in slot cur ^ 1, as launch_actuation with
// advance would.
hipError_t launch_step_io(const DeviceArrays& d, const float4* xin, const float* vin, float4* xout, float* vout,
                          float* vstar, const StepParams& p, hipStream_t st, const float* factor = nullptr,
                          int fuse = 0, int cur = 0);
// Whether launch_step computes the actuation factors inside the step (actuated systems in a
// compact table form); otherwise an actuation launch must precede each step.
bool fused_actuation(const DeviceArrays& d);
// Dynamic LDS bytes of one step workgroup (positions, table, factors; the resident form adds its
// staged entries).
size_t step_lds_bytes(const DeviceArrays& d);
// `steps` steps of a system held by one workgroup (resident form; table form, block >= n):
// positions stay in LDS between steps; the first step kicks for dtv0.  Reads x[cur], v[cur],
// writes x[cur ^ 1], v[cur ^ 1]; advances the device step counter by `steps`.
hipError_t launch_resident(const DeviceArrays& d, int cur, const StepParams& p, float dtv0, unsigned long long cycles,
                           int steps, hipStream_t st);
// Workgroups of a persistent launch that are resident at once on the device (multiple of 8).
hipError_t persistent_grid(const DeviceArrays& d, int exact, int* grid);
// Actuation table for the step index in counter slot cur (storing the next index in slot
// cur ^ 1 when advance != 0), or for the explicit step n_explicit >= 0 (counters untouched).
// cycles = frac(f dt) * 2^64, the part of an actuation period that one step advances, in
// 64-bit fixed point.  out (optional) receives the factors instead of the simulation's table.
hipError_t launch_actuation(const DeviceArrays& d, unsigned long long cycles, int advance, hipStream_t st,
                            long long n_explicit = -1, float* out = nullptr, int cur = 0);
// Adjoint of one step (see kernels.hip).
hipError_t launch_adj_local(const DeviceArrays& d, const float4* x, const float* vstar, const float* xb1,
                            const float* vb1, float4* w, float* vb0, float* xbl, const StepParams& p, hipStream_t st);
// adj_local of the previous step fused into the gather's end (x == nullptr: none); the
// buffers w and xbl are the previous step's, distinct from the ones the gather reads.
struct AdjNext {
    const float4* x = nullptr;      // positions at the previous step's start
    const float* vstar = nullptr;   // its v* (before friction)
    const float* vb1 = nullptr;     // v_bar after the previous step (written by this step's adj_local)
    float4* w = nullptr;
    float* vb0 = nullptr;
    float* xbl = nullptr;
};
hipError_t launch_adj_gather(const DeviceArrays& d, const float4* x, const float4* w, const float* xbl, float* xb0,
                             double2* sens, double cos_t, double sin_t, hipStream_t st, const float* factor,
                             const StepParams& p, const AdjNext& next);
// Per actuation group g: gsum[g] = the sum of the per-entry sensitivities sens[e] over the
// group's entries grp_entries[grp_ptr[g] .. grp_ptr[g + 1]) (one workgroup per group, a
// fixed summation order).
hipError_t launch_adj_group_sums(const double2* sens, const int32_t* grp_ptr, const int32_t* grp_entries, int n_groups,
                                 double2* gsum, hipStream_t st);
// Actuation factors of steps n0 .. n0 + steps - 1 in one launch, row k at out + k * stride.
hipError_t launch_actuation_steps(const DeviceArrays& d, unsigned long long cycles, long long n0, int steps,
                                  float* out, long long stride, hipStream_t st);
hipError_t launch_forces(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st);

// Lanczos iterations for the natural frequencies (modes.hip), FP64.
struct ModesBuffers {
    double* ism = nullptr;               // [n] M^-1/2 (0 for fixed masses)
    double* q[2] = {nullptr, nullptr};   // [3n] Lanczos vectors, alternating roles
    double* y = nullptr;                 // [3n] A q
    double* part_a = nullptr;            // [nblk] partial q . A q
    double* part_u = nullptr;            // [ceil(n / 256)] partial squared norms
    double* alpha = nullptr;             // [max_iter] diagonal of the tridiagonal matrix
    double* beta = nullptr;              // [max_iter] off-diagonal (beta[k] follows step k)
};
// Random start vector q_0 (normalised, in q[1]; q[0] cleared to zeros) and M^-1/2.
hipError_t launch_modes_init(const DeviceArrays& d, int cur, ModesBuffers& m, unsigned long long seed, hipStream_t st);
// Lanczos step k: alpha[k], beta[k] and q_{k+1} from q_k and q_{k-1}.
hipError_t launch_modes_iteration(const DeviceArrays& d, int cur, const StepParams& p, ModesBuffers& m, int k,
                                  hipStream_t st);
// Fixed FP64 workspace of the allocation-free frequency entry point: a file-scope device
// array of this many doubles (64 MiB) on every GPU the library runs on, held until the process
// ends.  modes_scratch returns its address on `device` (which must be current), looked up
// once per device.
constexpr size_t kModesScratchDoubles = size_t(8) << 20;
hipError_t modes_scratch(int device, double** ptr);
hipError_t launch_diagnostics(const DeviceArrays& d, int cur, const StepParams& p, hipStream_t st);

}  // namespace cronos
