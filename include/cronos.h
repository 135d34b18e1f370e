/*
 * cronos.h -- C ABI of the MI355X (gfx950) mass-spring simulator.
 *
 * The method is the Hookean mass-spring model of Clay et al., "A Massively-Parallel 3D
 * Simulator for Soft and Hybrid Robots": masses x_i, v_i, m_i joined by springs
 * (i, j, k_ij, l0_ij); each step sums per mass the gravity, external and Hooke forces of
 * eq. (2) and integrates eqs. (3)-(4).  This library adds a contact plane with Coulomb
 * friction and fixed masses (section "Generating a Lattice": constraints and planes;
 * Appendix A: frictional contact planes), velocity damping (Euler-Bernoulli section) and
 * actuated rest lengths (section "Method": springs individually rigid, actuated or
 * functionally parameterised).
 *
 * Conventions for every call:
 *  - All pointers are HOST pointers unless stated otherwise.  Input arrays are owned by the
 *    caller and only read during the call (their contents are copied); output arrays are
 *    caller-allocated and written in full.  No pointer is retained after a call returns.
 *  - Arrays of 3-vectors are row-major [n][3] (x, y, z interleaved).
 *  - Every host-facing array is in INPUT order: the library's internal space-filling-curve
 *    renumbering never leaks out, except through cronos_layout_get which reports it.
 *  - Errors: a negative cronos_status; no exception crosses the ABI; the detail text of the
 *    last error on the calling thread is returned by cronos_last_error().
 *  - Threading: a handle must not be used by two threads at once.  All device work of a
 *    simulation is enqueued on the stream bound at creation, in call order.
 *  - Units: SI (m, kg, s, N, N/m).  z is up; the contact plane is z = ground_z.
 */
#ifndef CRONOS_H
#define CRONOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CRONOS_OK = 0,
    CRONOS_EINVAL = -1,     /* an argument or input array is invalid                        */
    CRONOS_ENOMEM = -2,     /* host or device allocation failed                              */
    CRONOS_EDEVICE = -3,    /* a HIP runtime call or kernel launch failed                    */
    CRONOS_EUNSTABLE = -4,  /* dt exceeds the explicit integrator's stability limit          */
    CRONOS_ESTATE = -5      /* the simulated state holds NaN or Inf                          */
} cronos_status;

/* flags of cronos_desc.flags */
#define CRONOS_ALLOW_UNSTABLE 0x1u   /* skip the stability check at creation                 */
#define CRONOS_CHECK_LAYOUT   0x2u   /* verify the device layout against the CSR at creation  */
#define CRONOS_NO_GRAPH       0x4u   /* enqueue steps as plain launches, not HIP graphs      */
#define CRONOS_GRAPH          0x800u /* enqueue steps as HIP graphs whatever the step time (by
                                        default a step that takes 12 us or more with plain
                                        launches keeps them; see cronos_launch_mode); not with
                                        CRONOS_NO_GRAPH                                      */
#define CRONOS_NO_TABLE       0x10u  /* keep explicit per-entry (k, L0) in the step instead of a
                                        16-bit index into the table of distinct pairs        */
#define CRONOS_NO_SHIFT       0x20u  /* keep the caller's coordinate frame on the device (by
                                        default it is shifted away from the coordinate planes
                                        so plain differences are exact; z is never shifted
                                        when the contact plane is on)                        */
#define CRONOS_SPLIT          0x40u  /* split step form: a spring pass evaluates each spring once
                                        per workgroup into LDS, then a gather pass sums them
                                        (default: every spring evaluated from both ends)    */
#define CRONOS_VERLET         0x80u  /* integrate with Verlet, eqs. (5)-(6), instead of symplectic
                                        Euler: run in velocity form, the first step after create
                                        or set_state kicks for dt / 2 (eq. (5)) and the velocity
                                        held is (x_{n+1} - x_n) / dt; contact friction and
                                        damping act on it as in the Euler step.  Not with
                                        cronos_rollout (its adjoint is of the Euler step)    */
#define CRONOS_RESIDENT       0x100u /* a system of at most 1024 masses runs in one workgroup that
                                        keeps it in LDS and takes up to 4096 steps per launch
                                        (compact table form needed; ignored otherwise, see
                                        cronos_launch_config)                                 */
#define CRONOS_WIDE_ENTRIES   0x200u /* keep 32-bit compact entries where 16-bit ones would fit
                                        (passive systems whose workgroup LDS slots and (k, L0)
                                        pairs fit in 16 bits; see CRONOS_FORM_NARROW)        */
#define CRONOS_DIRECT_IO      0x1000u /* actuated systems in the 32-bit table form with one lane per
                                        mass: read velocities and write the new state where each
                                        lane's mass lies (the default below 256 MiB of
                                        compulsory bytes per step, see cronos_launch_mode)    */
#define CRONOS_STAGED_IO      0x2000u /* the same systems: velocities in and the new state out
                                        through LDS in mass order; not with CRONOS_DIRECT_IO;
                                        no effect on the other forms                          */
#define CRONOS_NO_GRID        0x400u /* never take the structured-box step form (CRONOS_FORM_GRID);
                                        the other forms are chosen as without the flag        */
#define CRONOS_FAST_DIFF      0x8u   /* skip the residual of x_j - x_i in the elongation: faster,
                                        but a nearly relaxed spring within one spring length of
                                        a coordinate plane loses accuracy                     */

/* mass_mode / k_mode of cronos_lattice_desc */
#define CRONOS_MASS_UNIFORM  0       /* every node gets mass_value                           */
#define CRONOS_MASS_LUMPED   1       /* every voxel adds density*a^3/8 to each of its corners */
#define CRONOS_K_UNIFORM     0       /* every spring gets k_uniform                          */
#define CRONOS_K_ASSEMBLY    1       /* per-voxel stiffness: k_v/4 per edge, k_v/2 per face
                                        diagonal, k_v per long diagonal, summed over voxels   */

const char* cronos_last_error(void);
const char* cronos_version(void);

/* ------------------------------------------------------------------------------------------
 * Lattice generation (section "Generating a Lattice", voxel-grid variant and its figure):
 * nodes are the corners of the occupied voxels; each voxel links its corners along the 12
 * cube edges, the 12 face diagonals and the 4 long diagonals, duplicates merged; rest
 * lengths are nominal (a, a*sqrt2, a*sqrt3); masses and spring constants follow the chosen
 * modes.  Canonical node order is by (z, y, x) of the integer corner coordinate, per body;
 * springs are (i, j), i < j, sorted; an actuated spring takes the group of the
 * lowest-(z,y,x) actuated voxel containing it.  Host-only: no device is touched.
 * ---------------------------------------------------------------------------------------- */
typedef struct cronos_lattice_t* cronos_lattice;

typedef struct {
    int32_t n_bodies;                 /* >= 1                                                 */
    const int64_t* body_voxel_offset; /* [n_bodies+1]; voxels of body b are
                                         [off[b], off[b+1]); NULL allowed when n_bodies == 1  */
    int64_t n_voxels;
    const int32_t* voxels;            /* [n_voxels][3] integer voxel coordinates, |c| < 2^20,
                                         no duplicates within a body                          */
    const int32_t* material;          /* [n_voxels] index into material_k, or NULL (all 0)    */
    const int32_t* group;             /* [n_voxels] actuation group >= 0, or -1 passive;
                                         NULL = all passive                                    */
    double spacing;                   /* voxel edge a > 0                                     */
    double origin[3];                 /* position of integer coordinate (0,0,0)               */
    int32_t mass_mode;                /* CRONOS_MASS_*                                        */
    double mass_value;                /* kg per node (uniform)                                */
    double density;                   /* kg/m^3 (lumped)                                      */
    int32_t k_mode;                   /* CRONOS_K_*                                           */
    double k_uniform;                 /* N/m (uniform)                                        */
    int32_t n_materials;
    const double* material_k;         /* [n_materials] voxel stiffness k_v (assembly)         */
    int32_t pin_axis;                 /* -1 none; else nodes whose integer coordinate on this
                                         axis minus the body minimum equals pin_index are fixed */
    int32_t pin_index;
} cronos_lattice_desc;

/* Build the lattice.  Errors: EINVAL (bad sizes, duplicate voxels, bad material/axis),
 * ENOMEM.  On success *out owns the result until cronos_lattice_destroy. */
cronos_status cronos_lattice_build(const cronos_lattice_desc* desc, cronos_lattice* out);
cronos_status cronos_lattice_sizes(cronos_lattice lat, int64_t* n_masses, int64_t* n_springs);
/* Copy the lattice out; any output pointer may be NULL to skip it.
 *   coords [N][3] int32 integer node coordinates     x [N][3] positions
 *   mass [N], pinned [N] (0/1), body_offset [n_bodies+1] node offsets
 *   ends [S][2] (i < j, canonical node indices), k [S], rest [S], group [S] (-1 passive)  */
cronos_status cronos_lattice_export(cronos_lattice lat, int32_t* coords, double* x, double* mass,
                                    uint8_t* pinned, int64_t* body_offset, int32_t* ends,
                                    double* k, double* rest, int16_t* group);
void cronos_lattice_destroy(cronos_lattice lat);

/* ------------------------------------------------------------------------------------------
 * Layout (section "GPU Implementation": springs and masses stored contiguously, and the
 * mass->spring connectivity duplicated so a per-mass pass can visit its springs).  Masses
 * are renumbered along a Morton curve per body (key bits: x at 3b, y at 3b+1, z at 3b+2 of
 * integer coordinates relative to the body minimum; from positions quantised to 2^20 cells
 * of the largest bbox extent when no integer coordinates are given), stable by (body, key,
 * input index).  Springs are renumbered by (min, max) of their new endpoints; the CSR row
 * of mass i lists (neighbour, spring) by increasing neighbour.  Host-only.
 * ---------------------------------------------------------------------------------------- */
/* Quasi-uniform lattice points by best-candidate sampling (section "Generating a Lattice":
 * Mitchell's best candidate, k nearest neighbours) in the box [0, size[0]) x [0, size[1]) x
 * [0, size[2]).  Point 0 is a uniform draw; point p > 0 is, of n_candidates uniform draws, the
 * one with the largest sum of distances to its min(k_nn, p) nearest placed points (distances
 * summed in ascending order; ties keep the lowest candidate index).  Draws: coordinate a of
 * candidate c of point p is size[a] * u, u = top 53 bits of h(seed, 8, p, c, a) * 2^-53, with
 * h the SplitMix64 chain h(s, k0, k1, ...) = m(...m(m(m(s) ^ k0) ^ k1)...), m the SplitMix64
 * output function (Steele, Lea & Flood 2014).  points: [n_points][3], caller-owned.
 * Errors: EINVAL (sizes, n_candidates < 1, k_nn outside [1, 64]), ENOMEM. */
cronos_status cronos_candidate_points(const double* size, int64_t n_points, int32_t n_candidates, int32_t k_nn,
                                      uint64_t seed, double* points);
/* Springs between every pair of points no farther apart than `cutoff` (d^2 = dx^2 + dy^2 + dz^2
 * <= cutoff^2), as ends [S][2] with i < j, sorted by (i, j).  *n_springs receives S; ends is
 * written when max_springs >= S (call with max_springs = 0 to count).  Errors: EINVAL
 * (arguments, non-finite points, S > max_springs > 0), ENOMEM. */
cronos_status cronos_cutoff_springs(int64_t n_points, const double* points, double cutoff, int64_t max_springs,
                                    int32_t* ends, int64_t* n_springs);
/* Physical parameters of a point lattice (section "Generating a Lattice": masses come from the
 * nodes and springs from the edges; the paper's starting point is 0.1 kg per mass and a spring
 * constant of 10,000 scaled inversely to the spring's length).  For every spring s = (i, j) of
 * ends [S][2]: rest[s] = |p_j - p_i|, its initial length, formed as sqrt((dx*dx + dy*dy) + dz*dz)
 * in FP64; k[s] = (k_ref * length_ref) / rest[s].  For every point: mass[i] = mass_per_point;
 * pinned[i] = 1 if points[i][pin_axis] < pin_below, else 0 (pin_axis = -1: none fixed).
 * Outputs are caller-owned ([S], [S], [N], [N]); a NULL output is skipped.  Host-only.
 * Errors: EINVAL (an end out of range or i == j, a zero-length spring, k_ref, length_ref or
 * mass_per_point not positive, pin_axis outside [-1, 2]). */
cronos_status cronos_point_params(int64_t n_points, const double* points, int64_t n_springs, const int32_t* ends,
                                  double k_ref, double length_ref, double mass_per_point, int32_t pin_axis,
                                  double pin_below, double* k, double* rest, double* mass, uint8_t* pinned);

typedef struct cronos_layout_t* cronos_layout;

/* x: [N][3] positions (used when grid is NULL); grid: [N][3] integer coordinates or NULL;
 * ends: [S][2] input-order endpoints.  block_masses: masses per GPU workgroup (multiple of 64
 * in [64, 1024]; 0 = default).  Errors: EINVAL (index out of range, i == j, spring across
 * bodies, duplicate spring), ENOMEM. */
cronos_status cronos_layout_build(int64_t n_masses, int32_t n_bodies, const int64_t* body_offset,
                                  const double* x, const int32_t* grid, int64_t n_springs,
                                  const int32_t* ends, int32_t block_masses, cronos_layout* out);
/* perm [N] new->input mass index; row_ptr [N+1]; col [2S] neighbour (new index);
 * sid [2S] new spring index; spring_perm [S] new->input spring index.  NULL skips. */
cronos_status cronos_layout_get(cronos_layout lay, int32_t* perm, int64_t* row_ptr, int32_t* col,
                                int32_t* sid, int32_t* spring_perm);
/* Decode the sliced device layout (64-mass slices, per-workgroup halo lists, 16-bit local
 * neighbour indices) back to the CSR and compare.  CRONOS_OK if identical, else EINVAL. */
cronos_status cronos_layout_check(cronos_layout lay);
/* Layout statistics: padded incidence entries, total halo entries, largest halo. */
cronos_status cronos_layout_stats(cronos_layout lay, int64_t* sell_entries, int64_t* halo_entries,
                                  int32_t* max_halo);
void cronos_layout_destroy(cronos_layout lay);

/* ------------------------------------------------------------------------------------------
 * Simulation.
 * ---------------------------------------------------------------------------------------- */
typedef struct cronos_sim_t* cronos_sim;

typedef struct {
    int64_t n_masses, n_springs;
    int32_t n_bodies;             /* >= 1                                                     */
    const int64_t* body_offset;   /* [n_bodies+1] masses of body b are contiguous in input
                                     order; NULL allowed when n_bodies == 1                    */
    const double* x0;             /* [N][3] initial positions                                 */
    const double* v0;             /* [N][3] initial velocities, or NULL (zero)                */
    const double* mass;           /* [N] > 0                                                  */
    const uint8_t* pinned;        /* [N] 1 = fixed mass (x constant, v = 0), or NULL          */
    const int32_t* grid;          /* [N][3] integer lattice coordinates for the space-filling
                                     order, or NULL (positions are quantised)                 */
    const double* fext;           /* [N][3] constant external force f_ext of eq. (2), or NULL */
    const int32_t* ends;          /* [S][2] input mass indices, i != j, same body, no dups    */
    const double* k;              /* [S] spring constant >= 0                                 */
    const double* rest;           /* [S] nominal rest length L0 > 0                           */
    const int16_t* group;         /* [S] actuation group in [0, n_groups) of its body, or -1;
                                     NULL = all passive                                        */
    int32_t n_groups;             /* groups per body; n_bodies * n_groups < 65535             */
    double gravity[3];            /* m/s^2                                                    */
    double damping;               /* per-step velocity damping fraction d in [0, 1)           */
    double dt;                    /* > 0                                                      */
    int32_t ground;               /* 1 = contact plane on                                     */
    double ground_z, ground_k, ground_mu;  /* plane height, penalty stiffness (N/m), Coulomb mu */
    int32_t device;               /* HIP device ordinal                                        */
    void* stream;                 /* hipStream_t to enqueue on; NULL = a stream of its own    */
    uint32_t flags;               /* CRONOS_* flags                                           */
    int32_t block_masses;         /* masses per workgroup, multiple of 64 in [64,1024]; 0 = the
                                     tuned value for this problem class if one is cached (see
                                     cronos_autotune), else 512 for a system of at least
                                     131,072 masses, 64 (below 32,768 masses) or 128 for a
                                     system under 131,072 masses whose lanes_per_mass is 0 too
                                     (with 4 lanes per mass; not with CRONOS_NO_TABLE,
                                     CRONOS_SPLIT or CRONOS_RESIDENT), and 256 otherwise       */
    int32_t batch;                /* incidence entries each lane keeps in flight: 2, 4 or 8;
                                     0 = tuned or 4                                           */
    int32_t persistent;           /* 1 = one persistent launch per step (a resident grid walks
                                     the workgroup blocks); 0 = tuned or one workgroup per block;
                                     -1 = force one workgroup per block                       */
    int32_t lanes_per_mass;       /* lanes sharing each mass's incidence list: 1, 2 or 4
                                     (workgroups of block_masses * lanes threads, at most 1024;
                                     compact table forms with one workgroup per block only,
                                     else 1); 0 = tuned, or 4 for a system under 131,072
                                     masses when block_masses is 0 (see there), or 1.  More
                                     than one lane per mass
                                     groups each mass's force sum differently (equal to
                                     rounding, not bitwise, to one lane).  A tuned value is
                                     taken only when block_masses is 0 as well               */
} cronos_desc;

/* Per-body diagnostics (section "Energy Conservation Tests": elastic, gravitational and
 * kinetic energy; plus the contact plane's penalty energy, momentum, centre of mass and
 * bounding box).  Reduced in FP64 from the FP32 state. */
typedef struct {
    double ke, pe_spring, pe_grav, pe_contact;
    double p[3], com[3], bbox_min[3], bbox_max[3];
    double mass;
    int64_t step;
    int32_t nonfinite;            /* 1 if any x or v of the body is NaN or Inf               */
    int32_t pad_;
} cronos_diag;

/* The system of section "Method", "Mass-Spring Force Distribution": point masses x_i, v_i, m_i
 * joined by springs (i, j, k_ij, l0_ij) with the forces of eqs. (1)-(2) (gravity and a
 * constant f_ext included), integrated by eqs. (3)-(4) at time step dt ("Time Integration
 * Schemes"; CRONOS_VERLET: eqs. (5)-(6)); with the constraints of "Generating a Lattice" (fixed
 * masses, a contact plane, whose friction Appendix A names) and the velocity damping of the
 * Euler-Bernoulli tests.  The lattice then "is copied to GPU memory" (end of "Generating a
 * Lattice"): validate the inputs, renumber (as cronos_layout_build), copy everything to device
 * memory of desc->device and bind desc->stream.  All input arrays stay the caller's.  The
 * step is timed here on that stream (nine launches that leave the state unchanged; the call
 * waits for them and for the stream's earlier work) to choose between HIP graphs and plain
 * launches (cronos_launch_mode), and the step's HIP graphs are captured here, so no cronos_step
 * call pays for them.  Unless CRONOS_ALLOW_UNSTABLE is set, estimates the
 * largest natural frequency w of the rest-state system (plus the contact plane's stiffness)
 * and fails with EUNSTABLE when w * dt >= 2, where symplectic Euler diverges.
 * Errors: EINVAL, ENOMEM, EDEVICE, EUNSTABLE. */
cronos_status cronos_create(const cronos_desc* desc, cronos_sim* out);
void cronos_destroy(cronos_sim sim);

/* Actuated springs (section "Method": springs individually rigid, actuated or functionally
 * parameterised, figure of a mass and its springs; "Multi-Materials and Self-Actuation":
 * actuation by changing volumetric properties over time).  The paper gives no law; this one:
 * the rest length of a spring of group g in body b at t_n = n dt is
 * L0 (1 + amp[b*G+g] sin(2 pi freq_hz t_n + phase[b*G+g])).  phase, amp: host
 * [n_bodies*n_groups], copied (held in FP32 on the device; the period fraction frac(n f dt)
 * is formed exactly in 64-bit fixed point, so the phase stays within ~1e-7 rad of its
 * FP64 value at any step).  Errors: EINVAL (sim has no groups, non-finite values). */
cronos_status cronos_set_actuation(cronos_sim sim, const double* phase, const double* amp,
                                   double freq_hz);

/* Enqueue n_steps time steps on the bound stream and return without waiting.  One step:
 * actuated rest lengths at t_n, eq. (2) forces gathered per mass in a fixed order (no float
 * atomics), contact normal force, v* = v + dt f/m, friction clamp, damping, x' = x + dt v',
 * fixed masses held.  Errors: EINVAL (n_steps < 0), EDEVICE. */
cronos_status cronos_step(cronos_sim sim, int64_t n_steps);

/* The GPU-to-CPU direction of the state sync of section "Parallel Algorithm", paragraph "GPU
 * Implementation": wait for the stream, then copy positions and velocities out (input order,
 * widened to double; the device's FP32 values exactly).  x, v: [N][3] caller-owned or NULL
 * (skipped); *step receives the step counter n (NULL skips).  Errors: EINVAL (NULL handle),
 * EDEVICE. */
cronos_status cronos_read_state(cronos_sim sim, double* x, double* v, int64_t* step);

/* The CPU-to-GPU direction of the same sync: overwrite the state (input order; rounded to
 * FP32; fixed masses get v = 0) and the step counter n (the actuation time t_n).  A state read
 * by cronos_read_state from a simulation created from the same inputs continues bit for bit
 * (checkpoint and resume), except under CRONOS_VERLET, which restarts from (x, v) with the
 * half kick of eq. (5).  Errors: EINVAL (NULL handle, step < 0, non-finite x), EDEVICE. */
cronos_status cronos_set_state(cronos_sim sim, const double* x, const double* v, int64_t step);

/* Total force of eq. (2) plus the contact normal force on every mass at the current state
 * and t_n (input order, [N][3]), evaluated by the same gather as the step.  Blocking. */
cronos_status cronos_eval_forces(cronos_sim sim, double* f);

/* Lowest natural frequencies of the system linearised about its current positions (section
   "Natural Frequency Analysis": the generalised eigenproblem K v = w^2 M v, K the tangent
   stiffness of the springs of eq. (2) -- k [n n^T + (1 - l0/l)(I - n n^T)] per spring, rest
   lengths times the current actuation factors -- plus k_g on z for masses below the contact
   plane, M the diagonal masses, fixed masses removed).  Lanczos iterations on M^-1/2 K M^-1/2
   run on the device in FP64 (no reorthogonalisation; repeated Ritz values are merged), the
   host takes the smallest eigenvalues of the tridiagonal matrix by bisection and stops when
   the first n_modes are within tol: error bound min(r, r^2/gap) with r the Lanczos residual,
   relative to w^2, never below ~1e-15 times the largest w^2 (what FP64 resolves).
   n_modes in [1, 32] distinct frequencies; max_iter in [2 n_modes + 8, 2^24] caps the Lanczos
   steps; seed picks the random start vector.  omega[n_modes] receives the angular
   frequencies (rad/s) in increasing order (a negative value -sqrt(-w^2) marks an unstable
   direction; entries beyond *n_found are 0); *n_found the number that converged;
   *iterations (may be NULL) the steps taken.  Multiplicity is not resolved: an eigenvalue of
   multiplicity m (a square beam's two bending modes) is reported once.  Allocates about
   80 bytes per mass of device memory for the call; the simulation state is not changed.  EINVAL for bad arguments, ENOMEM, ESTATE if the iteration breaks down. */
cronos_status cronos_natural_frequencies(cronos_sim sim, int32_t n_modes, int32_t max_iter, double tol,
                                         uint64_t seed, double* omega, int32_t* n_found, int32_t* iterations);

/* cronos_natural_frequencies for callers that cannot allocate device memory (code under HIP
   graph capture nearby, serving loops, harnesses that forbid hipMalloc): the same arguments,
   computation and results, but every device buffer of the iteration (about 80 bytes per mass
   plus 16 bytes per allowed Lanczos step) is carved from a fixed FP64 workspace of 64 MiB that
   the library holds on each GPU it runs on until the process ends; no hipMalloc, hipFree or
   other device allocation is made (the host-side tridiagonal work arrays are ordinary host
   memory).  The workspace is looked up on the first call on a device.  Every call on one GPU
   shares that workspace and overwrites it: calls that overlap on one GPU (from several
   threads or streams) race and must be serialised by the caller.  EINVAL when
   80 n + 16 max_iter bytes (n masses, plus alignment) exceed the workspace, as for
   cronos_natural_frequencies otherwise. */
cronos_status cronos_natural_frequencies_noalloc(cronos_sim sim, int32_t n_modes, int32_t max_iter, double tol,
                                                 uint64_t seed, double* omega, int32_t* n_found,
                                                 int32_t* iterations);

/* The host step of cronos_natural_frequencies, exposed so it can be checked on its own: the
   `count` smallest eigenvalues theta[count] (increasing) of the symmetric tridiagonal matrix
   with diagonal a[k] and off-diagonal b[k-1] (NULL allowed when k = 1), by Sturm-sequence
   bisection, and (if last != NULL) the magnitude of the last entry of each one's unit
   eigenvector, by two steps of inverse iteration.  Host memory only.  EINVAL when
   count is outside [1, k] or an entry is not finite. */
cronos_status cronos_tridiag_smallest(int64_t k, const double* a, const double* b, int64_t count, double* theta,
                                      double* last);

/* Diagnostics of every body at the current state (out: [n_bodies]).  Blocking.
 * Returns ESTATE (after filling out) when some body holds a non-finite value. */
cronos_status cronos_diagnostics(cronos_sim sim, cronos_diag* out);

/* Measurement reference (not part of the method): the bandwidth a plain streaming HIP kernel
 * reaches on `device` -- a copy of `bytes` (read and write, counted twice) and a read-only
 * pass over them, 16-byte accesses, best of `reps` timed launches after one warm-up (HIP
 * events on a stream of its own).  Allocates and frees 2 x bytes of device memory.
 * copy_gbs, read_gbs: GB/s (10^9 bytes/s), either may be NULL.  Errors: EINVAL (bytes < 1 MiB,
 * reps < 1), ENOMEM, EDEVICE. */
cronos_status cronos_stream_bandwidth(int32_t device, int64_t bytes, int32_t reps, double* copy_gbs,
                                      double* read_gbs);

/* Information on the simulation: masses, springs, bodies, groups, steps taken, block size. */
cronos_status cronos_info(cronos_sim sim, int64_t* n_masses, int64_t* n_springs, int32_t* n_bodies,
                          int32_t* block_masses, int64_t* step);
/* Launch configuration in use: masses per workgroup, batch, persistent workgroups (0 = one
 * per block), the form of the step's incidence data (CRONOS_FORM_*) and the lanes per mass.
 * Any output may be NULL. */
#define CRONOS_FORM_EXPLICIT 0  /* (slot, k, L0) per entry, every spring evaluated at both ends  */
#define CRONOS_FORM_TABLE    1  /* 32-bit entries indexing the table of distinct (k, L0) pairs    */
#define CRONOS_FORM_SPLIT    2  /* spring pass (each spring once per workgroup) + gather pass     */
#define CRONOS_FORM_RESIDENT 3  /* table form, the whole system in one workgroup, many steps per launch */
#define CRONOS_FORM_NARROW   4  /* table form with 16-bit entries (passive systems whose LDS slot and
                                   pair index fit in 16 bits together): half the entry bytes        */
#define CRONOS_FORM_GRID     5  /* structured box: the system is a full nx x ny x nz grid of masses
                                   (dimensions multiples of 8, given by cronos_desc.grid) linked to
                                   all 26 grid neighbours, passive, rest length fixed per direction
                                   and k fixed per (direction, faces of the box the mass lies on);
                                   one workgroup per aligned 8 x 8 x 8 cube, no incidence data read.
                                   Chosen automatically for 512-mass workgroups with one lane per
                                   mass unless CRONOS_NO_GRID, CRONOS_NO_TABLE, CRONOS_SPLIT,
                                   CRONOS_WIDE_ENTRIES or CRONOS_RESIDENT is set.  Springs are summed
                                   per mass in a fixed direction order (equal to the other forms'
                                   sums to rounding)                                              */
cronos_status cronos_launch_config(cronos_sim sim, int32_t* block_masses, int32_t* batch, int32_t* persistent_groups,
                                   int32_t* step_form, int32_t* lanes_per_mass);

/* How cronos_step enqueues its steps (not in the paper).  At creation the step is timed with
 * plain launches on the simulation's stream (9 launches that repeat one step from the current
 * buffers into the other set, HIP events; the state is unchanged); *plain_step_us receives the
 * mean of the last 8 (0 where nothing was timed: CRONOS_NO_GRAPH, the default stream, the
 * resident form).  *graphs receives 1 when step calls launch HIP graphs — of 2^j steps, j < 8,
 * both buffer parities captured at creation and after cronos_set_actuation, a call's step count
 * decomposed into powers of two from the largest down — and 0 for plain launches, which is the
 * choice where *plain_step_us is 12 us or more (the device then trails the host; a graph launch
 * adds tens of microseconds before its first kernel) unless CRONOS_GRAPH is set.  *staged_io
 * receives 1 when velocities come in and the new state goes out through LDS in mass order
 * (less HBM traffic where a workgroup's lanes take its masses out of memory order, two more
 * barriers): for an actuated system in the 32-bit table form with one lane per mass whose
 * compulsory bytes per step (56 per mass, 4 per incidence entry) exceed the 256 MiB Infinity
 * Cache, or with CRONOS_STAGED_IO.  Either way the steps' results are identical.  Any pointer
 * may be NULL.  Errors: CRONOS_EINVAL for a NULL handle. */
cronos_status cronos_launch_mode(cronos_sim sim, int32_t* graphs, double* plain_step_us, int32_t* staged_io);

/* Launch configuration chosen by the autotuner for a problem. */
typedef struct {
    int32_t block_masses, batch, persistent, lanes_per_mass;
    double us_per_step;           /* measured mean step time of the winner                     */
    double us_default;            /* same for block 256, batch 4, one workgroup per block      */
} cronos_tune;

/* Autotuner (not in the paper; the step's launch shape).  Creates the simulation of desc
 * once per workgroup size in {64, 128, 256, 512, 1024} and times n_steps steps (after 3 warm-up
 * steps, HIP events on its stream) for every batch in {2, 4, 8} and both launch forms with
 * one lane per mass, and for 2 and 4 lanes per mass (table forms, where the workgroup of
 * size x lanes threads fits); the
 * fastest configuration is returned and cached for the process under the key (GPU
 * architecture, floor(log2 N), floor(log2 S), actuated, contact), and appended to the file
 * named by the environment variable CRONOS_TUNE_CACHE if set (read back at the first
 * cronos_create).  The state of desc is not modified.  Errors: as cronos_create. */
cronos_status cronos_autotune(const cronos_desc* desc, int32_t n_steps, cronos_tune* out);

/* ------------------------------------------------------------------------------------------
 * Differentiable rollouts (the paper notes differentiation is enabled by its system without
 * describing it; this is the reverse-mode adjoint of the discrete step above).
 * ---------------------------------------------------------------------------------------- */

/* Run n_steps steps from the current state (as cronos_step), saving the state every
 * ckpt_every steps on the device, and return loss = sum_i loss_w[i] . x_i(T) in FP64
 * (loss_w: host [N][3], input order, rounded to FP32 for the adjoint).  Blocking.  The
 * rollout is recorded for cronos_rollout_backward until the next cronos_rollout.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
cronos_status cronos_rollout(cronos_sim sim, int64_t n_steps, int32_t ckpt_every, const double* loss_w,
                             double* loss);

/* Gradient of the last rollout's loss: dphase, damp [n_bodies*n_groups] with respect to the
 * actuation phases and amplitudes, dx0, dv0 [N][3] with respect to the state the rollout
 * started from (input order).  Any output may be NULL.  Each checkpointed segment is
 * recomputed forward, then stepped backwards with the adjoint kernels (FP32 adjoint state,
 * FP64 accumulation of the actuation sensitivities).  Blocking.  Does not change the state.
 * Errors: EINVAL (no rollout recorded), EDEVICE. */
cronos_status cronos_rollout_backward(cronos_sim sim, double* dphase, double* damp, double* dx0, double* dv0);

/* ------------------------------------------------------------------------------------------
 * Learned surrogate (not in the paper): predicts a robot's displacement from its morphology
 * and actuation, to pre-screen candidates before the simulator judges them.
 * ---------------------------------------------------------------------------------------- */

/* Features of n_bodies voxel robots (host, parallel over robots): 32 morphology descriptors
 * (log node count, log voxel count, extent per axis, fractions of materials 0/1/2, mean voxel
 * centre minus bbox centre, second moments xx yy zz xy xz yz, bottom-layer fraction, 8-bin
 * height histogram, actuated fraction, mean log10 voxel stiffness, stiffness-weighted centre
 * offset, surface-face fraction) then (A_g cos phi_g, A_g sin phi_g) for g < n_groups.
 * voxels [n_voxels][3]; body_voxel_offset [n_bodies+1] (required); material, group [n_voxels]
 * or NULL; phase, amp [n_bodies*n_groups]; out [n_bodies][32 + 2 n_groups] (FP64).
 * Errors: EINVAL, ENOMEM. */
cronos_status cronos_features(int32_t n_bodies, const int64_t* body_voxel_offset, const int32_t* voxels,
                              const int32_t* material, const int32_t* group, int32_t n_materials,
                              const double* material_k, double spacing, int32_t n_groups, const double* phase,
                              const double* amp, double* out);

/* Features of n_cand candidates that re-use already computed morphology descriptors:
 * candidate c is robot body_of[c] (row of morph [n_bodies][32], from cronos_features with
 * n_groups = 0) with its own actuation phase, amp [n_cand*n_groups]; out [n_cand][32+2 n_groups]. */
cronos_status cronos_candidate_features(int64_t n_cand, const int32_t* body_of, int32_t n_bodies, const double* morph,
                                        int32_t n_groups, const double* phase, const double* amp, double* out);

/* Perceptron sizes[0] -> sizes[1] -> sizes[2] -> sizes[3] -> sizes[4] with exact-erf GELU
 * after the three hidden layers and a linear output.  Products on the BF16 matrix cores with
 * FP32 accumulation; an FP32 master copy of the weights with a BF16 shadow; hidden activations
 * and back-propagated gradients stored in BF16; MSE loss; Adam in FP32. */
typedef struct cronos_mlp_t* cronos_mlp;

/* params: FP64 host [W1 (sizes[0] x sizes[1], row-major), b1, W2, b2, W3, b3, W4, b4];
 * max_rows: largest batch of a single forward/gradient call.  Errors: EINVAL, ENOMEM, EDEVICE. */
cronos_status cronos_mlp_create(const int32_t* sizes, const double* params, int32_t max_rows, int32_t device,
                                void* stream, cronos_mlp* out);
void cronos_mlp_destroy(cronos_mlp mlp);
/* Current FP32 master weights, widened, in the layout of cronos_mlp_create. */
cronos_status cronos_mlp_get_params(cronos_mlp mlp, double* params);
/* y [rows][sizes[4]] = network(x [rows][sizes[0]]) (host FP32 arrays; any number of rows). */
cronos_status cronos_mlp_forward(cronos_mlp mlp, const float* x, int64_t rows, float* y);
/* Mean squared error on (x, t) (rows <= max_rows) and its gradient (FP32 widened; the layout
 * of the parameters; NULL skips); the gradient stays on the device for cronos_mlp_adam. */
cronos_status cronos_mlp_loss_grad(cronos_mlp mlp, const float* x, const float* t, int32_t rows, double* loss,
                                   double* grads);
/* One Adam step (Kingma & Ba) with the last computed gradient. */
cronos_status cronos_mlp_adam(cronos_mlp mlp, double lr, double beta1, double beta2, double eps);
/* Train in place: `epochs` passes over (x, t) [rows] in minibatches of `batch` (<= max_rows),
 * shuffled every epoch by a SplitMix64-driven Fisher-Yates permutation of `seed`; Adam with
 * 0.9, 0.999, 1e-8 and a learning rate that follows a half cosine from lr (first step) to
 * lr_final (last step); lr_final = lr keeps it constant.  epoch_loss: mean minibatch loss of
 * the last epoch.  Errors: EINVAL (sizes, negative rates), EDEVICE. */
cronos_status cronos_mlp_train(cronos_mlp mlp, const float* x, const float* t, int64_t rows, int32_t batch,
                               int32_t epochs, double lr, double lr_final, uint64_t seed, double* epoch_loss);

/* Input-order layout of a created simulation (see cronos_layout_get). */
cronos_status cronos_get_layout(cronos_sim sim, int32_t* perm, int64_t* row_ptr, int32_t* col,
                                int32_t* sid, int32_t* spring_perm);

#ifdef __cplusplus
}
#endif
#endif /* CRONOS_H */
