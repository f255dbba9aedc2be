/*
 * snake.h - C ABI of the batched compliant-constraint snake solver for
 * AMD Instinct MI355X (gfx950).
 *
 * The solver advances batches of independent soft snakes.  Each snake is a
 * chain of B = M x S rigid segments (M actuator modules of S segments).
 * It follows Gasoto, Macklin et al., "A Validated Physical Model For
 * Real-Time Simulation of Soft Robotic Snakes":
 *   - bodies in maximal coordinates: centre x and unit quaternion
 *     q = (w, x, y, z), body to world (section "Rigid Bodies"), lumped
 *     mass (section "Particles");
 *   - compliant bilateral constraints c(q, p) + E lambda = 0 with a
 *     block-diagonal compliance E, plus unilateral ground contact with a
 *     Coulomb cone (section "Simulator", the equations of motion); the
 *     target pressures p are parameters of the actuation constraints;
 *   - per joint a stretch block in the form of the rigid attachment
 *     constraint (eq. rigid_to_particle) and a bend-twist block whose rest
 *     rotation follows the chamber pressure (eq. expansion: strain, hence
 *     rest curvature, linear in pressure);
 *   - chamber latency: first-order lag, or the quadratic-inflation /
 *     capped-deflation law (eq. delta_p_i, eq. deflation);
 *   - open-loop serpenoid command (eq. snake_control) or piecewise-constant
 *     schedules, evaluated on the device, or commands set by the caller;
 *   - a first-order implicit step (section "Time-Stepping") solved at the
 *     position level by block-Jacobi iterations on the compliant system
 *     whose linearisation is eq. schur_system.  Each block increment is
 *     scaled by relax / (largest number of blocks on one of its bodies)
 *     and applied to both the multipliers and the bodies.
 *
 * Conventions
 *   - Units are SI.  World z is up, the ground is the plane z = 0.  Body
 *     e_x runs along the chain (body i -> i+1).
 *   - Device arrays are structure-of-arrays FP32: component k of body i of
 *     the whole batch sits at [k * N + i] (N = total bodies).  Joint j of
 *     snake s has global index joint_off[s] + j = body_off[s] - s + j.
 *   - Calls are asynchronous on the stream given to sim_create unless a
 *     description says otherwise.  A HIP stream is passed as void*; NULL is
 *     the default stream.
 *   - Return values: SIM_OK (0) or a negative error code.  The message of
 *     the last error of the calling thread is returned by sim_last_error().
 *     No C++ exception crosses this boundary.
 */
#ifndef SNAKE_H
#define SNAKE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define SIM_OK 0
#define SIM_EINVAL (-1)  /* bad argument or descriptor                        */
#define SIM_ENOMEM (-2)  /* workspace smaller than sim_workspace_bytes()      */
#define SIM_EDEVICE (-3) /* HIP runtime or launch failure                     */
#define SIM_ESTATE (-4)  /* call not valid in the object's current state      */

/* ---- memory kinds for pointers passed to set/read/write calls ---- */
#define SIM_MEM_HOST 0
#define SIM_MEM_DEVICE 1

/* ---- chamber pressure law ---- */
#define SIM_LAW_LAG 0   /* p <- u + (p - u) exp(-h / tau) every substep,     */
                        /* tau = tau_inflate if u > p else tau_deflate        */
#define SIM_LAW_PAPER 1 /* once per step, in psi: inflating p += p_s k_i     */
                        /* ((u-p)/p_s)^2; deflating p -= min(k_d p, T_p),     */
                        /* not below the target (eq. delta_p_i, deflation)    */

/* ---- command source ---- */
#define SIM_CTRL_EXTERNAL 0  /* commands set by sim_set_pressures            */
#define SIM_CTRL_SERPENOID 1 /* a_m = clamp(sin(2 pi f t + alpha m + phase0) */
                             /*        + offset, -1, 1), t = (n+1) dt        */
#define SIM_CTRL_SCHEDULE 2  /* piecewise constant, lengths in steps         */

/* ---- multiplier initialisation at every substep ---- */
#define SIM_WARM_ZERO 0 /* lambda = 0                                        */
#define SIM_WARM_PREV 1 /* lambda = previous substep's, bodies moved by      */
                        /* W J^T lambda before iterating                      */
#define SIM_WARM_MLP 2  /* joint lambda predicted by the network set with     */
                        /* sim_set_mlp (contacts start at 0), bodies moved by */
                        /* W J^T lambda; with mlp_fallback the zero start is  */
                        /* used wherever it has the smaller residual after    */
                        /* mlp_fallback_k iterations (0: at the start)        */

/* ---- solver of the implicit step (section "Time-Stepping") ---- */
#define SIM_SOLVER_JACOBI 0 /* block-Jacobi iterations on the compliant      */
                            /* system (iters, tol, relax, warm_start)        */
#define SIM_SOLVER_NEWTON 1 /* the paper's scheme: newton_iters Newton       */
                            /* iterations, each solving eq. schur_system     */
                            /* [J W J^T + E] dl = b with pcr_iters           */
                            /* preconditioned conjugate-residual iterations  */
                            /* (diagonal preconditioner); normal contact by  */
                            /* the Fischer-Burmeister function, friction by  */
                            /* the natural map onto the Coulomb disc.  Stops */
                            /* early at a Newton iterate with residual <= tol*/
                            /* (tol > 0); the residual adds the friction     */
                            /* rows' natural map to the Jacobi measure.      */
                            /* Computes in double.  Takes SIM_WARM_ZERO or   */
                            /* SIM_WARM_PREV; no split substeps              */
                            /* (sim_step_record).                            */
#define SIM_SOLVER_GS 2     /* block Gauss-Seidel: sweeps over the greedy    */
                            /* block colouring (SIM_IDX_BLK_COLOR), each     */
                            /* colour's blocks taking their local solutions  */
                            /* scaled by relax (no averaging) at the current */
                            /* state; iters / tol count and stop sweeps as   */
                            /* the Jacobi solver does its iterations.  FP32. */
                            /* Needs SIM_WARM_ZERO; no split substeps.       */

/* ---- flags ---- */
#define SIM_FLAG_FIXED_ROOT 1u /* body 0 of every snake is immovable         */
#define SIM_FLAG_NO_GROUND 2u  /* no ground plane: no contact blocks         */
#define SIM_FLAG_WHEELS 16u    /* the wheeled carriage (section "Rigid Body */
                               /* Joints and Contact"): every segment       */
                               /* carries two rigid wheels on hinge joints  */
                               /* and the wheels, not the segments, touch   */
                               /* the ground, with Coulomb friction at the  */
                               /* wheel's contact point (so a snake rolls   */
                               /* along its wheels and grips sideways, the  */
                               /* anisotropic friction of section "Soft     */
                               /* robotic snake model").  A wheel is a thin */
                               /* disc of radius R/2 and mass m/8 centred   */
                               /* at (0, +-R, -R/2) in its segment's frame, */
                               /* axle along the segment's y axis (the      */
                               /* paper gives no wheel dimensions).  Blocks */
                               /* per wheel: hinge position (attachment     */
                               /* form of eq. rigid_to_particle), hinge     */
                               /* axis (two rigid rows: the bend-twist form */
                               /* at rest angle 0 without its spin row),    */
                               /* contact (normal at the lowest rim point,  */
                               /* friction on the material point that       */
                               /* touched at the start of the substep).     */
                               /* Needs SIM_SOLVER_JACOBI, SIM_WARM_ZERO;   */
                               /* computes in double; no autotune and no    */
                               /* split substeps.  State in SIM_F_WHEEL_*;  */
                               /* the index arrays (sim_read_index) keep    */
                               /* describing the segment chain.             */

/* ---- per-snake status bits (field SIM_F_STATUS) ---- */
#define SIM_STATUS_NONFINITE 1     /* residual became NaN or inf             */
#define SIM_STATUS_NOT_CONVERGED 2 /* tolerance not reached in iters        */
#define SIM_STATUS_FELL_BACK 4     /* a learned start was replaced by zero  */

/* ---- state fields: bit k selects dst[k] / src[k] ---- */
#define SIM_F_POS (1u << 0)            /* float [3][N] body centres          */
#define SIM_F_QUAT (1u << 1)           /* float [4][N] (w, x, y, z)          */
#define SIM_F_VEL (1u << 2)            /* float [3][N] linear velocity       */
#define SIM_F_ANGVEL (1u << 3)         /* float [3][N] angular vel., world   */
#define SIM_F_PRESSURE (1u << 4)       /* float [2][Mtot] chamber pressure,  */
                                       /* fraction of the amplitude          */
#define SIM_F_LAMBDA_JOINT (1u << 5)   /* float [6][Jtot] last substep's     */
                                       /* stretch xyz, twist, bend y, bend z */
#define SIM_F_LAMBDA_CONTACT (1u << 6) /* float [3][N] normal, tangent x, y  */
#define SIM_F_CMD (1u << 7)            /* float [Mtot] command of last step  */
#define SIM_F_RESIDUAL (1u << 8)       /* float [n_snakes] largest final     */
                                       /* residual over the last step        */
#define SIM_F_ITERS (1u << 9)          /* int32 [n_snakes] iterations of the */
                                       /* last step, summed over substeps    */
#define SIM_F_STATUS (1u << 10)        /* int32 [n_snakes] SIM_STATUS_* bits */
#define SIM_F_STEP (1u << 11)          /* int64 [n_snakes] step counter      */
#define SIM_F_ITERS_TOTAL (1u << 12)   /* int64 [n_snakes] all iterations    */
#define SIM_F_WHEEL_POS (1u << 13)     /* float [3][2N] wheel centres; wheel */
                                       /* 2 b + k of body b, k = 0 on +y    */
                                       /* (SIM_FLAG_WHEELS batches only)    */
#define SIM_F_WHEEL_QUAT (1u << 14)    /* float [4][2N]                     */
#define SIM_F_WHEEL_VEL (1u << 15)     /* float [3][2N]                     */
#define SIM_F_WHEEL_ANGVEL (1u << 16)  /* float [3][2N] world frame         */
#define SIM_F_LAMBDA_WHEEL (1u << 17)  /* float [9][2N] hinge position (3), */
                                       /* hinge axis (x, spin row = 0, z),  */
                                       /* contact (normal, tangent x, y)    */
#define SIM_F_COUNT 18

/* ---- index arrays (sim_read_index), all int32 ---- */
#define SIM_IDX_BODY_OFF 0    /* [n_snakes+1] exclusive prefix sum of B       */
#define SIM_IDX_JOINT_OFF 1   /* [n_snakes+1] of B - 1                        */
#define SIM_IDX_MODULE_OFF 2  /* [n_snakes+1] of M                            */
#define SIM_IDX_BLOCK_OFF 3   /* [n_snakes+1] of 2(B-1) + B (ground) or 2(B-1)*/
#define SIM_IDX_BLK_TYPE 4    /* [n_blocks] 0 stretch, 1 bend-twist, 2 contact*/
#define SIM_IDX_BLK_A 5       /* [n_blocks] first body (global)               */
#define SIM_IDX_BLK_B 6       /* [n_blocks] second body, -1 for a contact     */
#define SIM_IDX_BLK_COLOR 7   /* [n_blocks] greedy colour in block order      */
#define SIM_IDX_DEGREE 8      /* [N] blocks touching each body                */
#define SIM_IDX_BUCKET 9      /* [n_snakes] ceil(log2 B)                      */
#define SIM_IDX_ORDER 10      /* [n_snakes] by B descending, id ascending     */
#define SIM_IDX_COUNT 11

/* Descriptor.  Host memory, read during sim_workspace_bytes / sim_create
 * only (sim_create copies everything it needs).  Per-snake arrays have
 * n_snakes entries. */
typedef struct sim_desc {
    int32_t n_snakes;
    const int32_t* n_modules;       /* M per snake, >= 1                     */
    const int32_t* segs_per_module; /* S per snake, >= 1; B = M S <= 1024   */
    const double* alpha_stretch;    /* compliance per unit length, m/N * m  */
    const double* alpha_bend;       /* rad/(N m) * m; a joint gets value*L  */
    const double* alpha_twist;
    const double* mu;               /* Coulomb friction coefficient          */
    double seg_mass, seg_length, seg_radius, gravity;
    double dt;         /* step length, s                                     */
    int32_t substeps;  /* substeps per step, h = dt / substeps              */
    int32_t iters;     /* iterations per substep (tol <= 0) or the maximum, */
                       /* at most 1e6                                       */
    double tol;        /* > 0: stop a substep at residual <= tol            */
    double relax;      /* scale of every block increment, (0, 1]            */
    int32_t pressure_law;
    double tau_inflate, tau_deflate; /* s, SIM_LAW_LAG                      */
    double kappa_max;  /* rest curvature (1/m) per unit pressure difference */
    double k_inflate, k_deflate, T_p, p_source, amplitude_psi; /* LAW_PAPER  */
    int32_t controller;
    const double* ctrl_freq;   /* per snake, Hz (SERPENOID)                 */
    const double* ctrl_phase0; /* per snake, rad (SERPENOID)                */
    double ctrl_alpha;         /* phase shift between modules, rad          */
    double ctrl_offset;        /* offset inside the clamp                   */
    const int32_t* sched_off;  /* [Mtot+1] piece offsets (SCHEDULE)         */
    const int32_t* sched_steps;/* piece lengths in steps, >= 1              */
    const double* sched_val;   /* piece commands in [-1, 1]                 */
    int32_t warm_start;        /* SIM_WARM_*                                */
    uint32_t flags;            /* SIM_FLAG_*                                */
    int32_t use_graph;         /* 1: replay sim_step launches from a graph  */
    /* Mapping of snakes to lanes.  A workgroup of map_waves wavefronts takes
     * tiles of snakes; each snake owns an aligned power-of-two lane segment
     * of at least map_min_seg lanes (16, 32 or 64), or with map_rows = 1 a
     * segment of its length rounded up to 16 lanes, placed without
     * alignment (map_rows = 2: the same, with snakes of up to 8 bodies in
     * 8-lane half rows, two to a row); map_grid workgroups loop over the tiles (0: one workgroup
     * per tile).  0 selects the default.  autotune = 1 times the candidate
     * mappings on the real batch inside sim_create (the state is restored
     * afterwards) and keeps the fastest; explicit map_* values are then
     * ignored.  Every mapping gives bit-identical results. */
    int32_t autotune;
    int32_t map_waves;         /* 1, 2, 4, 8 or 16; 64 * map_waves >= every segment */
    int32_t map_min_seg;
    int32_t map_grid;
    int32_t mlp_fallback;      /* 1: per snake and substep, keep the learned */
                               /* start only if its residual is not larger   */
                               /* than the zero start's ...                  */
    int32_t map_rows;          /* 0, 1 or 2, see the mapping above          */
    int32_t mlp_fallback_k;    /* ... after this many iterations from each   */
                               /* start (0: the starts themselves; at most   */
                               /* iters).  For k > 0 the zero start runs k   */
                               /* iterations, then the learned start k; the  */
                               /* solve continues from the winner's iterate  */
                               /* k, and the other start's k iterations      */
                               /* count in SIM_F_ITERS.                      */
    int32_t solver;            /* SIM_SOLVER_* (0: Jacobi)                  */
    int32_t newton_iters;      /* NEWTON: Newton iterations per substep,    */
                               /* [0, 10000]                                */
    int32_t pcr_iters;         /* NEWTON: inner iterations per Newton       */
                               /* iteration, [1, 100000]; SIM_F_ITERS counts */
                               /* these                                     */
    int32_t newton_keep_best;  /* NEWTON, 0 or 1: end each substep at the   */
                               /* evaluated Newton iterate of smallest      */
                               /* residual (the earliest of equals), not at */
                               /* the last; 0 is the paper's fixed budget   */
} sim_desc_t;

typedef struct sim sim_t;

/* Workspace size for a descriptor.  Pure host computation: the state of the
 * system described in section "Simulator" (generalized coordinates of every
 * body, section "Rigid Bodies"; one multiplier per constraint row) plus the
 * index work and the tile plan.  Returns SIM_EINVAL for an invalid
 * descriptor. */
int sim_workspace_bytes(const sim_desc_t* d, size_t* bytes);

/* Build a solver (the bodies of sections "Particles" / "Rigid Bodies" with
 * lumped mass, the compliant joint constraints with block-diagonal
 * compliance E and the ground contacts of section "Simulator") in
 * caller-owned device memory `workspace` (at least
 * sim_workspace_bytes, 256-byte aligned, kept alive until sim_destroy) on
 * stream `hip_stream` (borrowed).  Runs the index work on the device,
 * uploads the parameters and sets every snake straight at rest on the
 * ground along +x with zero pressure.  Synchronises the stream before it
 * returns.  Errors: SIM_EINVAL, SIM_ENOMEM, SIM_EDEVICE. */
int sim_create(const sim_desc_t* d, void* workspace, size_t bytes, void* hip_stream,
               sim_t** out);

/* The target pressures p of section "Simulator" (parameters of the
 * actuation constraints), as the commands a_i of eq. snake_control that
 * eq. delta_p_i and eq. deflation turn into chamber pressures.
 * Set one command per module (n == Mtot), in [-1, 1] (clamped): a > 0
 * drives chamber 0 (bends toward positive rotation about body z), a < 0
 * chamber 1.  Used by SIM_CTRL_EXTERNAL and held until the next call.
 * Host memory: NaN gives SIM_EINVAL.  Device memory: NaN is read as 0.
 * Stream-ordered. */
int sim_set_pressures(sim_t* s, const float* cmd, int64_t n, int mem);

/* Advance every snake by n_steps steps of the first-order implicit
 * discretisation of section "Time-Stepping" (each step = `substeps`
 * substeps; each substep solves the compliant system whose linearisation is
 * eq. schur_system with the descriptor's solver), asynchronously.  Launch failures
 * return SIM_EDEVICE; numerical failures are per-snake status bits. */
int sim_step(sim_t* s, int32_t n_steps);

/* Read the state of section "Simulator": body centres and orientations
 * (maximal coordinates, section "Rigid Bodies"), their velocities, the
 * chamber pressures, and the multipliers lambda_b (joints) and lambda_n,
 * lambda_f (contact normal and friction) of the equations of motion.
 * Copy the selected fields (SIM_F_*) to dst[k] for each selected bit k.
 * Host memory: the call synchronises the stream.  Layouts as listed with
 * the field bits. */
int sim_read_state(sim_t* s, uint32_t fields, void* const* dst, int mem);

/* Write the same state (section "Simulator" quantities, as read by
 * sim_read_state).
 * Overwrite the selected fields from src[k] (checkpoint restore and state
 * injection).  A round trip through sim_read_state is bitwise.  Host
 * memory: the call synchronises the stream. */
int sim_write_state(sim_t* s, uint32_t fields, const void* const* src, int mem);

/* Load the warm-start network (snake_mlp.h layout): params[6467] and
 * mean_std[64], host or device memory.  Needed before sim_step when the
 * descriptor's warm_start is SIM_WARM_MLP.  Stream-ordered. */
int sim_set_mlp(sim_t* s, const float* params, const float* mean_std, int mem);

/* Advance n_steps steps like sim_step, substep by substep, and record for
 * every substep and every joint two rows (stretch, bend-twist) of network
 * inputs and targets into caller device memory:
 *   features[rows][32], targets[rows][3], rows = n_steps substeps 2 Jtot,
 * ordered substep-major, then joint (global index), then block.
 * Inputs, at the substep's predicted state (positions x + h v, predicted
 * orientations), vectors in the predicted axes of the joint's first body A:
 *   0-2   stretch violation / L          3-5   2 Im(q0* qA* qB)
 *   6-8   (vA + wA x rA - vB - wB x rB) h / L   9-11 (wB - wA) h
 *   12-14 world up                       15-18 p0, p1, command, rest angle
 *   19-21 this block's previous multipliers / scale
 *   22-24 log10 of the stretch, bend, twist compliance / h^2
 *   25 mu   26-27 previous normal multipliers of A, B / (m 9.81 h^2)
 *   28-29 (z - R) / L of A, B   30 block type (0, 1)   31 i / (B - 1)
 * Targets: the substep's final multipliers, stretch in the axes of A over
 * m 9.81 h^2, bend-twist over m 9.81 h^2 L.  SIM_ENOMEM if capacity_rows is
 * smaller than rows; *written receives rows. */
int sim_step_record(sim_t* s, int32_t n_steps, float* features, float* targets, int64_t capacity_rows,
                    int64_t* written);

/* Copy index array `which` (SIM_IDX_*) to host int32 memory `dst` holding
 * `count` entries (must equal the array's length).  Synchronous. */
int sim_read_index(sim_t* s, int32_t which, int32_t* dst, int64_t count);

/* Sizes: n_snakes, N, Jtot, Mtot, n_blocks (host int64 out[5]). */
int sim_sizes(const sim_t* s, int64_t* out5);

/* Tile plan of a descriptor for a mapping, on the host (no device, no
 * state): snakes in work order (longest first, ties by index) packed into
 * tiles of 64 * waves lanes, aligned power-of-two segments of at least
 * min_seg lanes (rows = 0) or segments of the length rounded up to 16 lanes,
 * best fit (rows = 1; rows = 2: snakes of up to 8 bodies in 8-lane half
 * rows, consecutive ones sharing a row) -- the layout sim_create builds for
 * that mapping.
 * Outputs in caller host memory with room for n_snakes entries:
 *   hdr[tile][4] = {first slot, slot count, some segment crosses a wave
 *                   boundary, rows}
 *   slots[slot][2] = {snake, lane offset << 16 | segment lanes}
 * and *n_tiles.  SIM_EINVAL for a bad descriptor or mapping. */
int sim_plan_tiles(const sim_desc_t* d, int32_t waves, int32_t min_seg, int32_t rows, int32_t* hdr,
                   int32_t* slots, int64_t* n_tiles);

/* Mapping in use: waves per workgroup, minimum segment, grid, tiles,
 * rows layout (host int32 out[5]). */
int sim_mapping(const sim_t* s, int32_t* out5);

/* Release host resources (the caller frees the workspace).  NULL is a
 * no-op.  Waits for the stream. */
void sim_destroy(sim_t* s);

/* Message of the calling thread's last error ("" if none). */
const char* sim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SNAKE_H */
