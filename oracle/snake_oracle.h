/*
 * FP64 CPU oracle of the compliant-constraint snake solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark call it.  It shares no source, header,
 * table or helper with the GPU library and does not include its headers.
 *
 * What it computes (Gasoto, Macklin et al., "A Validated Physical Model For
 * Real-Time Simulation of Soft Robotic Snakes"):
 *   - bodies in maximal coordinates, centre x and unit quaternion q
 *     (section "Rigid Bodies"), lumped mass (section "Particles");
 *   - compliant bilateral constraints c(q,p) + E lambda = 0 with a
 *     block-diagonal compliance E, unilateral ground contact and a Coulomb
 *     cone (section "Simulator", the equations of motion);
 *   - the stretch block has the form of the rigid attachment constraint
 *     (eq. rigid_to_particle) between neighbouring segment end points;
 *   - a pressure-dependent rest shape (eq. expansion: strain 1 + p/Y grows
 *     linearly with pressure, so the rest curvature does too);
 *   - chamber latency: a first-order lag, or the paper's quadratic-inflate /
 *     capped-deflate law (eq. delta_p_i and eq. deflation);
 *   - the open-loop serpenoid command (eq. snake_control);
 *   - a first-order implicit step (section "Time-Stepping") solved at the
 *     position level by block-Jacobi iterations on the compliant system whose
 *     linearisation is eq. schur_system, or by the paper's own scheme:
 *     Newton iterations, each solving eq. schur_system with a fixed number
 *     of preconditioned conjugate-residual iterations (diagonal
 *     preconditioner), contact by a Fischer-Burmeister reformulation; or
 *     block Gauss-Seidel sweeps over the greedy block colouring;
 *   - optionally the wheeled carriage (section "Rigid Body Joints and
 *     Contact"): every segment carries two rigid wheels on hinge joints, and
 *     the wheels, not the segments, touch the ground, with Coulomb friction
 *     at the wheel's contact point.  The paper gives no wheel dimensions;
 *     here a wheel is a thin disc of radius R/2 and mass m/8 whose centre
 *     sits at (0, +-R, -R/2) in its segment's frame, axle along the
 *     segment's y axis (so a segment at rest has its centre at height R,
 *     as without wheels).
 * Every floating-point quantity is double.  No fast-math.
 *
 * Memory layout: array-of-structures per body (x[3*i+k], q[4*i+k] with
 * q = (w, x, y, z)), batch-flat with per-snake offsets given by the caller.
 */
#ifndef SNAKE_ORACLE_H
#define SNAKE_ORACLE_H

#include <stdint.h>

#define ORC_FLAG_FIXED_ROOT 1   /* body 0 has infinite mass and inertia     */
#define ORC_FLAG_NO_GROUND 2    /* no ground plane, no contact blocks       */
#define ORC_FLAG_LINEARISED 8   /* Jacobians frozen at the predicted state  */
#define ORC_FLAG_WHEELS 16      /* wheel carriage: two wheels per segment on */
                                /* hinge joints carry the ground contact    */
                                /* (block-Jacobi solver, zero start only)    */

#define ORC_CTRL_EXTERNAL 0
#define ORC_CTRL_SERPENOID 1
#define ORC_CTRL_SCHEDULE 2

#define ORC_LAW_LAG 0
#define ORC_LAW_PAPER 1

#define ORC_WARM_ZERO 0
#define ORC_WARM_PREV 1
#define ORC_WARM_GIVEN 2        /* lambda0 supplied by the caller in lam_* */

#define ORC_SOLVER_JACOBI 0     /* block-Jacobi iterations (the default)    */
#define ORC_SOLVER_NEWTON 1     /* Newton + preconditioned conjugate residual */
#define ORC_SOLVER_GS 2         /* block Gauss-Seidel over the block colouring */

#define ORC_STATUS_NONFINITE 1
#define ORC_STATUS_NOT_CONVERGED 2
#define ORC_STATUS_FELL_BACK 4

/* Batch description: one entry per snake plus shared constants. */
typedef struct {
    int32_t n_snakes;
    const int32_t* n_modules;        /* [n_snakes] */
    const int32_t* segs;             /* [n_snakes] segments per module */
    const double* alpha_s;           /* [n_snakes] compliance per unit length */
    const double* alpha_b;
    const double* alpha_t;
    const double* mu;                /* [n_snakes] */
    const double* freq;              /* [n_snakes] serpenoid frequency, Hz */
    const double* phase0;            /* [n_snakes] serpenoid phase, rad */
    const int32_t* sched_off;        /* [total_modules+1] piece offsets */
    const int32_t* sched_steps;      /* [pieces] piece length in steps */
    const double* sched_val;         /* [pieces] command value */
    double mass, length, radius, gravity;
    double dt;
    int32_t substeps, iters;
    double tol, relax;
    int32_t law;
    double tau_inf, tau_def, kappa_max;
    double k_i, k_d, T_p, p_s, amp_psi;
    int32_t flags, controller, warm;
    double ctrl_alpha, ctrl_offset;
    int32_t fallback;   /* GIVEN warm start: keep lambda0 only if it is closer */
    int32_t fallback_k; /* ... after this many iterations (0: at the start) */
    int32_t solver;       /* ORC_SOLVER_*; NEWTON takes the zero or previous  */
                          /* warm start, GS the zero one                      */
    int32_t newton_iters; /* NEWTON: outer iterations per substep            */
    int32_t pcr_iters;    /* NEWTON: inner iterations per outer iteration     */
    int32_t newton_keep_best; /* NEWTON: end at the evaluated iterate with the
                               * smallest residual (the earliest of equals)  */
} orc_batch;

/* Batch state, owned by the caller.  Offsets: body_off / module_off /
 * joint_off from orc_offsets().  Bodies hold 3 (x, v, w) or 4 (q) doubles. */
typedef struct {
    double* x;          /* [N*3] */
    double* q;          /* [N*4] */
    double* v;          /* [N*3] */
    double* w;          /* [N*3] angular velocity, world frame */
    double* p;          /* [Mtot*2] chamber pressures, fraction of amp_psi */
    double* cmd;        /* [Mtot] command in effect for the current step */
    double* lam_j;      /* [Jtot*6] stretch (3), twist, bend_y, bend_z */
    double* lam_c;      /* [N*3] normal, tangential x, tangential y */
    double* residual;   /* [n_snakes] max final residual over the last step */
    int32_t* iters;     /* [n_snakes] iterations summed over the last step */
    int32_t* status;    /* [n_snakes] */
    int64_t* iters_total; /* [n_snakes] cumulative iterations */
    int64_t* step;      /* [n_snakes] step counter */
    /* wheel carriage only (NULL otherwise): wheel 2i+k of body i (k = 0 on
     * the +y side), same per-body layouts as above */
    double* wx;         /* [N*2*3] */
    double* wq;         /* [N*2*4] */
    double* wv;         /* [N*2*3] */
    double* ww;         /* [N*2*3] */
    double* lam_w;      /* [N*2*9] hinge position (3), hinge axis (x, unused
                         * spin row, z), wheel contact (normal, tx, ty) */
} orc_state;

/* offsets: body_off, joint_off, module_off, block_off each [n_snakes+1] */
void orc_offsets(const orc_batch* b, int64_t* body_off, int64_t* joint_off,
                 int64_t* module_off, int64_t* block_off);

/* straight chains at rest on the ground plane along +x, zero pressure */
void orc_init_state(const orc_batch* b, orc_state* s);

/* command of every module of snake range [s0,s1) for the snake's step */
void orc_commands(const orc_batch* b, orc_state* s, int32_t s0, int32_t s1);

/* advance snakes [s0,s1) by n_steps steps (commands from the controller,
 * or the values already in cmd for the external controller) */
int orc_run(const orc_batch* b, orc_state* s, int32_t s0, int32_t s1, int32_t n_steps);

/* Dense linearised system of one snake at configuration (x,q) with previous
 * positions xp and chamber pressures p (row-major):
 *   C[rows], J[rows][6B] (columns x_i then rotation vector theta_i, world),
 *   W[6B][6B] inverse mass, comp[rows] = alpha~ per row.
 * rows = 6(B-1) joint rows + 3B contact rows (if ground).  Returns rows. */
int orc_assemble(const orc_batch* b, int32_t snake, const double* x, const double* q,
                 const double* xp, const double* p, double* C, double* J, double* W,
                 double* comp);

/* The same for a wheel-carriage batch: x, q, xp, qp hold the snake's B
 * segments followed by its 2B wheels (start-of-substep pose xp, qp, which
 * anchors the wheels' friction rows); columns 6 per body in that order;
 * rows 3 per block in block order (joints, then per wheel: hinge position,
 * hinge axis with its free spin row all zero, contact if ground). */
int orc_assemble_wheels(const orc_batch* b, int32_t snake, const double* x, const double* q,
                        const double* xp, const double* qp, const double* p, double* C, double* J,
                        double* W, double* comp);

/* stages of one substep of one snake, exposed for tests (for a wheel-carriage
 * batch the arrays hold the snake's B segments followed by its 2B wheels) */
void orc_predict_snake(const orc_batch* b, int32_t snake, double* x, double* q, double* v,
                       double* w, double h);

/* split substep: command effects on pressure and prediction, then the solve
 * (the plain chain only: both return at once for a wheel-carriage batch) */
void orc_pre_substep(const orc_batch* b, int32_t snake, int32_t sub, const double* x, const double* q,
                     double* v, double* w, double* p, const double* cmd, double* q_pred);
void orc_solve_substep(const orc_batch* b, int32_t snake, double* x, double* q, const double* q_pred,
                       double* v, double* w, const double* p, double* lam_j, double* lam_c,
                       double* residual, int32_t* iters, int32_t* status);

/* network inputs [2(B-1)][32] and targets [2(B-1)][3] of one snake */
void orc_features(const orc_batch* b, int32_t snake, const double* x, const double* v, const double* w,
                  const double* q_pred, const double* p, const double* cmd, const double* lam_j,
                  const double* lam_c, double* feat);
void orc_targets(const orc_batch* b, int32_t snake, const double* q_pred, const double* lam_j, double* tgt);

/* index work: per block type (0 stretch, 1 bend-twist, 2 contact), bodies,
 * greedy colour; per body degree; per snake bucket; work order. */
void orc_index(const orc_batch* b, int32_t* blk_type, int32_t* blk_a, int32_t* blk_b,
               int32_t* blk_color, int32_t* body_degree, int32_t* bucket, int32_t* order);

#endif
