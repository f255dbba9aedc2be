/*
 * link.h - C ABI of the full-resolution soft-link solver for AMD Instinct
 * MI355X (gfx950).
 *
 * A batch of snakes built from soft links (Gasoto, Macklin et al., "A
 * Validated Physical Model For Real-Time Simulation of Soft Robotic
 * Snakes"): every snake is n_links links joined end to end by n_links + 1
 * rigid frames.  A link is a tetrahedral particle mesh given in
 * cross-sections along the link (section "Soft robotic snake model": a
 * radially symmetric mesh of 13 cross-sections); its particles carry lumped
 * masses (section "Particles": each particle a quarter of every element it
 * belongs to).  Constraints, all of the form c + E lambda = 0 (section
 * "Simulator"):
 *   - every tetrahedron: the six corotational constant-strain components in
 *     Voigt order (xx, yy, zz, yz, xz, xy; tensor shear strains), rotation
 *     from the polar decomposition of the deformation gradient at the
 *     current iterate and held in the Jacobian, compliance
 *     E_tetra = M / (V Y) with M = [1 -nu -nu; -nu 1 -nu; -nu -nu 1] on the
 *     normal strains and 1 + nu on the shear strains (section "Tetrahedral
 *     Finite-Elements");
 *   - distance constraints |x_i - x_j| - L = 0 along the link between the
 *     same slot of neighbouring cross-sections, and from the centre to the
 *     ring within every section but the two end ones: the centre slot and
 *     the ring slots in the plane y = 0 form the inextensible centre layer,
 *     the ring slots with y > 0 chamber 0 and y < 0 chamber 1 (section "Soft
 *     robotic snake model");
 *   - actuation (section "Actuation Constraints"): while a link's command
 *     selects chamber c (a > 0 chamber 0, a < 0 chamber 1) that chamber's
 *     axial rows take the rest length r (1 + P / Y) (eq. expansion), P =
 *     p_max times the chamber pressure (a fraction of full, lagging the
 *     command), and the other chamber's axial rows are absent (one chamber
 *     active at a time); with a = 0 neither chamber's rows act;
 *   - attachments of both end sections' particles to their frames,
 *     x_f + R(q_f) r - x_p = 0 (eq. rigid_to_particle), r the particle's
 *     rest position relative to the frame;
 *   - ground contact of every particle (z >= 0) with Coulomb friction.
 * The distance and attachment rows carry the compliance rigid_compliance.
 * One substep: chamber pressures by a first-order lag, prediction
 * (particles: gravity; frames: gravity and the gyroscopic term, section
 * "Time-Stepping"), then block-Jacobi iterations from zero multipliers:
 * every block takes its local solution -(K + E/h^2)^-1 (C + E/h^2 lambda),
 * K = J W J^T, scaled by relax / (the largest number of blocks on one of
 * its bodies), and every body gathers W J^T (scaled increment) in the
 * fixed block order (tetrahedra, distance rows, attachments, contact);
 * velocities from the displacement.  FP32 on the device.
 *
 * Conventions: SI units, world z up, ground z = 0; a link's mesh runs
 * along +x.  Device arrays are structure-of-arrays FP32: component k of
 * item i at [k * count + i].  Particle i of the batch is
 * (snake * n_links + link) * per_link + section * (ring + 1) + slot; frame
 * snake * (n_links + 1) + junction; tetrahedron (snake * n_links + link) *
 * n_tets + t; distance row (snake * n_links + link) * dist_per_link + d in
 * the order of link_read_index; attachment (snake * n_links + link) *
 * 2 (ring + 1) + a, section 0's slots then the last section's.  Calls are
 * asynchronous on the stream given to link_create unless said otherwise.
 * Return values: LINK_OK (0) or a negative error code; link_last_error()
 * gives the calling thread's last message.  No C++ exception crosses this
 * boundary.
 */
#ifndef LINK_H
#define LINK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LINK_OK 0
#define LINK_EINVAL (-1)  /* bad argument or descriptor                      */
#define LINK_ENOMEM (-2)  /* workspace smaller than link_workspace_bytes()    */
#define LINK_EDEVICE (-3) /* HIP runtime or launch failure                    */

#define LINK_MEM_HOST 0
#define LINK_MEM_DEVICE 1

#define LINK_FLAG_FIXED_FRAME0 1u /* frame 0 of every snake has infinite mass */
#define LINK_FLAG_NO_GROUND 2u    /* no ground plane, no contact blocks       */

#define LINK_STATUS_NONFINITE 1
#define LINK_STATUS_NOT_CONVERGED 2

/* state fields (bit k of `fields` selects dst[k] / src[k]) */
#define LINK_F_POS (1u << 0)           /* float [3][P] particle positions        */
#define LINK_F_VEL (1u << 1)           /* float [3][P]                            */
#define LINK_F_FRAME_POS (1u << 2)     /* float [3][F] frame centres              */
#define LINK_F_FRAME_QUAT (1u << 3)    /* float [4][F] (w, x, y, z), body to world */
#define LINK_F_FRAME_VEL (1u << 4)     /* float [3][F]                            */
#define LINK_F_FRAME_ANGVEL (1u << 5)  /* float [3][F] world frame                */
#define LINK_F_PRESSURE (1u << 6)      /* float [2][L] chamber pressures, fraction of full */
#define LINK_F_CMD (1u << 7)           /* float [L] held command per link         */
#define LINK_F_LAMBDA_TET (1u << 8)    /* float [6][T] last substep's multipliers */
#define LINK_F_LAMBDA_DIST (1u << 9)   /* float [D]                               */
#define LINK_F_LAMBDA_ATT (1u << 10)   /* float [3][A]                            */
#define LINK_F_LAMBDA_CONTACT (1u << 11) /* float [3][P] normal, tangential x, y  */
#define LINK_F_RESIDUAL (1u << 12)     /* float [n_snakes] largest over the last step's substeps */
#define LINK_F_ITERS (1u << 13)        /* int32 [n_snakes] iterations in the last step */
#define LINK_F_STATUS (1u << 14)       /* int32 [n_snakes] LINK_STATUS_* of the last step */
#define LINK_F_ITERS_TOTAL (1u << 15)  /* int32 [n_snakes] iterations since creation */
#define LINK_F_COUNT 16

/* index arrays of one snake (link_read_index; bit-exact index work) */
#define LINK_IDX_DIST_I 0       /* [D1] first particle of each distance row (snake-local) */
#define LINK_IDX_DIST_J 1       /* [D1] second particle                    */
#define LINK_IDX_DIST_KIND 2    /* [D1] 0 centre layer, 1 radial, 2 chamber 0, 3 chamber 1 */
#define LINK_IDX_DEG_PARTICLE 3 /* [P1] blocks touching each particle     */
#define LINK_IDX_DEG_FRAME 4    /* [F1] blocks touching each frame        */
#define LINK_IDX_COUNT 5

/* Descriptor (host memory, read by link_workspace_bytes and link_create
 * only; link_create copies what it needs). */
typedef struct link_desc {
    int32_t n_snakes;      /* >= 1                                            */
    int32_t n_links;       /* links per snake, 1..4                           */
    int32_t sections;      /* cross-sections per link, >= 3                   */
    int32_t ring;          /* ring particles per section, a multiple of 4, 4..28 */
    int32_t n_tets;        /* tetrahedra per link                             */
    const double* X;       /* [sections * (ring + 1)][3] rest positions in the */
                           /* link frame, section-major, centre first, ring    */
                           /* particle k at angle 2 pi k / ring; x in [0, length] */
    const int32_t* tets;   /* [n_tets][4] positively oriented, local indices  */
    const double* mu;      /* [n_snakes] friction coefficient                 */
    double link_length;    /* m, distance between a link's two frames         */
    double radius;         /* m; the link axis rests at z = radius            */
    double young, poisson, density; /* Pa, -, kg/m^3                          */
    double p_max;          /* Pa of a chamber at full pressure                */
    double frame_mass;     /* kg; a frame is a solid cylinder along x of       */
    double frame_length;   /* radius `radius` and this length (inertia only)   */
    double gravity, dt;
    int32_t substeps;      /* h = dt / substeps                               */
    int32_t iters;         /* iterations per substep (tol <= 0) or the maximum */
    double tol;            /* > 0: stop a substep at residual <= tol          */
    double relax;          /* (0, 1]                                          */
    double tau_inflate, tau_deflate; /* s, chamber lag                        */
    double rigid_compliance;         /* m/N, distance and attachment rows     */
    uint32_t flags;        /* LINK_FLAG_*                                     */
} link_desc_t;

typedef struct link link_t;

/* Workspace bytes for a descriptor: the state of section "Simulator" for
 * every particle (section "Particles") and frame (section "Rigid Bodies"),
 * one multiplier per constraint row, and the per-mesh constants.  Pure host
 * computation; LINK_EINVAL for an invalid descriptor. */
int link_workspace_bytes(const link_desc_t* d, size_t* bytes);

/* Build the solver in caller-owned device memory `workspace` (at least
 * link_workspace_bytes, kept alive until link_destroy) on stream
 * `hip_stream` (borrowed; NULL the default stream).  Builds the constraint
 * lists of section "Soft robotic snake model" on the host, computes the
 * per-mesh constants (lumped masses of section "Particles", element rest
 * shapes and the element blocks' (K + E/h^2)^-1, constant because the
 * rotation cancels from J W J^T) on the device, and sets every snake
 * straight at rest along +x with zero pressure and commands.  Synchronises
 * the stream.  Errors: LINK_EINVAL, LINK_ENOMEM, LINK_EDEVICE. */
int link_create(const link_desc_t* d, void* workspace, size_t bytes, void* hip_stream, link_t** out);

/* The commands whose chambers' pressures parameterise the actuation
 * constraints (section "Actuation Constraints", eq. expansion): one signed
 * command per link (n == n_snakes * n_links), clamped to [-1, 1], held
 * until the next call.  Host memory: NaN gives LINK_EINVAL; device memory:
 * NaN is read as 0.  Stream-ordered. */
int link_set_commands(link_t* s, const float* cmd, int64_t n, int mem);

/* Advance every snake by n_steps steps of the first-order implicit
 * discretisation of section "Time-Stepping" (substeps each, block-Jacobi
 * iterations on the compliant system whose linearisation is
 * eq. schur_system), asynchronously.  One workgroup per snake.  Launch
 * failures return LINK_EDEVICE; numerical failures are per-snake status
 * bits. */
int link_step(link_t* s, int32_t n_steps);

/* Read the state of section "Simulator" (particle positions, frame poses,
 * velocities, chamber pressures, the multipliers of every constraint row):
 * copy the selected LINK_F_* fields to dst[k].  Host memory: synchronises
 * the stream. */
int link_read_state(link_t* s, uint32_t fields, void* const* dst, int mem);

/* Overwrite the selected fields from src[k] (checkpoint restore and the
 * parity protocol's state injection); a round trip is bitwise.  Host
 * memory: synchronises the stream. */
int link_write_state(link_t* s, uint32_t fields, const void* const* src, int mem);

/* Copy index array `which` (LINK_IDX_*) of one snake (every snake has the
 * same) to host memory `dst` of `count` int32 (must equal its length).
 * Synchronous. */
int link_read_index(link_t* s, int32_t which, int32_t* dst, int64_t count);

/* The solver kernel's lane plan of the particles' gathers for a
 * descriptor, on the host (no device, no state), as link_create builds it.
 * A snake's workgroup has 1024 lanes; each particle of the snake owns an
 * aligned group of 1, 2, 4 or 8 lanes of one wave, whose lanes sum
 * consecutive ranges of the particle's incidence list (its blocks of
 * section "Soft robotic snake model" in the gather order: elements,
 * distance rows, attachment; a link's lists follow one another particle by
 * particle, 4 T1 + 2 D1 + A1 entries per link).  Caller host memory:
 *   out[lane] = particle | log2(group size) << 16, or -1 for no particle
 *   out[1024 + lane] = first | end << 16, the lane's range of entries
 *   (in its link's list)
 * and *gmax the largest group.  LINK_EINVAL for an invalid descriptor. */
int link_plan_gathers(const link_desc_t* d, int32_t* out2048, int32_t* gmax);

/* Sizes of the batch: n_snakes, P, F, T, D, A (totals) and L = links,
 * per snake P1, D1, A1 (host int64 out[10]). */
int link_sizes(const link_t* s, int64_t* out10);

/* Release host resources (the caller frees the workspace); NULL is a
 * no-op.  Waits for the stream. */
void link_destroy(link_t* s);

/* Message of the calling thread's last error ("" if none). */
const char* link_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LINK_H */
