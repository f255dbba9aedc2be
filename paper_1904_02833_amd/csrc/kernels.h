// Kernel parameter block and launch wrappers shared by the HIP translation
// units of the snake solver.  Host-visible; no torch types.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snake {

enum : int { kFixedRoot = 1, kNoGround = 2 };
enum : int { kLawLag = 0, kLawPaper = 1 };
enum : int { kCtrlExternal = 0, kCtrlSerpenoid = 1, kCtrlSchedule = 2 };
enum : int { kWarmZero = 0, kWarmPrev = 1, kWarmMlp = 2 };
enum : int { kStatusNonfinite = 1, kStatusNotConverged = 2, kStatusFellBack = 4 };
// kPhaseFull runs whole steps; a split substep is kPhasePre (command,
// pressure, prediction into q_pred) followed by kPhaseSolve (multiplier
// initialisation, iterations, velocities).
enum : int { kPhaseFull = 0, kPhasePre = 1, kPhaseSolve = 2 };

// Everything one step kernel needs.  Device pointers into the workspace,
// structure-of-arrays (component k of body i at [k * N + i]).
struct KParams {
    int n_snakes, N, J, Mt;
    // per snake
    const int* Bn;
    const int* Mn;
    const int* Sn;
    const int* body_off;
    const int* joint_off;
    const int* module_off;
    const float* comp;      // [3][n]: stretch, bend, twist compliance / h^2
    const float* mu;        // [n]
    const double* freq;     // [n]
    const double* phase0;   // [n]
    const int* sched_off;   // [Mt+1]
    const int* sched_start; // [pieces] first step of each piece
    const float* sched_val; // [pieces]
    // state
    float* x;
    float* q;
    float* v;
    float* w;
    float* p;               // [2][Mt]
    float* cmd;             // [Mt]
    float* lam_j;           // [6][J]
    float* lam_c;           // [3][N]
    float* q_pred;          // [4][N] predicted orientation (split substeps)
    float* probe;           // [16][N] zero start's iterate K (fallback after K iterations)
    const float* mlp_y;     // [2J][3] network outputs (learned warm start)
    float* residual;        // [n]
    int* iters_out;         // [n]
    int* status;            // [n]
    long long* step;        // [n]
    long long* iters_total; // [n]
    // constants
    float h, inv_h, inv_m, L, half_L, inv_L, R, g;
    float c1, c2;           // 1/I_perp and 1/I_axis - 1/I_perp
    float I_ax, I_pe;
    float tol, relax;
    int iters, substeps;
    float lag_in, lag_de;   // exp(-h / tau)
    int law;
    float k_i, k_d, T_p, p_s, amp, kappa_max;
    int controller;
    double dt, ctrl_alpha, ctrl_offset;
    int flags, warm, fallback, fallback_k;
    float lam_ref;          // multiplier scale m 9.81 h^2 of the network units
};

// Constants of the Newton solver kernel, which computes in double: the
// body constants again at full precision, per-snake compliances / h^2 and
// the iteration budget.
struct NParams {
    const double* comp;     // [3][n]: stretch, bend, twist compliance / h^2
    const double* mu;       // [n]
    double h, m, L, R, g, I_ax, I_pe, tol;
    double lag_in, lag_de;  // exp(-h / tau)
    double amp, p_s, k_i, k_d, T_p, kappa_max;
    int newton_iters, pcr_iters;
    int keep_best;          // end at the evaluated iterate of smallest residual
};

// Index-work parameters.
struct IParams {
    int n_snakes, N, n_blocks, ground;
    const int* Bn;
    const int* Mn;
    int* body_off;
    int* joint_off;
    int* module_off;
    int* block_off;
    int* blk_type;
    int* blk_a;
    int* blk_b;
    int* blk_color;
    int* degree;
    int* bucket;
    int* order;
    int* color_scratch;     // [N]
};

// Solver launch: workgroups of nw waves over n_tiles tiles (grid-stride
// when grid < n_tiles), aligned power-of-two layout or (rows = 1) segments
// of whole 16-lane rows placed without alignment.
// hdr[t] = {first slot, slots, some segment crosses a wave boundary, rows};
// slot = {snake, lane offset << 16 | segment lanes}.
hipError_t launch_tiles(int nw, int rows, const KParams& P, const int4* hdr, const int2* slots,
                        int n_tiles, int grid, int n_steps, int phase, int sub, hipStream_t stream);
// Newton solver: one launch per class of snakes whose lane count (the
// power of two >= B, at least 8) is 8 << c; list holds the snakes class by
// class, class c at [off[c], off[c+1]), c < 8.  Runs n_steps whole steps.
hipError_t launch_newton(const KParams& P, const NParams& Q, const int* list, const int* off,
                         int n_steps, hipStream_t stream);
// Block Gauss-Seidel solver, same lane classes and snake list as the Newton
// solver; colours from the index work (block_off, blk_color).
hipError_t launch_gs(const KParams& P, const int* block_off, const int* blk_color, const int* list,
                     const int* off, int n_steps, hipStream_t stream);
hipError_t launch_features(const KParams& P, float* feat, hipStream_t stream);
hipError_t launch_targets(const KParams& P, float* tgt, hipStream_t stream);
// network outputs of the learned start from the predicted state, inputs
// computed in the kernel (mlp.hip)
hipError_t launch_warm_net(const KParams& P, const float* params, const float* mean_std, float* y,
                           hipStream_t stream);
hipError_t launch_index(const IParams& P, hipStream_t stream);
hipError_t launch_init_state(const KParams& P, hipStream_t stream);
hipError_t launch_set_cmd(float* dst, const float* src, int n, hipStream_t stream);

}  // namespace snake
