// lbsq_launch.h -- host-side launch interface between the C ABI and the
// gfx950 kernels of the lattice Boltzmann squirmer library.
#pragma once

#include "lbsq_device.h"

namespace lbsq {

// Scalars every kernel of a step needs (FP32 for the collision, FP64 where
// the force and refill arithmetic runs in double).
struct StepArgs {
    Box box;
    float lam_e, lam_o, rho0;
    float g[3];
    float scale, inv_scale;  // 2^k and 2^-k of the stored deviations
    double rho0d;
    // Constants of the bulk collision, which works on the deviations as
    // stored: s is the storage scale (2^k in the half-width forms, 1 in FP32)
    // and w_k the weight of the rest (k = 0), axis (1) and diagonal (2)
    // directions.
    float c_lew[3];     // lam_e w_k
    float c_lews[3];    // lam_e w_k s
    float c_low3s[3];   // 3 lam_o w_k s
    float c_k1, c_k2;   // (1 - lam_e) / 2, (1 - lam_o) / 2
    float c_1mle;       // 1 - lam_e
    float c_s, c_is;    // s, 1 / s
};

// Most simulations one batched launch can take.
constexpr int MAXSIM = 64;

// One simulation as the step kernels see it.  The kernels of step k of a
// launch sequence advance time level t = t0 + k: populations in place in f
// (streaming direction by the parity of t), owners and bodies read from
// [t & 1] and written to [(t & 1) ^ 1], link densities read from dens[(t & 1)
// ^ 1] and written to dens[t & 1]; steps with t >= t_end are skipped.
// Force sums: set t % 3 collects step t's momentum exchange (and already
// holds the conversion force of the previous move), set (t+1) % 3 receives
// the conversion force of this move, set (t+2) % 3 is zeroed.
struct SimDesc {
    StepArgs a;
    void *f;   // the population buffer (the first of two in the pull layout)
    void *f2;  // the second buffer of the two-buffer pull layout; null in place
    float *dens[2];
    uint8_t *own[2];
    DevBody *bodies[2];
    unsigned long long *acc;  // NACCSET sets of ACCSET_SIZE integers
    const int *mov_ids, *mov_start;  // moving bodies and the block ranges of their boxes
    const int *all_ids, *all_start;  // every body and the block ranges of its shell cells
    const int *all_base, *all_count;  // where each body's shell cells sit in shell, and how many
    const uint32_t *shell;            // packed offsets relative to the floor of the body position
    const uint32_t *wmask;            // per cell: bit i set when x - c_i is a static wall (null: no walls)
    const uint32_t *sgrp;             // the groups of BLOCK cells holding a non-wall cell (null: every group)
    const int4 *blkinfo;              // per boundary block: body, first shell cell, cells, list position
    double *audit_part;
    int *err;
    unsigned int *arrive;  // arrival counter of the boundary blocks, zero between launches
    double wca_sigma, wca_eps;
    int64_t t0, t_end;
    int nbody, nmov;
    int nblk_b, nblk_s;  // boundary and streaming blocks of the fluid launch
};

// Block ranges of the simulations of a batched launch: simulation j owns
// blocks [fluid0[j], fluid0[j+1]) of the fluid launch and [geo0[j],
// geo0[j+1]) of the geometry launch.
struct BatchMap {
    int nsim;
    uint32_t fluid0[MAXSIM + 1];
    uint32_t geo0[MAXSIM + 1];
};

// One step of a batch: the fluid launch (which also updates the bodies of
// simulations with at most FUSE_MAX bodies), then (one simulation only) the
// audit reduction and the one-block body update for more bodies, then the
// geometry launch.
struct BatchLaunch {
    const SimDesc *desc;  // device array of map.nsim descriptors
    BatchMap map;
    int64_t k;
    int nbody_max;        // most bodies of any simulation (LDS size)
    bool force;           // a body force g is set (one simulation only)
    bool audit;           // fused audit (one simulation only)
    double *audit_part, *audit_out;
    int npart;
    int *err;
    bool body_kernel;     // body update by k_body (one simulation only)
    hipEvent_t ev_start, ev_stop;  // optional timing of the fluid launch
    hipStream_t stream;
};

// Geometry blocks of a simulation: those of the moving bodies' boxes (the
// body update itself runs in the fluid launch, or in k_body for more than
// FUSE_MAX bodies).
inline int geo_blocks(int nbody, int nblk_mov)
{
    return nbody == 0 ? 0 : nblk_mov;
}

hipError_t launch_batch_step(int storage, const BatchLaunch &L);
// Owner flags of the fluid cells (set_flags) and, if wmask is given, each
// cell's static-wall mask.
hipError_t launch_classify(const Box &bx, uint8_t *own, uint32_t *wmask, int set_flags, hipStream_t s);
hipError_t launch_body_cells(const Box &bx, const DevBody *bodies, int b, int side, uint8_t *own, int check,
                             int *err, hipStream_t s);
// Readouts of the state after a completed step: A is the buffer holding it
// and lay its layout (LAY_AA_ODD / LAY_AA_EVEN: in place, after an odd or
// even step; LAY_AB: the buffer the last step of the pull layout wrote).
hipError_t launch_audit(int storage, const StepArgs &a, const void *A, const uint8_t *own, int lay,
                        double *part, double *out, int *err, hipStream_t s);
// Fields of cells [c0, c0 + cnt) into rho[cnt], u[3][cnt] and own_out[cnt].
hipError_t launch_fields(int storage, const StepArgs &a, const void *A, const uint8_t *own, int lay, uint32_t c0,
                         uint32_t cnt, double *rho, double *u, uint8_t *own_out, hipStream_t s);
hipError_t launch_plane(int storage, const StepArgs &a, void *A, const uint8_t *own, int lay, int i,
                        double *buf, int to_f64, hipStream_t s);
hipError_t launch_dens(int storage, const StepArgs &a, const void *A, const uint8_t *own, int lay, float *dens,
                       hipStream_t s);
hipError_t launch_link_mask(const Box &bx, const uint8_t *own, uint32_t *mask, hipStream_t s);

}  // namespace lbsq
