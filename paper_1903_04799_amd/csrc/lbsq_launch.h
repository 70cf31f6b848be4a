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
};

// Everything one time step t needs.  Buffers with _cur hold time t, those
// with _nxt receive time t+1 (populations, owners, body table).  Force sums:
// acc_cur collects this step's momentum exchange (and already holds the
// conversion force of the previous move), acc_conv receives the conversion
// force of this move, acc_clear is zeroed for the step after next.
struct StepLaunch {
    StepArgs args;
    const void *A;  // populations of time t
    void *B;        // receives time t+1
    const uint8_t *own_cur;
    uint8_t *own_nxt;
    const DevBody *bodies_cur;
    DevBody *bodies_nxt;
    int nbody;
    const int *all_ids, *all_start;  // every body and the block ranges of its box
    const int *mov_ids, *mov_start;  // moving bodies and theirs
    int nblk_all, nmov, nblk_mov;  // blocks of CPB cells
    unsigned long long *acc_cur, *acc_conv, *acc_clear;  // integer sum sets, ACCSET_SIZE each
    double *audit_part, *audit_out;
    int *err;
    double wca_sigma, wca_eps;
    bool audit;
    hipEvent_t ev_start, ev_stop;  // optional timing of the streaming kernel
    hipStream_t stream;
};

hipError_t launch_step(int storage, const StepLaunch &L);
hipError_t launch_classify(const Box &bx, uint8_t *own, hipStream_t s);
hipError_t launch_body_cells(const Box &bx, const DevBody *bodies, int b, int side, uint8_t *own, int check,
                             int *err, hipStream_t s);
hipError_t launch_audit(int storage, const StepArgs &a, const void *A, const uint8_t *own, double *part,
                        double *out, int *err, hipStream_t s);
hipError_t launch_fields(int storage, const StepArgs &a, const void *A, const uint8_t *own, double *rho, double *u,
                         uint8_t *own_out, hipStream_t s);
hipError_t launch_plane(int storage, const StepArgs &a, void *A, const uint8_t *own, int i, double *buf, int to_f64,
                        hipStream_t s);
hipError_t launch_link_mask(const Box &bx, const uint8_t *own, uint32_t *mask, hipStream_t s);

}  // namespace lbsq
