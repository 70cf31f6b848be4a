// lbsq_sim.h -- the simulation handle of the C ABI, shared by the
// single-simulation calls and the batching server.
#pragma once

#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/lbsq.h"
#include "lbsq_launch.h"

// A roctx range over a host-side phase of the API (stepping, set-up,
// readout, the server's admission and chunks), visible in a profiler's
// marker trace; without a profiler it costs a call.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

struct lb_sim {
    lb_params p;
    int device = 0;
    hipStream_t stream = nullptr;
    lbsq::StepArgs args{};
    size_t esize = 4;
    // populations in place (one buffer); owners and bodies double-buffered,
    // index cur holding the current time level; link densities of the
    // previous and current step
    void *f = nullptr;
    void *f2 = nullptr;  // the second buffer of the pull layout (LB_LAYOUT_AB)
    float *d_dens[2] = {nullptr, nullptr};
    uint8_t *own[2] = {nullptr, nullptr};
    lbsq::DevBody *d_bodies[2] = {nullptr, nullptr};
    int cur = 0;  // always steps & 1
    lbsq::SimDesc *d_desc = nullptr;  // the step kernels' view of this simulation
    lbsq::SimDesc *d_batch_desc = nullptr;  // MAXSIM descriptors for lb_step_batch led by this handle
    std::vector<lbsq::DevBody> bodies;
    int *d_lists = nullptr;  // mov_ids | mov_start | all_ids | all_start | all_base | all_count
    uint32_t *d_shell = nullptr;  // packed shell-cell offsets of every body
    uint32_t *d_wmask = nullptr;  // static-wall bits of each cell's sources (only with static walls)
    uint32_t *d_sgrp = nullptr;   // groups of 256 cells holding a non-wall cell (only with static walls)
    uint32_t nsgrp = 0;
    size_t shell_cap = 0;
    int4 *d_blkinfo = nullptr;  // per boundary block: body, first shell cell, cells, list position
    size_t blkinfo_cap = 0;
    int nmov = 0, nblk_mov = 0, nblk_all = 0;
    unsigned long long *d_acc = nullptr;  // NACCSET sets of ACCSET_SIZE integer sums
    size_t audit_blocks = 0;
    double *d_audit_part = nullptr, *d_audit_out = nullptr;
    int *d_err = nullptr;
    int64_t steps = 0;
    bool started = false, need_classify = true;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
    double ms = 0.0;
    int64_t launches = 0;
};

// The step kernels' descriptor of simulation s for time levels t = t0 + k.
void lbsq_fill_desc(const lb_sim *s, int64_t t0, int64_t t_end, lbsq::SimDesc &d);
// Blocks of the fluid and geometry launches of simulation s.
void lbsq_sim_blocks(const lb_sim *s, uint32_t *fluid, uint32_t *geo);
// Pending owner flags computed; the handle counts as started.
int lbsq_prepare(lb_sim *s);
// Device memory through the handle's allocator.
void *lbsq_dev_alloc(lb_sim *s, size_t bytes);
void lbsq_dev_free(lb_sim *s, void *p);
// Stream synchronised and device error flags turned into a status.
int lbsq_sync_check(lb_sim *s);
// The buffer holding the populations after the steps taken so far, and its
// layout (LAY_*), for the readout kernels.
const void *lbsq_pop_buf(const lb_sim *s);
int lbsq_pop_lay(const lb_sim *s);
// Device address of this GPU's no-allocation scratch array, looked up once
// per device with that device current (lbsq_noalloc.hip).
int lbsq_noalloc_init(int device);
