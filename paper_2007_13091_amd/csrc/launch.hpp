// Host-callable launchers of the UGKWP kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace ugkwp {

// scan partial slots needed for an exclusive scan over n integers
long long scan_partials_needed(long long n);

// measurement hook: called around each group of launches of a step (no-op by default)
enum ProfSlot : int {
    kSlotPrim = 0,      // k_prim_dt
    kSlotCellPrep,      // k_cell_prep
    kSlotScan,          // scan of N_sam, capacity check, clearing of the bucket counters
    kSlotFlux,          // k_flux
    kSlotSample,        // k_sample
    kSlotStream,        // k_stream
    kSlotStreamWall,    // k_stream_wall (diffuse re-emissions queued by k_stream)
    kSlotCount,         // k_count
    kSlotScan2,         // scan of the bucket counts
    kSlotScatter,       // k_scatter
    kSlotGather,        // k_gather
    kSlotFinal,         // k_finalize (and the averaging kernels when averaging is on)
    kNumSlots
};
struct Prof {
    virtual ~Prof() {}
    virtual void begin(int) {}
    virtual void end(int) {}
};

// launch shapes of the kernels whose shape is tunable; every choice gives the same results
struct LaunchCfg {
    int stream_bs = 256;  // k_stream block size: 128, 256 or 512
    int stream_ilp = 1;   // k_stream particles per thread: 1 or 2
    int sample_wpb = 4;   // k_sample waves (cells) per block: 1, 2, 4 or 8
    int flux_bs = 128;    // k_flux block size: 64, 128 or 256
};
bool launch_cfg_valid(const LaunchCfg &c);

void launch_fill_i32(int32_t *p, long long n, int32_t v, hipStream_t s);
void launch_fill_f64(double *p, long long n, double v, hipStream_t s);
// one full time step on stream s; particles are read from pa[buf] and left in pa[buf ^ 1]
void launch_step(const Dev &D, int buf, const LaunchCfg &cfg, hipStream_t s, Prof *pr);
// a wave-only step when no particle exists anywhere (the same results as launch_step)
void launch_step_wave_only(const Dev &D, int buf, const LaunchCfg &cfg, hipStream_t s, Prof *pr);
// Shakhov model: each cell's heat flux from the particles in pa[buf] (after the state is set;
// the gather keeps it up to date from then on)
void launch_heat(const Dev &D, int buf, hipStream_t s);
// [nc][5] field (0 W, 1 W^p, 2 W^h, 3 primitives) into device memory out
void launch_moments(const Dev &D, int which, double *out, hipStream_t s);
// Wbar = A / D of the time averaging, [nc][5] in out
void launch_avg_out(const Dev &D, double *out, hipStream_t s);

}  // namespace ugkwp
