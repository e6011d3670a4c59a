// Device-side pieces of a tempering stage captured whole into one graph: the random counters of
// the resampling uniform and of the mixture seeding read from device memory, and the end-of-stage
// rule (acceptance rate, step size, record, parking) on the device.
#pragma once
#include "common.hpp"

namespace smc {

// Counter block of the resampling uniform (the host's smc_philox_u53 draws from the same block).
constexpr uint32_t RESAMPLE_BLOCK = 0x80000001u;

// Systematic resampling whose uniform is drawn on the device from (seed, *ctr + ctr_off).
hipError_t launch_resample_ctr(int64_t N, const double* W, uint64_t seed, const uint64_t* ctr, uint64_t ctr_off,
                               int32_t* idx, int32_t* flags, hipStream_t s);
// The mixture fit with its seeding counter *ctr + ctr_off read on the device.
hipError_t launch_gm_fit_ctr(int64_t N, int K, int kr, const int32_t* active, const double* xi, int M, int iters,
                             double var_floor, uint64_t seed, const uint64_t* ctr, uint64_t ctr_off,
                             const FitWorkspace& w, int32_t* centers, double* logw, double* mean, double* scale,
                             hipStream_t s);

// End of a stage of G samplers (group g owns rows [off_g, off_g + count_g)).
struct StageRule {
    int32_t G = 0;
    int64_t off[MAX_LEVELS] = {}, count[MAX_LEVELS] = {};
    int32_t n_moves = 0;
    const int32_t* n_acc = nullptr;
    const double* tau = nullptr;
    const double* h = nullptr;
    const double* log_z = nullptr;
    double* beta = nullptr;
    int32_t* level = nullptr;     // null: one group, always running
    uint64_t* ctr = nullptr;
    uint64_t stride = 0;
    double* record = nullptr;     // [max_stages][G][5]
    int32_t max_stages = 0;
};
hipError_t launch_stage_rule(const StageRule& r, hipStream_t s);

}  // namespace smc
