// Launch-shape knobs of the C ABI (ddf_set_tuning / ddf_get_tuning).  They change how work
// is spread over the GPU, never a result; the autotuner times their candidates.
#include <atomic>

#include "common.hpp"
#include "tuning.hpp"

namespace ddf {
namespace {

std::atomic<int> g_knob[DDF_TUNE_COUNT] = {{2}, {2048}, {2}};

bool valid(int knob, int v) {
    switch (knob) {
        case DDF_TUNE_STREAM_WG_PER_CU: return v == 1 || v == 2;
        case DDF_TUNE_CULL_RAYS_PER_BLOCK: return v >= 256 && v <= 16384 && (v & (v - 1)) == 0;
        case DDF_TUNE_GRAD_WG_PER_CU: return v == 1 || v == 2 || v == 4;
        default: return false;
    }
}

}  // namespace

int tuning(int knob) { return g_knob[knob].load(std::memory_order_relaxed); }

}  // namespace ddf

extern "C" ddf_status ddf_set_tuning(int32_t knob, int32_t value) {
    DDF_REQUIRE(knob >= 0 && knob < DDF_TUNE_COUNT, DDF_ERR_INVALID_ARG, "ddf_set_tuning: unknown knob %d", knob);
    DDF_REQUIRE(ddf::valid(knob, value), DDF_ERR_INVALID_ARG, "ddf_set_tuning: value %d not allowed for knob %d", value,
                knob);
    ddf::g_knob[knob].store(value, std::memory_order_relaxed);
    return DDF_OK;
}

extern "C" ddf_status ddf_get_tuning(int32_t knob, int32_t *value) {
    DDF_REQUIRE(knob >= 0 && knob < DDF_TUNE_COUNT && value, DDF_ERR_INVALID_ARG, "ddf_get_tuning: bad argument");
    *value = ddf::tuning(knob);
    return DDF_OK;
}
