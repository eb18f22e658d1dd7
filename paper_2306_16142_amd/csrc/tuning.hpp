// Current value of a launch-shape knob (DDF_TUNE_* in ddf.h).
#pragma once

namespace ddf {
int tuning(int knob);
}
