// Host stand-in for hip_ext.h: nothing beyond the runtime stand-in is used
// by the host code built against it.
#pragma once
#include "hip_runtime.h"
