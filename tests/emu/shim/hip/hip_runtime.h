// CPU stand-in for <hip/hip_runtime.h>, for building the evaluation code of
// the HIP kernels as host code under the wave64 emulator (wave_emu.h). Only
// what the shared evaluation code and the internal header use is provided.
#pragma once
#include "../../wave_emu.h"
