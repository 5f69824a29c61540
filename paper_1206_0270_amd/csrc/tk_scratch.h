// Static device scratch area (tk_scratch.hip), host side.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>

namespace tk {

// Size of the static scratch array on each device: 64 MiB.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchMaxDevices = 64;

// Device address of the scratch array on `device`, looked up (with that
// device current) on the first call per device and cached.
hipError_t scratch_area(int device, void **ptr);

// Held by a user of the array for the whole use: calls that would overlap on
// one process's devices are serialised (other processes have arrays of their
// own).
std::mutex &scratch_user_lock();

}  // namespace tk
