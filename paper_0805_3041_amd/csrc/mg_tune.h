// Autotuning support (mg_tune.hip): the persistent cache of tuned launch
// choices and the device facts the choices depend on.
#pragma once

#include <string>

namespace mg {

// Identity of the running device and of the kernel sources: "<gcn arch>|<source digest>".
std::string tune_identity();

// Tuned value stored under `key` (empty string: none).  The cache is a JSON
// object of string pairs in the file named by MG_TUNE_CACHE, or in
// libmg_tune.json beside the library; MG_TUNE_CACHE=off disables it.
std::string tune_lookup(const std::string& key);
void tune_store(const std::string& key, const std::string& value);

// Compute units of the current device (hipDeviceProp multiProcessorCount).
int device_cus();

}  // namespace mg
