// Table of autotuned launch shapes (host code; see tune_table.hip).
#pragma once

#include <string>

namespace sm {

// Hash of the sources the library was built from (set by the build).
const char* build_id();
// Replaces the table with the entries of the tuner's cache file that were
// tuned on this build; on any error the table is unchanged and err says why.
bool tune_load(const char* path, int* kept, std::string* err);
void tune_clear();
int tune_entries();
// Lane counts a kernel family launches with: 1, 4, 8, 16 or 64 lanes per
// sightline (the batch kernels: 1, 4, 16 or 64).
bool lanes_valid(long long kernel, long long lanes);
// Lanes per sightline and grid read mode (0: none) tuned for this exact shape
// on the current device, if the table holds one.
bool tune_lookup(int kernel, int kind, long long npix, long long steps, long long freqs,
                 int* lanes, int* grid_mode);

}  // namespace sm
