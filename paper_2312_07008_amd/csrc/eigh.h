// Internal interface of the FP64 symmetric eigensolver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "host.h"

namespace dfpt2 {

constexpr int kEighMaxN = 16384;

size_t eigh_workspace_bytes(int n);
// w_out [n] and Z_out [n][n] (column k = eigenvector of w_out[k]); ascending, or
// descending when `descending` is set.  With vec_floor_rel > 0 only eigenvalues
// above vec_floor_rel * max|w| get eigenvectors (the other columns are zero).
// Synchronizes the stream.
int eigh_run(const double* A, int n, double* w_out, double* Z_out, char* ws, size_t ws_bytes, hipStream_t st,
             int descending, double vec_floor_rel = -1.0);

}  // namespace dfpt2
