// Host helpers shared by the entry points.
#pragma once
#include "dcstedc.h"
#include <hip/hip_runtime.h>

#include <cstddef>

dc_opts dc_resolve_opts(const dc_opts* opt);
hipError_t dc_fill_int(int* p, int n, int v, hipStream_t s);
// Copies nbytes (<= 1024) from host memory into device memory through a
// kernel argument (graph-safe, no host pointer is retained).
hipError_t dc_write_blob(void* dst, const void* src, int nbytes, hipStream_t s);
// Library-owned status word of a stream (created on first use).
hipError_t dc_status_word(hipStream_t s, int** out);
