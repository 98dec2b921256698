// passes.h -- host-side launchers for the per-precision pass kernels.  Each launcher
// maps a runtime axis length to the compiled plan for it; unsupported lengths return
// kUnsupported without launching anything.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace eifp {

enum LaunchRc { kOk = 0, kUnsupported = 2, kLaunchFailed = 4 };

// Supported axis lengths: 2^a 3^b between 4 and 512 whose plans are compiled below.
bool supported_axis(int n);

template <typename T>
int launch_x(bool inv, int nx, const void* src, void* dst, long nrows, const void* twx, hipStream_t st);

template <typename T>
int launch_y(bool inv, int ny, void* buf, int M, int nz, const void* twy, hipStream_t st);

// mode: Z_STEP (forward, propagate, partials, inverse) or Z_FORWARD (partials only).
// *nparts receives the number of partial records written when want_inv != 0.
template <typename T>
int launch_z(int mode, int nz, void* buf, int M, int ny, long comp_stride, const void* twz, const PropParams& pp,
             double* partials, int want_inv, hipStream_t st);

template <typename T>
int z_partial_count(int nz, int M, int ny);

template <typename T>
int launch_z_fwd_store(int nz, void* buf, int M, int ny, long comp_stride, const void* twz, hipStream_t st);

}  // namespace eifp
