// passes.h -- host-side launchers for the per-precision pass kernels.  Each launcher
// maps a runtime axis length to the compiled plan for it; unsupported lengths return
// kUnsupported without launching anything.
//
// Pass order of one step: x forward (R2C split, rows), z forward (C2C, single component),
// fused y (forward, propagator, invariant partials, inverse; all six components),
// z inverse (with the invariant finalize), x inverse (C2R merge); between two steps the
// x inverse and the next x forward run as one kernel.  Grids whose (y, z) plane fits in
// LDS run the three middle passes as one plane pass.  The fused pass runs along y
// because its pencils are then M complex elements apart, while the strided z axis is
// handled by the single-component pass, which can use wide tiles.
//
// Every launcher advances a batch of nm members of one shape; md is a device array of
// nm member descriptors (see kernels.h).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace eifp {

enum LaunchRc { kOk = 0, kUnsupported = 2, kLaunchFailed = 4 };
enum Axis { AXIS_Y = 1, AXIS_Z = 2 };

// Geometry of the state: nx reals per row, M = nx/2 complex per row.
struct Grid3 {
    int nx, ny, nz, M;
    long cs() const { return (long)nz * ny * M; }  // complex elements per component
};

// x pass: X_FWD (state -> work), X_INV (work -> state), or X_INVFWD (between two steps
// with work != state: the inverse and the next step's forward, in place on work)
enum XKind { X_FWD = 0, X_INV = 1, X_INVFWD = 2 };
// fin_nparts > 0 (X_INV and X_INVFWD only): one extra workgroup per member also
// finalizes that many invariant partial records (those of a preceding plane pass)
template <typename T>
int launch_x(int kind, const Grid3& g, const void* md, int nm, const void* twx, hipStream_t st, int fin_nparts = 0);

// Small grids: the plane pass (z forward, y forward, propagator and invariant partials,
// y inverse, z inverse) of one step, one workgroup per packed x column, whose (Ny, Nz)
// plane of the six components is held in LDS; it writes g.M partial records per member
// (want_inv), which the x kernel after it finalizes.  plane_ok: the grid has a compiled
// plane pass (kUnsupported from launch_plane otherwise).
template <typename T>
bool plane_ok(const Grid3& g);
template <typename T>
int launch_plane(const Grid3& g, const void* md, int nm, const void* twy, const void* twz, int want_inv,
                 hipStream_t st);

// single-component C2C along y or z on each member's work buffer (six components, in
// place); fin_nparts > 0 also finalizes each member's invariant partials (that many
// records) in one extra workgroup per member, alongside the transform.  comp_desc: a
// forward pass takes the components in descending order (after X_FWD; ascending after
// X_INVFWD)
template <typename T>
int launch_c2c(bool inv, int axis, const Grid3& g, const void* md, int nm, const void* tw, hipStream_t st,
               int fin_nparts = 0, int comp_desc = 1);

// fused pass along `axis` on each member's work buffer: mode Z_STEP (forward, propagate,
// partials, inverse, store), Z_FORWARD (forward, partials only; memory untouched),
// Z_FORWARD_EXT (the same with the extended invariant record) or Z_JUMP (read the
// member's anchored spectrum, propagate, partials, inverse into work)
template <typename T>
int launch_fused(int mode, int axis, const Grid3& g, const void* md, int nm, const void* tw, int want_inv,
                 hipStream_t st);

// number of partial records the fused pass writes per member (-1: unsupported length)
template <typename T>
int fused_partial_count(int axis, const Grid3& g);

// finalize each member's partials into its invariant record (extended: the INV_XPART-value
// record of Z_FORWARD_EXT)
template <typename T>
int launch_finalize(const void* md, int nm, int nparts, hipStream_t st, bool extended = false);

}  // namespace eifp
