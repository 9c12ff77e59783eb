// launch.hpp -- host-side launchers of the HIP kernels (library-internal).
#pragma once
#include <hip/hip_runtime_api.h>

#include "device.hpp"

namespace ibdvm {

// tile of the marching updates: V velocity nodes per lane, TX grid columns
// per workgroup (2D: a row of 4 or 8; 3D: a 4 x 4 or 4 x 2 tile, TX = 16 or
// 8) and LY rows (2D) or planes (3D) per segment
struct Tile {
    int V, TX, LY;
};

hipError_t launch_update2d(const Dev &d, int storage, int cur, int slot, const Tile &t, hipStream_t s);
hipError_t launch_update3d(const Dev &d, int storage, int cur, int slot, const Tile &t, hipStream_t s);
// launches over several solves: the 2D update of solves sharing (storage, V,
// TX, outer walls or not), and the three fill phases of solves sharing (D,
// storage); implicit: some solve of the fill batch has the semi-implicit
// collision and a moment finish in it
hipError_t launch_update2d_batch(int storage, int V, int TX, bool walls, const BatchArgs &a, hipStream_t s);
hipError_t launch_fill_batch(int D, int storage, const BatchArgs &fin, const BatchArgs &spec, const BatchArgs &ghost,
                             bool implicit, hipStream_t s);
// the FP64 forms of the two above, defined in their own translation unit
hipError_t launch_update2d_f64(const Dev &d, int V, int TX, int cur, int slot, int LY, int ntx, int nys, int ncv,
                               dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_update2d_batch_f64(int V, int TX, bool walls, const BatchArgs &a, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_fill_fin(const Dev &d, int storage, int cur, int slot, bool fill, bool fin, hipStream_t s);
// ghost rows of the diffuse outer walls from buffer cur (no-op unless the
// outer boundary is walls)
hipError_t launch_wall_fill(const Dev &d, int storage, int cur, hipStream_t s);
hipError_t launch_moments_direct(const Dev &d, int storage, int cur, int slot, hipStream_t s);
hipError_t launch_force(const Dev &d, int storage, int cur, hipStream_t s);
// the force kernel with its per-pair records in the library's static device
// scratch (at most kStaticMaxPairs pairs), then the totals, C_D, C_L and up to
// cap wall points written to the device array out; allocates nothing
hipError_t launch_force_static(const Dev &d, int storage, int cur, double *out, int cap, double qd, double Uinf,
                               hipStream_t s);
hipError_t launch_state_freestream(const Dev &d, int storage, int buf, int A, const double *u, double amp, long long off,
                                   long long n, hipStream_t s);
hipError_t launch_state_hashed(const Dev &d, int storage, int buf, int A, unsigned long long seed, double amp,
                               hipStream_t s);
hipError_t launch_state_set(const Dev &d, int storage, int buf, int A, const double *src, long long off, long long n,
                            hipStream_t s);
hipError_t launch_state_get(const Dev &d, int storage, int buf, int A, double *dst, long long off, long long n,
                            hipStream_t s);
hipError_t launch_moments_out(const Dev &d, double *out, hipStream_t s);
// plain streaming copy of words16 16-byte words (measurement)
hipError_t launch_stream_copy(const void *src, void *dst, long long words16, hipStream_t s);

}  // namespace ibdvm
