// The memory bound of the stream-collide: its pull alone, as a copy.
#pragma once

#include "fslbm_device.hpp"

namespace fslbm {

// The pull of the streaming step alone (measurement aid): every cell of a
// periodic nx x ny x nz lattice copies the 19 values upstream of it to its
// own slots, dst_q(x) = src_q(x - c_q), with no collision and no cell
// types. Grid, chunk order (runs of `run` chunks per XCD), launch bounds
// and non-temporal stores are those of the bulk stream-collide, so its
// duration is what that kernel's memory traffic costs when no arithmetic
// is added; S is the stored element (8, 4 or 2 bytes).
template <class S>
__global__ __launch_bounds__(SC_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_pull_copy(
    const S *__restrict__ src, S *__restrict__ dst, int nx, int ny, int nz, int NS, int run)
{
    const unsigned n = unsigned(nx) * unsigned(ny) * unsigned(nz);
    for (int c = xcd_chunk(blockIdx.x, gridDim.x, run); unsigned(c) * SC_BLOCK < n; c += gridDim.x) {
        const unsigned k = unsigned(c) * SC_BLOCK + threadIdx.x;
        if (k >= n) continue;
        const unsigned r = k / unsigned(nx);
        const Nbr nb(int(k - r * unsigned(nx)), int(r % unsigned(ny)), int(r / unsigned(ny)), nx, ny, nz);
        const int i = nb.at(0, 0, 0);
        S v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = src[(size_t)q * (size_t)NS + nb.at(-dir_x(q), -dir_y(q), -dir_z(q))];
#pragma unroll
        for (int q = 0; q < NQ; ++q) __builtin_nontemporal_store(v[q], dst + (size_t)q * (size_t)NS + i);
    }
}

}  // namespace fslbm
