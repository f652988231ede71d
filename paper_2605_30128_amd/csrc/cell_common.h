// Device helpers shared by the cell-operator kernels (internal).
#pragma once

#include "internal.h"

namespace chfsi {

// Workgroup ids are dealt to the 8 XCDs round robin; map them so that the
// workgroups of one XCD take a contiguous range of logical tiles (the vector
// blocks of the same cells share that XCD's L2).  A bijection of [0, total).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t total) {
    int64_t q = total >> 3, r = total & 7;
    int64_t x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

struct CellParams {
    const void *X;
    void *Y;
    int64_t ld, nvec;
    const int *cells;
    int64_t ncl;
    int px, py, pz;
    int64_t ncx, ncy, Nx, Ny, Nz;
    int p, n1, n;
    const void *Bk, *BphiT, *Bphi, *W, *dinv;
    double alpha;
    const int *cell_pair_ptr, *cell_pairs, *pair_atom;
    const void *P, *dcoef;
    int nbeta;
    int ldw;      // row length of the bfloat16 w|J| phi table
    int64_t ldd;  // row length of the projector coefficients d
    int mode, flags;
};

// global node of the local node packed as i | j << 8 | k << 16 in cell (ex, ey, ez)
__device__ __forceinline__ int64_t gnode_of(int ijk, int64_t ex, int64_t ey, int64_t ez, int p,
                                            int64_t Nx, int64_t Ny, int64_t Nz) {
    int64_t gx = ex * p + (ijk & 255), gy = ey * p + ((ijk >> 8) & 255), gz = ez * p + (ijk >> 16);
    gx -= gx >= Nx ? Nx : 0;
    gy -= gy >= Ny ? Ny : 0;
    gz -= gz >= Nz ? Nz : 0;
    return gx + Nx * (gy + Ny * gz);
}

// Colour-ordered assembly: the first colour to reach a node (parity 0 in
// every direction in which the node lies on a cell face) writes the node,
// later colours add to it.  With FLAG_ACCUM every colour adds.
__device__ __forceinline__ bool first_touch(int c, int p, int px, int py, int pz, bool accum) {
    int i = c & 255, j = (c >> 8) & 255, k = c >> 16;
    bool fx = (i == 0 || i == p), fy = (j == 0 || j == p), fz = (k == 0 || k == p);
    return !accum && !(fx && px) && !(fy && py) && !(fz && pz);
}

}  // namespace chfsi
