// The one-level local expansion of the block-mode coarse field as a
// convolution on the moment grid, evaluated with 64-point FFTs along each
// axis of a zero-padded 64^3 grid (grids of at most 32 cells a side).
#pragma once

#include <hip/hip_runtime.h>

namespace ld {

constexpr int kConvMaxGrid = 32;       // linear convolution of G^3 on a 64^3 period

struct LocalConv {
    int B = 0;                         // block side the kernels exclude
    float2* work = nullptr;            // [15][64^3] transforms (and set-up scratch)
    float* spec = nullptr;             // [30][64^3] kernel spectra (real or imaginary part)
};

// Allocates the buffers and transforms the derivative kernels of 1/r (zero
// inside the B^3 block) once; enqueued on s.
hipError_t conv_setup(LocalConv* lc, int B, hipStream_t s);

// E[cell][19] (cells of the G^3 grid, G <= kConvMaxGrid): the field E (0-2),
// its gradient J (xx xy xz yy yz at 3-7) and second gradient H (xxx xxy xxz
// xyy xyz at 9-13, yyy yyz at 15-16) at each cell centre from the monopole
// and dipole moments mom[cell][4] = (Q, Px, Py, Pz) of every cell outside
// the block around it; h points at the cell side (device).  The traceless
// components 8, 14, 17, 18 are left for the evaluation.
hipError_t conv_local(const LocalConv* lc, const double* mom, int G, const double* h, double* E,
                      hipStream_t s);

void conv_free(LocalConv* lc);

}  // namespace ld
