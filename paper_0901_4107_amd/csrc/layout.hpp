// layout.hpp -- record layouts of libmm's device arrays (element offsets).
//
// Cell reconstruction record, one per cell, array-of-structures so that the
// face kernel gathers a neighbour with a few wide loads:
//   [0, NV)            primitives rho, v (D), P
//   [NV, NV + NV*D)    limited gradient, entry NV + c*D + k = dW_c/dx_k
//   [NV + NV*D, +D)    s_i - r_i (centre of mass minus generator)
//   padding to REC elements (24 in 3D, 16 in 2D)
// In double precision the velocities are lab-frame; in the mixed mode the
// record is float and holds v_i - w_i.
//
// Face record (double path), one per face:
//   A, |d|, n (D) = d/|d|, c (D) = f - (r_L + r_R)/2, w_f (D), padding.
// Mixed face record (float), one per face:
//   A, |d|, n (D), c (D), w_L - w_f (D), w_R - w_f (D), padding;
//   plus the double face velocity w_f in its own array of stride WSTRIDE.
// Side record, one per (cell, face) pair in CSR order:
//   double path: A/|d|, f - r_i (D)             stride 4
//   mixed path:  A/|d|, f - r_i (D), w_j - w_i (D)  stride 8 (float)
#pragma once

namespace mm {

template <int D> struct Lay {
    static constexpr int NV = D + 2;
    static constexpr int W = 0;
    static constexpr int G = NV;
    static constexpr int DL = NV + NV * D;
    static constexpr int REC = (D == 3) ? 24 : 16;
    // double face record
    static constexpr int FA = 0, FELL = 1, FN = 2, FC = 2 + D, FW = 2 + 2 * D;
    static constexpr int FREC = (D == 3) ? 12 : 8;
    // mixed face record
    static constexpr int MDWL = 2 + 2 * D, MDWR = 2 + 3 * D;
    static constexpr int MREC = 16;
    static constexpr int WSTRIDE = (D == 3) ? 4 : 2;
    // side records
    static constexpr int SREC64 = 4;
    static constexpr int SREC32 = 8;
};

}  // namespace mm
