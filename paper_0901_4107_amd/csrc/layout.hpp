// layout.hpp -- record layouts of libmm's device arrays (element offsets).
//
// Reconstruction of the cells, two blocks in one buffer of REC elements
// per cell (24 in 3D, 16 in 2D), each record written whole and gathered
// with 16-byte loads:
//   primitive block [N][PREC]: rho, v (D), P, s_i - r_i (D), padding to 8
//   gradient block  [N][GREC]: limited gradient, element c*D + k = dW_c/dx_k,
//                              padding to 16 (3D) / 8 (2D)
// In double precision the velocities are lab-frame; in the mixed mode the
// records are float and hold v_i - W0, W0 the midrange of the generator
// velocities (a bulk motion the mesh follows leaves these differences small,
// so it costs no float bits).
//
// Face record (double geometry), one per face, 64-byte aligned in 3D:
//   A, |d|, n (D) = d/|d|, c (D) = f - (r_L + r_R)/2;
// the double face velocity w_f in its own array, D per face (the double
// path, the volume rate).
// Mixed face record (float), one per face, 32 bytes in 3D:
//   A, |d|, n (D), c (D);
// and beside it the face velocity relative to W0, w_f - W0 (formed in
// double, rounded once), D floats per face in its own array (a 12-byte
// access per lane, contiguous over a wavefront). With the cells' v_K - W0
// the face-frame velocities are (v_K - W0) - (w_f - W0), and the lab-frame
// flux takes the face velocity as W0 + (w_f - W0) in double: the same
// velocity both ways;
// Face fluxes: face-major, D + 2 doubles per face.
// Side record, one per (cell, face) pair in CSR order:
//   double path: A/|d|, f - r_i (D)             stride 4
//   mixed path:  A/|d|, f - r_i (D)             stride 4 (float)
#pragma once

namespace mm {

template <int D> struct Lay {
    static constexpr int NV = D + 2;
    // primitive and gradient records
    static constexpr int W = 0, DL = NV;
    static constexpr int PREC = 8;
    static constexpr int GREC = (D == 3) ? 16 : 8;
    static constexpr int REC = PREC + GREC;
    // double face record
    static constexpr int FA = 0, FELL = 1, FN = 2, FC = 2 + D;
    static constexpr int FREC = 2 + 2 * D;
    // mixed face record
    static constexpr int MREC = 2 + 2 * D;
    static constexpr int WSTRIDE = D;
    // face fluxes
    static constexpr int FSTRIDE = NV;
    // side records
    static constexpr int SREC64 = 4;
    static constexpr int SREC32 = 4;
};

}  // namespace mm
