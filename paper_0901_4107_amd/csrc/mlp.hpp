// mlp.hpp -- learned starting guess for the star pressure: a 3 -> 64 -> 64 -> 1
// ReLU network evaluated by one wavefront for its 64 faces on the matrix
// cores (bf16 operands, fp32 accumulation), fused into the flux kernels.
//
// Features of a Riemann problem (density ratio, pressure ratio, velocity
// jump over the sound speeds), scaled to O(1):
//   x0 = ln(rho_R/rho_L)/5, x1 = ln(P_R/P_L)/5, x2 = (u_R - u_L)/(c_L + c_R)/2,
// target y = ln(p* / p_std), the log of the standard guess's error (a
// function of the same three dimensionless numbers), so the learned guess is
// p = p_std exp(y): the network learns a correction, which is small where
// the standard guess is good (it is exact for two rarefactions), and the
// bf16 rounding of the network scales with that correction, not with p*.
//
// The network runs transposed, H^T = W^T X^T (rows = hidden units, columns =
// faces), on v_mfma_f32_16x16x16_bf16. For that instruction lane l holds
//   A[m][k]: m = l%16, k = 4(l/16)+j;  B[k][n]: n = l%16, k = 4(l/16)+j;
//   C[m][n]: n = l%16, m = 4(l/16)+i   (j, i = 0..3),
// so the accumulator of hidden tile t is, lane for lane, the B operand of
// k-step t of the next layer: no data moves between layers 1 and 2. The
// wave's 64 faces form four 16-face column tiles; the bias of layer 1 rides
// in k = 3 (feature 1), the rest of k = 4..15 is zero.
#pragma once

#include <hip/hip_runtime.h>

namespace mm {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMlpHidden = 64;
// Parameter vector (float, trained form): W1 [3][64] (in-major), b1 [64],
// W2 [64][64] (in-major), b2 [64], w3 [64], b3 [1].
constexpr int kMlpOffW1 = 0, kMlpOffB1 = 192, kMlpOffW2 = 256, kMlpOffB2 = 4352, kMlpOffW3 = 4416,
              kMlpOffB3 = 4480, kMlpParams = 4481;
constexpr float kMlpScaleRho = 0.2f, kMlpScaleP = 0.2f, kMlpScaleU = 0.5f, kMlpScaleY = 1.0f;

// Packed inference form (device, built by k_mlp_pack): per (tile, k-step)
// the A operand of every lane (4 bf16 = 8 bytes), then the fp32 biases.
struct MlpPacked {
    bf16x4_t a1[4][64];          // layer 1: hidden tile t, lane l
    bf16x4_t a2[4][4][64];       // layer 2: hidden tile t, k-step s, lane l
    float b2[64], w3[64], b3;
};

struct MlpGuess {
    const MlpPacked *p;
};

__device__ __forceinline__ short f2bf(float x) {
    // round to nearest even (finite inputs)
    unsigned u = __builtin_bit_cast(unsigned, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// Features of one problem; valid = false gives zeros.
__device__ __forceinline__ void mlp_features(float rhoL, float uL, float PL, float rhoR, float uR, float PR,
                                             float gamma, float &x0, float &x1, float &x2) {
    const float cL = __builtin_sqrtf(gamma * PL / rhoL), cR = __builtin_sqrtf(gamma * PR / rhoR);
    x0 = kMlpScaleRho * __logf(rhoR / rhoL);
    x1 = kMlpScaleP * __logf(PR / PL);
    x2 = kMlpScaleU * (uR - uL) / (cL + cR);
}

// Whole-wavefront inference: every lane of the wave must call this (full
// exec mask); lane l supplies the features of its face and receives y.
__device__ __forceinline__ float mlp_wave_infer(const MlpPacked *__restrict__ P, float x0, float x1, float x2) {
    const int lane = threadIdx.x & 63;
    const int src = lane & 15;
    const bool low = lane < 16;
    // layer 1 B operands: column tile n holds faces 16n..16n+15
    bf16x4_t xb[4];
    for (int n = 0; n < 4; n++) {
        const float a = __shfl(x0, 16 * n + src, 64);
        const float b = __shfl(x1, 16 * n + src, 64);
        const float c = __shfl(x2, 16 * n + src, 64);
        bf16x4_t v;
        v[0] = low ? f2bf(a) : (short)0;
        v[1] = low ? f2bf(b) : (short)0;
        v[2] = low ? f2bf(c) : (short)0;
        v[3] = low ? f2bf(1.0f) : (short)0;
        xb[n] = v;
    }
    // layer 1 -> h1 (relu, bf16), kept as the B operands of layer 2
    bf16x4_t h1[4][4];  // [hidden tile t][column tile n]
    for (int t = 0; t < 4; t++) {
        const bf16x4_t a = P->a1[t][lane];
        for (int n = 0; n < 4; n++) {
            f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, xb[n], acc, 0, 0, 0);
            bf16x4_t h;
            for (int i = 0; i < 4; i++) h[i] = f2bf(acc[i] > 0.0f ? acc[i] : 0.0f);
            h1[t][n] = h;
        }
    }
    // layer 2 (+ b2, relu) and layer 3 (w3 dot, + b3), one hidden tile at a time
    float y[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const int rbase = 4 * (lane >> 4);
    for (int t = 0; t < 4; t++) {
        f32x4_t acc[4];
        for (int n = 0; n < 4; n++)
            for (int i = 0; i < 4; i++) acc[n][i] = P->b2[16 * t + rbase + i];
        for (int s = 0; s < 4; s++) {
            const bf16x4_t a = P->a2[t][s][lane];
            for (int n = 0; n < 4; n++) acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, h1[s][n], acc[n], 0, 0, 0);
        }
        for (int n = 0; n < 4; n++)
            for (int i = 0; i < 4; i++) {
                const float h = acc[n][i] > 0.0f ? acc[n][i] : 0.0f;
                y[n] += P->w3[16 * t + rbase + i] * h;
            }
    }
    // sum the four row groups of each column (lanes l, l^16, l^32, l^48)
    for (int n = 0; n < 4; n++) {
        y[n] += __shfl_xor(y[n], 16, 64);
        y[n] += __shfl_xor(y[n], 32, 64);
    }
    // lane l's face is column l%16 of tile l/16
    const int me = lane >> 4;
    const float yy = me == 0 ? y[0] : me == 1 ? y[1] : me == 2 ? y[2] : y[3];
    return yy + P->b3;
}

}  // namespace mm
