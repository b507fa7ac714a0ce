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
// faces). Layer 1 (K = 3 features + bias, padded to 16) runs on
// v_mfma_f32_16x16x16_bf16, layer 2 (K = 64) on v_mfma_f32_16x16x32_bf16.
// For these instructions lane l holds
//   16x16x16  A[m][k]: m = l%16, k = 4(l/16)+j;  B[k][n]: n = l%16, k = 4(l/16)+j
//   16x16x32  A[m][k]: m = l%16, k = 8(l/16)+j;  B[k][n]: n = l%16, k = 8(l/16)+j
//   both      C[m][n]: n = l%16, m = 4(l/16)+i   (i = 0..3)
// The accumulators of hidden tiles 2s and 2s+1 of layer 1, side by side,
// are lane for lane the B operand of k-step s of layer 2 once the input
// units of that step are numbered (g = l/16, slot j) -> 32s + 4g + (j%4) +
// 16(j/4); the packed A operand of layer 2 uses the same numbering, so no
// data moves between the layers. The wave's 64 faces form four 16-face
// column tiles; the bias of layer 1 rides in k = 3, the rest of k is zero.
#pragma once

#include <hip/hip_runtime.h>

namespace mm {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMlpHidden = 64;
// Parameter vector (float, trained form): W1 [3][64] (in-major), b1 [64],
// W2 [64][64] (in-major), b2 [64], w3 [64], b3 [1].
constexpr int kMlpOffW1 = 0, kMlpOffB1 = 192, kMlpOffW2 = 256, kMlpOffB2 = 4352, kMlpOffW3 = 4416,
              kMlpOffB3 = 4480, kMlpParams = 4481;
constexpr float kMlpScaleRho = 0.2f, kMlpScaleP = 0.2f, kMlpScaleU = 0.5f, kMlpScaleY = 1.0f;
// Strength gate of the learned guess: a density or pressure ratio of at
// least e (scaled log feature >= 0.2) or a velocity jump of at least
// 0.4 (c_L + c_R) (scaled feature >= 0.2).
constexpr double kMlpGateRatio = 2.718281828459045, kMlpGateDu = 0.4;

// Packed inference form (device, built by k_mlp_pack): per (tile, k-step)
// the A operand of every lane (4 bf16 = 8 bytes), then the fp32 biases.
struct MlpPacked {
    bf16x4_t a1[4][64];          // layer 1: hidden tile t, lane l
    bf16x8_t a2[4][2][64];       // layer 2: output tile t, k-step s, lane l
    float b2[64], w3[64], b3;
};

// Input unit of layer 2 held in slot j of lane group g at k-step s.
__host__ __device__ constexpr int mlp_l2_unit(int s, int g, int j) { return 32 * s + 4 * g + (j & 3) + 16 * (j >> 2); }

struct MlpGuess {
    const MlpPacked *p;
};

// float -> bf16, round to nearest even (one v_cvt_pk_bf16_f32 per pair)
__device__ __forceinline__ short f2bf(float x) { return __builtin_bit_cast(short, (__bf16)x); }

// max(x, 0) as one integer max on the bit pattern: a float with the sign bit
// set is a negative integer (-0 included), so it maps to +0.
__device__ __forceinline__ float relu(float x) {
    const int b = __builtin_bit_cast(int, x);
    return __builtin_bit_cast(float, b > 0 ? b : 0);
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
// The four 16-face column tiles go in two passes of two: layer 1 for the
// pass's columns, then layers 2 and 3 one output tile at a time. Each weight
// is read twice per wavefront (L1 hits); the scheduling barriers keep each
// tile's weight loads next to their use, so the network adds few registers
// to the flux code's. npass (1 or 2, the same for the whole wavefront):
// with 1 only the first 32 lanes' columns are evaluated.
__device__ __forceinline__ float mlp_wave_infer(const MlpPacked *__restrict__ P, float x0, float x1, float x2,
                                                int npass = 2) {
    const int lane = threadIdx.x & 63;
    const int src = lane & 15;
    const bool low = lane < 16;
    const int rbase = 4 * (lane >> 4);
    float yy = 0.0f;
#pragma unroll 1
    for (int pass = 0; pass < npass; pass++) {
        // the weights are re-read in each pass rather than held in
        // registers across both: the empty asm makes the offset opaque, so
        // the loads stay inside the pass
        int zero = 0;
        asm volatile("" : "+s"(zero));
        const MlpPacked *Q = P + zero;
        // layer 1 -> relu -> bf16; h1[s][j] is the B operand of k-step s of
        // layer 2 for column tile 2 pass + j: tiles 2s and 2s+1 side by side
        bf16x8_t h1[2][2];
        for (int j = 0; j < 2; j++) {
            const int n = 2 * pass + j;
            const float a = __shfl(x0, 16 * n + src, 64);
            const float b = __shfl(x1, 16 * n + src, 64);
            const float c = __shfl(x2, 16 * n + src, 64);
            bf16x4_t xb;
            xb[0] = low ? f2bf(a) : (short)0;
            xb[1] = low ? f2bf(b) : (short)0;
            xb[2] = low ? f2bf(c) : (short)0;
            xb[3] = low ? f2bf(1.0f) : (short)0;
            for (int t = 0; t < 4; t++) {
                f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Q->a1[t][lane], xb, acc, 0, 0, 0);
                for (int i = 0; i < 4; i++) h1[t >> 1][j][4 * (t & 1) + i] = (__bf16)relu(acc[i]);
            }
        }
        // layer 2 (+ b2, relu) and layer 3 (w3 dot), one output tile at a time
        float yp[2] = {0.0f, 0.0f};
        for (int t = 0; t < 4; t++) {
            __builtin_amdgcn_sched_barrier(0);
            const bf16x8_t w0 = Q->a2[t][0][lane], w1 = Q->a2[t][1][lane];
            const f32x4_t bias = *reinterpret_cast<const f32x4_t *>(Q->b2 + 16 * t + rbase);
            const f32x4_t w3 = *reinterpret_cast<const f32x4_t *>(Q->w3 + 16 * t + rbase);
            for (int j = 0; j < 2; j++) {
                f32x4_t acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, h1[0][j], bias, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, h1[1][j], acc, 0, 0, 0);
                for (int i = 0; i < 4; i++) yp[j] += w3[i] * relu(acc[i]);
            }
        }
        // sum the four row groups of each column (lanes l, l^16, l^32, l^48);
        // lane l's face is column l%16 of tile l/16
        for (int j = 0; j < 2; j++) {
            yp[j] += __shfl_xor(yp[j], 16, 64);
            yp[j] += __shfl_xor(yp[j], 32, 64);
            yy = (lane >> 4) == 2 * pass + j ? yp[j] : yy;
        }
    }
    return yy + P->b3;
}

}  // namespace mm
