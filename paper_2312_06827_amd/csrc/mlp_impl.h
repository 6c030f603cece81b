// The per-pixel network's forward pass on the matrix cores, shared by the
// network kernels and by the temporal kernel's learned mode.
//
// Matrix layout.  Each layer is computed transposed, Y^T = W X^T, with
// v_mfma_f32_32x32x8_bf16: A = the weights (32 output units x 8 inputs per
// instruction), B = 32 pixels x 8 inputs.  Lane l supplies A[l % 32][4 (l/32)
// + 0..3] and B[4 (l/32) + 0..3][l % 32] of each 8-wide K block and receives
// D[8 (r/4) + 4 (l/32) + r % 4][l % 32] in accumulator r = 0..15.  So after a
// layer, accumulators 4 kb .. 4 kb + 3 of a lane are exactly that lane's B
// operand for K block kb of the next layer: activations never leave
// registers in the forward pass.
#pragma once
#include "sv_internal.h"

namespace sv {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kOffW1 = 0, kOffB1 = 448, kOffW2 = 480, kOffB2 = 1504, kOffW3 = 1536,
              kOffB3 = 1600;
static_assert(kOffB3 + 2 == SV_MLP_PARAMS, "parameter layout");
constexpr float kAlphaMin = 0.05f;

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

__device__ __forceinline__ f32x16 mfma(bf16x4 a, bf16x4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}

// Output unit (row of D) held in accumulator r by a lane of half `hf`.
__device__ __forceinline__ int drow(int r, int hf) { return 8 * (r >> 2) + 4 * hf + (r & 3); }

// Weights one lane holds for the forward pass.
struct FwdW {
    bf16x4 w1[2], w2[4];
    float w3a[16], w3b[16];  // W3 rows 0 and 1 at this lane's units (bf16 values)
    float b3a, b3b;
};

__device__ __forceinline__ void load_fwd(const float *params, const uint16_t *wq, int col, int hf,
                                         FwdW &f) {
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 8 * kb + 4 * hf + i;
            f.w1[kb][i] = (short)(k < SV_MLP_IN ? wq[kOffW1 + col * SV_MLP_IN + k] : 0);
        }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            f.w2[kb][i] = (short)wq[kOffW2 + col * SV_MLP_HIDDEN + 8 * kb + 4 * hf + i];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        f.w3a[r] = from_bf16(wq[kOffW3 + drow(r, hf)]);
        f.w3b[r] = from_bf16(wq[kOffW3 + SV_MLP_HIDDEN + drow(r, hf)]);
    }
    f.b3a = params[kOffB3];
    f.b3b = params[kOffB3 + 1];
}

// Forward pass of one 32-pixel block.  x: this lane's B operands of layer
// 1; returns the layer-1 and layer-2 pre-activations (with biases), the
// bfloat16 layer-2 activations as floats, and the two outputs (the same in
// both halves of the wave).
struct FwdOut {
    f32x16 a1, a2;
    bf16x4 h1[4];
    float h2[16];
    float o0, o1;
};

__device__ __forceinline__ void forward_block(const float *params, const FwdW &f,
                                              const bf16x4 (&x)[2], int hf, FwdOut &r) {
#pragma unroll
    for (int i = 0; i < 16; ++i) r.a1[i] = params[kOffB1 + drow(i, hf)];
    r.a1 = mfma(f.w1[0], x[0], r.a1);
    r.a1 = mfma(f.w1[1], x[1], r.a1);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i) r.h1[kb][i] = (short)to_bf16(fmaxf(r.a1[4 * kb + i], 0.f));
#pragma unroll
    for (int i = 0; i < 16; ++i) r.a2[i] = params[kOffB2 + drow(i, hf)];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) r.a2 = mfma(f.w2[kb], r.h1[kb], r.a2);
    float o0 = 0.f, o1 = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        r.h2[i] = from_bf16(to_bf16(fmaxf(r.a2[i], 0.f)));
        o0 = fmaf(f.w3a[i], r.h2[i], o0);
        o1 = fmaf(f.w3b[i], r.h2[i], o1);
    }
    o0 += __shfl_xor(o0, 32, 64);
    o1 += __shfl_xor(o1, 32, 64);
    r.o0 = o0 + f.b3a;
    r.o1 = o1 + f.b3b;
}


// The parameters one workgroup stages in LDS for forward_block_lds: every
// bfloat16 copy (wq) and the three float bias vectors, packed as B1 | B2 | B3.
constexpr int kNetBiases = 2 * SV_MLP_HIDDEN + 2;
constexpr int kNetB1 = 0, kNetB2 = SV_MLP_HIDDEN, kNetB3 = 2 * SV_MLP_HIDDEN;
constexpr int kNetStageIt = (SV_MLP_PARAMS + 255) / 256;  // bf16 values per thread

struct NetStage {  // one thread's share of the staging loads
    uint16_t w[kNetStageIt];
    float b;
};

// Issue this thread's staging loads (256 threads cover every value).
__device__ __forceinline__ void net_issue(const float *params, const uint16_t *wq, NetStage &ns) {
    // indices clamped into the arrays, so no load can leave them
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kNetStageIt; ++k)
        ns.w[k] = wq[min(t + 256 * k, SV_MLP_PARAMS - 1)];
    const int tb = min(t, kNetBiases - 1);
    const int bi = tb < SV_MLP_HIDDEN ? kOffB1 + tb
                   : tb < 2 * SV_MLP_HIDDEN ? kOffB2 + tb - SV_MLP_HIDDEN
                                            : kOffB3 + tb - 2 * SV_MLP_HIDDEN;
    ns.b = params[bi];
}

// Store them (each index once; the clamped duplicates are not stored);
// visible after the caller's next barrier.
__device__ __forceinline__ void net_store(const NetStage &ns, uint16_t *s_w, float *s_b) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kNetStageIt; ++k) {
        const int i = t + 256 * k;
        if (i < SV_MLP_PARAMS) s_w[i] = ns.w[k];
    }
    if (t < kNetBiases) s_b[t] = ns.b;
}

// forward_block with every parameter read from the workgroup's LDS copy
// (s_w: the bfloat16 values, s_b: the biases) where it is used: the same
// operands, operations and order, so bitwise the same outputs, with no
// weight held in registers across blocks.
__device__ __forceinline__ void forward_block_lds(const uint16_t *s_w, const float *s_b, int col,
                                                  int hf, const bf16x4 (&x)[2], FwdOut &r) {
    bf16x4 w1[2], w2[4];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 8 * kb + 4 * hf + i;
            w1[kb][i] = (short)(k < SV_MLP_IN ? s_w[kOffW1 + col * SV_MLP_IN + k] : 0);
        }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            w2[kb][i] = (short)s_w[kOffW2 + col * SV_MLP_HIDDEN + 8 * kb + 4 * hf + i];
#pragma unroll
    for (int i = 0; i < 16; ++i) r.a1[i] = s_b[kNetB1 + drow(i, hf)];
    r.a1 = mfma(w1[0], x[0], r.a1);
    r.a1 = mfma(w1[1], x[1], r.a1);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i) r.h1[kb][i] = (short)to_bf16(fmaxf(r.a1[4 * kb + i], 0.f));
#pragma unroll
    for (int i = 0; i < 16; ++i) r.a2[i] = s_b[kNetB2 + drow(i, hf)];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) r.a2 = mfma(w2[kb], r.h1[kb], r.a2);
    float o0 = 0.f, o1 = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        r.h2[i] = from_bf16(to_bf16(fmaxf(r.a2[i], 0.f)));
        o0 = fmaf(from_bf16(s_w[kOffW3 + drow(i, hf)]), r.h2[i], o0);
        o1 = fmaf(from_bf16(s_w[kOffW3 + SV_MLP_HIDDEN + drow(i, hf)]), r.h2[i], o1);
    }
    o0 += __shfl_xor(o0, 32, 64);
    o1 += __shfl_xor(o1, 32, 64);
    r.o0 = o0 + s_b[kNetB3];
    r.o1 = o1 + s_b[kNetB3 + 1];
}

// alpha = 0.05 + 0.95 sigmoid(o0), kappa = 2^(2 tanh(o1)).
__device__ __forceinline__ void mlp_heads(float o0, float o1, float &alpha, float &kappa) {
    alpha = kAlphaMin + (1.0f - kAlphaMin) / (1.0f + expf(-o0));
    kappa = exp2f(2.0f * tanhf(o1));
}

}  // namespace sv
