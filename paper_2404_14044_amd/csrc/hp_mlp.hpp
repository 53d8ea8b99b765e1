// The 32 -> 64 -> 64 -> 4 decoder on matrix cores, shared by the render and
// its backward pass.  Sixteen samples form the N dimension of each product
// (H^T = W X^T): lane l holds sample l % 16 and, in every accumulator, rows
// 4 (l / 16) .. +3 of a 16-row output block.  Those accumulators feed the next
// layer's B operand directly; the contraction index is permuted consistently
// in the weights instead of moving activations between lanes.
#pragma once

#include "hp_device.hpp"

namespace hp {

struct MlpWeights {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

// Rounding to bfloat16 (round to nearest, ties to even): gfx950 converts two
// binary32 values per instruction (v_cvt_pk_bf16_f32), subnormals kept in
// the kernels' floating-point mode; checked bit for bit against the
// definition by the exact-rounding test of hp_bf16_eval.
__device__ __forceinline__ uint32_t bf16_pair_bits(float lo, float hi)
{
    bf16x2 v;
    v[0] = (__bf16)lo;
    v[1] = (__bf16)hi;
    return __builtin_bit_cast(uint32_t, v);
}

// x rounded to bfloat16, as a float
__device__ __forceinline__ float bf16_round(float x)
{
    return __uint_as_float(bf16_pair_bits(x, 0.0f) << 16);
}

__device__ __forceinline__ bf16x8 pack_bf16x8(const float *v)
{
    union {
        uint32_t u[4];
        bf16x8 b;
    } r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.u[i] = bf16_pair_bits(v[2 * i], v[2 * i + 1]);
    return r.b;
}

// Hidden-feature index that lane l's element e feeds at contraction block kb
// of a 64-wide layer input: the previous layer's output block 2 kb + e / 4,
// row 4 (l / 16) + e % 4.
__device__ __forceinline__ int hid_index(int kb, int l, int e)
{
    return 32 * kb + 16 * (e >> 2) + 4 * (l >> 4) + (e & 3);
}

// max(x, 0) of a matrix-core result as the integer maximum of its bits (a
// negative number or -0 has the sign bit set and becomes +0): one
// instruction, where the floating-point maximum takes two (the compiler first
// quiets a possible signalling NaN, which these results never are).  Equal to
// fmaxf(x, 0) for every x that is not a NaN.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ __forceinline__ float softplus_f(float x)
{
    return __builtin_fmaxf(x, 0.0f) + log1pf(expf(-__builtin_fabsf(x)));
}

__device__ __forceinline__ float sigmoid_f(float x) { return 1.0f / (1.0f + expf(-x)); }


// ---------------------------------------------------------------------------
// decoder on one tile of 16 samples; returns o[0..3] of sample l (lanes 0..15)
// ---------------------------------------------------------------------------
struct MlpBf16 {
    bf16x8 w1[4];      // [out block]
    bf16x8 w2[4][2];   // [out block][k block]
    bf16x8 w3[2];      // [k block]
    float b1[4][4], b2[4][4], b3[4];

    __device__ __forceinline__ bf16x8 W1(int ob) const { return w1[ob]; }
    __device__ __forceinline__ bf16x8 W2(int ob, int kb) const { return w2[ob][kb]; }
    __device__ __forceinline__ bf16x8 W3(int kb) const { return w3[kb]; }
    __device__ __forceinline__ f32x4 B1(int ob) const { return {b1[ob][0], b1[ob][1], b1[ob][2], b1[ob][3]}; }
    __device__ __forceinline__ f32x4 B2(int ob) const { return {b2[ob][0], b2[ob][1], b2[ob][2], b2[ob][3]}; }
    __device__ __forceinline__ f32x4 B3() const { return {b3[0], b3[1], b3[2], b3[3]}; }
};

// The lane's A-operand fragments (8 bf16 of one weight row), one function
// per piece so that the register and the shared copies of the weights hold
// the same bits.
__device__ __forceinline__ bf16x8 w1_fragment(const MlpWeights &a, int ob, int l)
{
    const int r = l & 15, q = l >> 4;
    float tmp[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) tmp[e] = a.W1[(16 * ob + r) * HP_FEAT_DIM + 8 * q + e];
    return pack_bf16x8(tmp);
}

__device__ __forceinline__ bf16x8 w2_fragment(const MlpWeights &a, int ob, int kb, int l)
{
    const int r = l & 15;
    float tmp[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) tmp[e] = a.W2[(16 * ob + r) * HP_HIDDEN + hid_index(kb, l, e)];
    return pack_bf16x8(tmp);
}

// rows 4 .. 15 of the output block are zero padding; their lanes load a
// real row and drop it, so that no load waits behind a branch
__device__ __forceinline__ bf16x8 w3_fragment(const MlpWeights &a, int kb, int l)
{
    const int r = l & 15, r3 = r < 4 ? r : 3;
    float tmp[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float w = a.W3[r3 * HP_HIDDEN + hid_index(kb, l, e)];
        tmp[e] = r < 4 ? w : 0.0f;
    }
    return pack_bf16x8(tmp);
}

__device__ __forceinline__ void load_mlp_bf16(const MlpWeights &a, MlpBf16 &m)
{
    const int l = lane_id();
    const int q = l >> 4;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        m.w1[ob] = w1_fragment(a, ob, l);
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) m.w2[ob][kb] = w2_fragment(a, ob, kb, l);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            m.b1[ob][e] = a.b1[16 * ob + 4 * q + e];
            m.b2[ob][e] = a.b2[16 * ob + 4 * q + e];
        }
    }
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) m.w3[kb] = w3_fragment(a, kb, l);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float b = a.b3[(4 * q + e) & 3];
        m.b3[e] = q == 0 ? b : 0.0f;
    }
}

// The same weights in the LDS, shared by the waves of a workgroup: each lane
// reads its own fragments (16-byte reads) when a tile needs them, so they
// hold no registers between tiles.
struct MlpBf16Shared {
    bf16x8 w1[4][WAVE];
    bf16x8 w2[4][2][WAVE];
    bf16x8 w3[2][WAVE];
    float4 b1[16], b2[16], b3[4];  // [4 ob + q]: biases 16 ob + 4 q .. + 3; b3: [q]

    __device__ __forceinline__ bf16x8 W1(int ob) const { return w1[ob][lane_id()]; }
    __device__ __forceinline__ bf16x8 W2(int ob, int kb) const { return w2[ob][kb][lane_id()]; }
    __device__ __forceinline__ bf16x8 W3(int kb) const { return w3[kb][lane_id()]; }
    __device__ __forceinline__ f32x4 B1(int ob) const
    {
        const float4 v = b1[4 * ob + (lane_id() >> 4)];
        return {v.x, v.y, v.z, v.w};
    }
    __device__ __forceinline__ f32x4 B2(int ob) const
    {
        const float4 v = b2[4 * ob + (lane_id() >> 4)];
        return {v.x, v.y, v.z, v.w};
    }
    __device__ __forceinline__ f32x4 B3() const
    {
        const float4 v = b3[lane_id() >> 4];
        return {v.x, v.y, v.z, v.w};
    }
};

// Fill the shared weights: wave `w` of `nw` packs every nw-th fragment (all
// waves of the workgroup call this; a barrier must follow before use).
__device__ __forceinline__ void store_mlp_bf16_shared(const MlpWeights &a, MlpBf16Shared &m, int w,
                                                      int nw)
{
    const int l = lane_id();
    for (int p = w; p < 14; p += nw) {
        if (p < 4) m.w1[p][l] = w1_fragment(a, p, l);
        else if (p < 12) m.w2[(p - 4) >> 1][(p - 4) & 1][l] = w2_fragment(a, (p - 4) >> 1, (p - 4) & 1, l);
        else m.w3[p - 12][l] = w3_fragment(a, p - 12, l);
    }
    if (w == 0) {
        reinterpret_cast<float *>(m.b1)[l] = a.b1[l];
        reinterpret_cast<float *>(m.b2)[l] = a.b2[l];
        if (l < 16) reinterpret_cast<float *>(m.b3)[l] = l < 4 ? a.b3[l] : 0.0f;
    }
}

// The register copy from a packed image (global or LDS memory): sixteen-byte
// reads straight into the operand registers, no conversion.
__device__ __forceinline__ void load_mlp_bf16_image(const MlpBf16Shared &img, MlpBf16 &m)
{
    const int l = lane_id(), q = l >> 4;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        m.w1[ob] = img.w1[ob][l];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) m.w2[ob][kb] = img.w2[ob][kb][l];
        const float4 b1 = img.b1[4 * ob + q], b2 = img.b2[4 * ob + q];
        m.b1[ob][0] = b1.x, m.b1[ob][1] = b1.y, m.b1[ob][2] = b1.z, m.b1[ob][3] = b1.w;
        m.b2[ob][0] = b2.x, m.b2[ob][1] = b2.y, m.b2[ob][2] = b2.z, m.b2[ob][3] = b2.w;
    }
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) m.w3[kb] = img.w3[kb][l];
    const float4 b3 = img.b3[q];
    m.b3[0] = b3.x, m.b3[1] = b3.y, m.b3[2] = b3.z, m.b3[3] = b3.w;
}

template <typename M>
__device__ __forceinline__ f32x4 decode_bf16(const M &m, const float *f, f32x4 *keep1 = nullptr,
                                             f32x4 *keep2 = nullptr)
{
    const bf16x8 x = pack_bf16x8(f);
    f32x4 h1[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = m.B1(ob);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.W1(ob), x, acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = relu(acc[e]);
        h1[ob] = acc;
        if (keep1) keep1[ob] = acc;
    }
    bf16x8 x2[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        float t8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t8[e] = h1[2 * kb + (e >> 2)][e & 3];
        x2[kb] = pack_bf16x8(t8);
    }
    f32x4 h2[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = m.B2(ob);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.W2(ob, 0), x2[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.W2(ob, 1), x2[1], acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = relu(acc[e]);
        h2[ob] = acc;
        if (keep2) keep2[ob] = acc;
    }
    bf16x8 x3[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        float t8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t8[e] = h2[2 * kb + (e >> 2)][e & 3];
        x3[kb] = pack_bf16x8(t8);
    }
    f32x4 o = m.B3();
    o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.W3(0), x3[0], o, 0, 0, 0);
    o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.W3(1), x3[1], o, 0, 0, 0);
    return o;
}

// FP32: v_mfma_f32_16x16x4f32, lane l supplies contraction row l / 16 of
// each 4-deep step.  Layer 1 step ks takes feature 8 (l / 16) + ks; layer 2
// and 3 step (ob, e) take hidden feature 16 ob + 4 (l / 16) + e.
struct MlpF32 {
    float w1[4][8];    // [out block][step]
    float w2[4][16];   // [out block][step]
    float w3[16];
    float b1[4][4], b2[4][4], b3[4];

    // steps 4 i .. 4 i + 3 of a layer's A operands, and the bias quarters
    __device__ __forceinline__ f32x4 W1q(int ob, int i) const
    {
        return {w1[ob][4 * i], w1[ob][4 * i + 1], w1[ob][4 * i + 2], w1[ob][4 * i + 3]};
    }
    __device__ __forceinline__ f32x4 W2q(int ob, int i) const
    {
        return {w2[ob][4 * i], w2[ob][4 * i + 1], w2[ob][4 * i + 2], w2[ob][4 * i + 3]};
    }
    __device__ __forceinline__ f32x4 W3q(int i) const
    {
        return {w3[4 * i], w3[4 * i + 1], w3[4 * i + 2], w3[4 * i + 3]};
    }
    __device__ __forceinline__ f32x4 B1(int ob) const { return {b1[ob][0], b1[ob][1], b1[ob][2], b1[ob][3]}; }
    __device__ __forceinline__ f32x4 B2(int ob) const { return {b2[ob][0], b2[ob][1], b2[ob][2], b2[ob][3]}; }
    __device__ __forceinline__ f32x4 B3() const { return {b3[0], b3[1], b3[2], b3[3]}; }
};

// The lane's FP32 A operands, four steps at a time (one function per piece,
// shared by the register and the LDS copies).
__device__ __forceinline__ float4 w1_quad_f32(const MlpWeights &a, int ob, int i, int l)
{
    const int r = l & 15, q = l >> 4;
    const float *w = a.W1 + (16 * ob + r) * HP_FEAT_DIM + 8 * q + 4 * i;
    return make_float4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ float4 w2_quad_f32(const MlpWeights &a, int ob, int i, int l)
{
    const int r = l & 15, q = l >> 4;
    const float *w = a.W2 + (16 * ob + r) * HP_HIDDEN + 16 * i + 4 * q;
    return make_float4(w[0], w[1], w[2], w[3]);
}

// (padding rows: see w3_fragment)
__device__ __forceinline__ float4 w3_quad_f32(const MlpWeights &a, int i, int l)
{
    const int r = l & 15, q = l >> 4, r3 = r < 4 ? r : 3;
    const float *w = a.W3 + r3 * HP_HIDDEN + 16 * i + 4 * q;
    const float4 v = make_float4(w[0], w[1], w[2], w[3]);
    return r < 4 ? v : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

__device__ __forceinline__ void load_mlp_f32(const MlpWeights &a, MlpF32 &m)
{
    const int l = lane_id();
    const int q = l >> 4;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float4 v = w1_quad_f32(a, ob, i, l);
            m.w1[ob][4 * i] = v.x, m.w1[ob][4 * i + 1] = v.y, m.w1[ob][4 * i + 2] = v.z, m.w1[ob][4 * i + 3] = v.w;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float4 v = w2_quad_f32(a, ob, i, l);
            m.w2[ob][4 * i] = v.x, m.w2[ob][4 * i + 1] = v.y, m.w2[ob][4 * i + 2] = v.z, m.w2[ob][4 * i + 3] = v.w;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            m.b1[ob][e] = a.b1[16 * ob + 4 * q + e];
            m.b2[ob][e] = a.b2[16 * ob + 4 * q + e];
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float4 v = w3_quad_f32(a, i, l);
        m.w3[4 * i] = v.x, m.w3[4 * i + 1] = v.y, m.w3[4 * i + 2] = v.z, m.w3[4 * i + 3] = v.w;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float b = a.b3[(4 * q + e) & 3];
        m.b3[e] = q == 0 ? b : 0.0f;
    }
}

// The FP32 weights in the LDS, shared by a workgroup's waves (as MlpBf16Shared).
struct MlpF32Shared {
    float4 w1[4][2][WAVE];
    float4 w2[4][4][WAVE];
    float4 w3[4][WAVE];
    float4 b1[16], b2[16], b3[4];

    __device__ __forceinline__ f32x4 W1q(int ob, int i) const { return as_f32x4(w1[ob][i][lane_id()]); }
    __device__ __forceinline__ f32x4 W2q(int ob, int i) const { return as_f32x4(w2[ob][i][lane_id()]); }
    __device__ __forceinline__ f32x4 W3q(int i) const { return as_f32x4(w3[i][lane_id()]); }
    __device__ __forceinline__ f32x4 B1(int ob) const { return as_f32x4(b1[4 * ob + (lane_id() >> 4)]); }
    __device__ __forceinline__ f32x4 B2(int ob) const { return as_f32x4(b2[4 * ob + (lane_id() >> 4)]); }
    __device__ __forceinline__ f32x4 B3() const { return as_f32x4(b3[lane_id() >> 4]); }
    static __device__ __forceinline__ f32x4 as_f32x4(const float4 &v) { return {v.x, v.y, v.z, v.w}; }
};

__device__ __forceinline__ void store_mlp_f32_shared(const MlpWeights &a, MlpF32Shared &m, int w, int nw)
{
    const int l = lane_id();
    for (int p = w; p < 28; p += nw) {
        if (p < 8) m.w1[p >> 1][p & 1][l] = w1_quad_f32(a, p >> 1, p & 1, l);
        else if (p < 24) m.w2[(p - 8) >> 2][(p - 8) & 3][l] = w2_quad_f32(a, (p - 8) >> 2, (p - 8) & 3, l);
        else m.w3[p - 24][l] = w3_quad_f32(a, p - 24, l);
    }
    if (w == 0) {
        reinterpret_cast<float *>(m.b1)[l] = a.b1[l];
        reinterpret_cast<float *>(m.b2)[l] = a.b2[l];
        if (l < 16) reinterpret_cast<float *>(m.b3)[l] = l < 4 ? a.b3[l] : 0.0f;
    }
}

template <typename M>
__device__ __forceinline__ f32x4 decode_f32(const M &m, const float *f, f32x4 *keep1 = nullptr,
                                            f32x4 *keep2 = nullptr)
{
    f32x4 h1[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = m.B1(ob);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const f32x4 w = m.W1q(ob, i);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[e], f[4 * i + e], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = relu(acc[e]);
        h1[ob] = acc;
        if (keep1) keep1[ob] = acc;
    }
    f32x4 h2[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = m.B2(ob);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const f32x4 w = m.W2q(ob, i);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[e], h1[i][e], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = relu(acc[e]);
        h2[ob] = acc;
        if (keep2) keep2[ob] = acc;
    }
    f32x4 o = m.B3();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const f32x4 w = m.W3q(i);
#pragma unroll
        for (int e = 0; e < 4; ++e) o = __builtin_amdgcn_mfma_f32_16x16x4f32(w[e], h2[i][e], o, 0, 0, 0);
    }
    return o;
}


}  // namespace hp
