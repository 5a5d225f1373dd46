// common.hpp -- device helpers shared by the libmxp kernels (gfx950 only).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) for the counter-based
// generator, and round-to-nearest-even conversions into the storage and
// operand formats, written with integer operations on the IEEE encodings.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MXP_DEV __device__ __forceinline__

namespace mxp {

// ------------------------------------------------------------------ formats
enum Dtype : int { F64 = 0, F32 = 1, F16 = 2, BF16 = 3, F8 = 4 };

typedef _Float16 half_t;
typedef uint16_t bf16_t;  // raw bfloat16 bits
typedef uint8_t f8_t;     // raw e4m3fn bits

// ------------------------------------------------------------------ Philox
struct PhiloxKeys {
    uint32_t k0[10], k1[10];  // round keys: key + r * Weyl constants
};

// a ^ b ^ c in one gfx950 three-input bitwise instruction (truth table 0x96)
MXP_DEV uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); }

// The Philox S-box: two 32x32->64 multiplies, the high halves xor-ed into
// the other lanes with the round key, the low halves carried over.
MXP_DEV void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0, uint32_t k1) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
}

// keys for all ten rounds from the 64-bit seed (k0 = low half, k1 = high half)
MXP_DEV void philox_keys(uint64_t seed, uint32_t k0[10], uint32_t k1[10]) {
    uint32_t a = (uint32_t)seed, b = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        k0[r] = a + (uint32_t)r * 0x9E3779B9u;
        k1[r] = b + (uint32_t)r * 0xBB67AE85u;
    }
}

// four 32-bit words for counter (c0, c1, stream, 0)
MXP_DEV void philox4(uint32_t c0, uint32_t c1, uint32_t stream, const uint32_t k0[10], const uint32_t k1[10],
                     uint32_t out[4]) {
    uint32_t x0 = c0, x1 = c1, x2 = stream, x3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) philox_round(x0, x1, x2, x3, k0[r], k1[r]);
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// signed offset of a draw: k - 2^31, so that the value is s * 2^-32 exactly
MXP_DEV int32_t draw_offset(uint32_t k) { return (int32_t)(k ^ 0x80000000u); }

MXP_DEV double draw_value(uint32_t k) { return (double)draw_offset(k) * 0x1p-32; }

// ------------------------------------------------------------------ RNE conversions
// Round a finite double to a binary format with `mbits` stored fraction bits,
// exponent bias `bias`, minimum normal exponent 1-bias; returns the encoded
// bits (sign at bit 1+ebits+mbits-1).  Overflow -> infinity encoding.
template <int EBITS, int MBITS>
MXP_DEV uint32_t rne_from_f64(double d) {
    const int bias = (1 << (EBITS - 1)) - 1;
    uint64_t u = (uint64_t)__double_as_longlong(d);
    uint32_t sign = (uint32_t)(u >> 63) << (EBITS + MBITS);
    int e = (int)((u >> 52) & 0x7FF);
    uint64_t m = u & ((1ull << 52) - 1);
    if (e == 0x7FF) return sign | (((1u << EBITS) - 1) << MBITS) | (m ? (1u << (MBITS - 1)) : 0u);
    if (e == 0) return sign;  // double subnormals underflow to zero in every target format
    m |= (1ull << 52);
    int ex = e - 1023;        // value = m * 2^(ex - 52)
    int emin = 1 - bias;
    int shift;                // bits dropped from m
    uint32_t efield;
    if (ex >= emin) {
        shift = 52 - MBITS;
        efield = (uint32_t)(ex + bias);
    } else {
        shift = 52 - MBITS + (emin - ex);
        efield = 0;
    }
    if (shift > 63) return sign;
    uint64_t q = m >> shift;
    uint64_t rem = m & ((1ull << shift) - 1);
    uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) q += 1;
    uint32_t bits;
    if (efield == 0) {
        bits = (uint32_t)q;  // subnormal; may round up into the smallest normal (correct encoding)
    } else {
        // q in [2^MBITS, 2^(MBITS+1)]; carry into the exponent when it reaches 2^(MBITS+1)
        if (q >> (MBITS + 1)) { q >>= 1; efield += 1; }
        if (efield >= (uint32_t)((1 << EBITS) - 1)) return sign | (((1u << EBITS) - 1) << MBITS);
        bits = (efield << MBITS) | ((uint32_t)q & ((1u << MBITS) - 1));
    }
    return sign | bits;
}

MXP_DEV uint16_t f64_to_f16_bits(double d) { return (uint16_t)rne_from_f64<5, 10>(d); }
MXP_DEV uint16_t f64_to_bf16_bits(double d) { return (uint16_t)rne_from_f64<8, 7>(d); }

// FP32 -> bf16 with round-to-nearest-even (finite inputs; NaN kept quiet)
MXP_DEV uint16_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

MXP_DEV float bf16_bits_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// FP32 -> fp8 e4m3fn, round to nearest even, saturating at +-448.
MXP_DEV uint8_t f32_to_e4m3_sat(float f) {
    uint32_t u = __float_as_uint(f);
    uint32_t sign = (u >> 24) & 0x80u;
    uint32_t a = u & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return (uint8_t)(sign | 0x7Fu);  // NaN
    if (a >= 0x43E00000u) return (uint8_t)(sign | 0x7Eu);  // |f| >= 448 (incl. inf): saturate
    int e = (int)(a >> 23);          // biased fp32 exponent
    uint32_t m = (a & 0x7FFFFFu) | (e ? 0x800000u : 0u);
    int ex = e - 127;                // unbiased (normal inputs)
    if (e == 0) return (uint8_t)sign; // fp32 subnormal -> 0 (far below e4m3 range)
    int shift;
    uint32_t efield;
    if (ex >= -6) { shift = 20; efield = (uint32_t)(ex + 7); }
    else { shift = 20 + (-6 - ex); efield = 0; }
    if (shift > 24) return (uint8_t)sign;  // below half the smallest subnormal (2^-10)
    uint32_t q = m >> shift;
    uint32_t rem = m & ((1u << shift) - 1);
    uint32_t half = 1u << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) q += 1;
    uint32_t bits;
    if (efield == 0) {
        bits = q;                    // subnormal (or carried into the first normal)
    } else {
        if (q >> 4) { q >>= 1; efield += 1; }
        bits = (efield << 3) | (q & 7u);
        if (bits > 0x7Eu) bits = 0x7Eu;  // rounding up past 448 saturates
    }
    return (uint8_t)(sign | bits);
}

MXP_DEV float e4m3_bits_to_f32(uint8_t b) {
    uint32_t s = (b & 0x80u) ? 0x80000000u : 0u;
    uint32_t e = (b >> 3) & 0xFu, m = b & 7u;
    if (e == 0) return __uint_as_float(s) + (s ? -1.0f : 1.0f) * (float)m * 0x1p-9f;
    return __uint_as_float(s | ((e - 7 + 127) << 23) | (m << 20));
}

// storage loads / stores -----------------------------------------------------
template <int ST> struct Store;
template <> struct Store<F64> {
    typedef double T;
    static MXP_DEV float load(const T* p, int64_t i) { return (float)p[i]; }
    static MXP_DEV T from_f64(double d) { return d; }
    static MXP_DEV T from_f32(float f) { return f; }
    static constexpr int scale_exp = 0;
    static constexpr bool scaled = false;
};
template <> struct Store<F32> {
    typedef float T;
    static MXP_DEV float load(const T* p, int64_t i) { return p[i]; }
    static MXP_DEV T from_f64(double d) { return (float)d; }  // v_cvt_f32_f64: RNE
    static MXP_DEV T from_f32(float f) { return f; }
    static constexpr int scale_exp = 0;  // no power-of-two scaling needed
    static constexpr bool scaled = false;
};
template <> struct Store<F16> {
    typedef half_t T;
    static MXP_DEV float load(const T* p, int64_t i) { return (float)p[i]; }
    static MXP_DEV T from_f64(double d) { uint16_t b = f64_to_f16_bits(d); return *(half_t*)&b; }
    static MXP_DEV T from_f32(float f) { return (half_t)f; }  // v_cvt_f16_f32: RNE
    static constexpr int scale_exp = 15;
    static constexpr bool scaled = true;
};
template <> struct Store<BF16> {
    typedef bf16_t T;
    static MXP_DEV float load(const T* p, int64_t i) { return bf16_bits_to_f32(p[i]); }
    static MXP_DEV T from_f64(double d) { return f64_to_bf16_bits(d); }
    static MXP_DEV T from_f32(float f) { return f32_to_bf16_bits(f); }
    static constexpr int scale_exp = 0;
    static constexpr bool scaled = false;
};

// operand formats of the trailing update (element types as stored in the
// K-major operand buffers) ------------------------------------------------
template <int OP> struct Operand;
template <> struct Operand<F32> {
    typedef float T;
    static constexpr int scale_exp = 0;
    static constexpr bool scaled = false;
    static MXP_DEV T from_f32(float f) { return f; }
};
template <> struct Operand<F16> {
    typedef half_t T;
    static constexpr int scale_exp = 15;  // amax scaled into (2^14, 2^15]
    static constexpr bool scaled = true;
    static MXP_DEV T from_f32(float f) { return (half_t)f; }
};
template <> struct Operand<BF16> {
    typedef bf16_t T;
    static constexpr int scale_exp = 0;
    static constexpr bool scaled = false;
    static MXP_DEV T from_f32(float f) { return f32_to_bf16_bits(f); }
};
template <> struct Operand<F8> {
    typedef f8_t T;
    static constexpr int scale_exp = 8;   // amax scaled into (128, 256], below 448
    static constexpr bool scaled = true;
    static MXP_DEV T from_f32(float f) { return f32_to_e4m3_sat(f); }
};

// power-of-two scale 2^(target - ceil(log2 amax)); 1 for amax == 0 / non-finite
MXP_DEV float pow2_scale(float amax, int target) {
    if (!(amax > 0.0f) || !(amax < 3.0e38f)) return 1.0f;
    int e;
    float fr = frexpf(amax, &e);  // amax = fr * 2^e, fr in [0.5, 1): ceil(log2 amax) = e, or e-1 if fr == 0.5
    int c = (fr == 0.5f) ? e - 1 : e;
    int p = target - c;
    if (p > 126) p = 126;
    if (p < -126) p = -126;
    return ldexpf(1.0f, p);
}

// ------------------------------------------------------------------ cross-work-group hand-over
// Kernels that hand data from one work-group to another (the diagonal-block
// LU, the dataflow substitution) write and read every shared value with
// agent-scope atomic accesses: on gfx950 these go to the device's coherence
// point (sc1), past any cache that could hold a stale or unwritten copy.
// The producer then waits until all of its stores are acknowledged
// (s_waitcnt vmcnt(0)) before it raises the flag or counter; the consumer
// issues its data loads only after its load of the flag has returned.  That
// is the whole of an agent-scope release / acquire for data that never sits
// in a non-coherent cache: the compiler's release fence adds a write-back of
// the XCD's L2 (buffer_wbl2) and its acquire fence an L2 invalidation
// (buffer_inv), which matter only for ordinary cached stores and loads.
// With MXP_SYNC = 2 the kernels use those fences (release and acquire in
// the language's memory model); measured on the MI355X they cost 9 % of the
// n = 32768 solve (327 vs 359 TFLOP/s: the write-backs also disturb the
// concurrent trailing update), so the default is the hardware form above.
#ifndef MXP_SYNC
#define MXP_SYNC 0
#endif
// before a flag or counter publishes this thread's stores to other work-groups
MXP_DEV void sync_release() {
#if MXP_SYNC >= 1
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#else
    __builtin_amdgcn_s_waitcnt(0);
#endif
}
// after a flag or counter seen set, before the published data is read
MXP_DEV void sync_acquire() {
#if MXP_SYNC >= 2
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#endif
}

// ------------------------------------------------------------------ reductions
MXP_DEV double warp_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
MXP_DEV double warp_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
MXP_DEV float warp_maxf(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

}  // namespace mxp
