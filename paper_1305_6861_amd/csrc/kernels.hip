// Spin-stepping kernels for gfx950 (CDNA4).
//
// Mapping: one workgroup = 4 wave64s; every lane owns S spins, held in
// registers for the whole sequence.  Spin i of a workgroup's tile lives in
// lane (i % 64), slot (i / 64) % S of wave i / (64 S), so every per-slot load
// of the structure-of-arrays object is a coalesced 256-byte row.
//
// The compiled sequence (ps_ops.h) is streamed through LDS in chunks of
// kOpChunk operations; every wave reads the same record (LDS broadcast), so
// all control flow is wave-uniform.  Shaped-pulse rotation tables are staged
// into LDS once per workgroup.
//
// Readout (section 5.1.1: one sub-step per sample, magnetisation recorded
// after each): inside an ADC interval a spin's transverse magnetisation is
// a geometric sequence p_n = p_0 z^n with z = E2(tau) exp(-j 2 pi (mu.x +
// dw tau / 2 pi)), because precession about z and T2 decay compose by
// adding phases and times (eq. 3.5 / 3.14).  p_0, z and Z = z^32 come from
// FP64 phases reduced modulo one revolution; the FP32 recurrence p <- p z
// runs for at most 31 steps before it is re-anchored from p <- p Z, so its
// rounding grows like (31 + n/32) ulps instead of n ulps.
//
// Readouts are split across waves by sample chunk instead of by spin: the
// G waves of a wave group publish their spins' readout anchors in LDS, and
// wave g of the group then runs chunks g, g + G, g + 2G, ... (32 samples
// each) for all G * S spins of the group.  Each lane thus sums G * S spins
// per sample, the butterfly cost is shared by that many spins, and no
// cross-wave reduction or barrier sits inside the sample loop.
//
// Inside a chunk the samples are taken in blocks of M = 4: a spin adds p,
// p z, p z^2, p z^3 (powers from FP64 phases, held in registers) to the
// lane's four sample sums as complex multiply-accumulates, then steps
// p <- p z^4.
//
// Per-sample superposition (eq. 3.32): each lane first sums its G * S
// spins, then a butterfly over 32 consecutive samples (64 reals) reduces the
// 64 lanes with permlane32/16 swaps and DPP, and the wave writes the partial
// sum each lane ends with into its wave group's row.  A second kernel sums
// all rows in FP64 in row order.  Every order is fixed, so results are
// bitwise reproducible for a given tiling.
//
// Matrix-core readout (FP32, one spin per lane, readouts the host flags
// OPF_MATRIX): with sample t = 16 b + j of a 128-sample tile, the signal is
//   s(16 b + j) = sum_n (m_n z_n^(16 b)) z_n^j,
// a complex matrix product over the spins n of (8 x N) and (N x 16), where
// m_n is the spin's value at the tile's first sample.  Written with real
// operands (rows (b, re/im), two contraction slots (re, im) per spin) it is
// one v_mfma_f32_16x16x4_f32 per two spins and tile.  The factors z^j and
// z^(16 b) depend only on the spin and the readout's per-sample step, so
// they are built once per step and kept in registers: z^j in the B operand's
// layout, z^(16 b) for the lane's own spin.  Per tile each lane forms its
// spin's eight a_b = m z^(16 b) and stores them (Re, Im, -Im: the three
// entries the real form of a complex product needs) in the wave's LDS tile,
// from which the A operands are read four MFMAs at a time.  The waves'
// 16 x 16 results are added in LDS in wave order (two tiles of a readout per
// barrier), and one row per workgroup is written, as in the vector path.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "ps_kernels.h"
#include "ps_ops.h"

namespace ps {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kOpChunk = 32;
constexpr int kT = 32;  // samples per reduction chunk (64 reals -> 64 lanes)

// Samples per readout block.  Inside a block of M samples a spin adds
// p z^m (m = 0 .. M-1) to the sample sums, with z^m precomputed, and only
// then steps p <- p z^M: a complex multiply-accumulate is 4 FMAs, so a
// sample costs 4 + 2 / M instructions per spin instead of 6 (multiply, then
// add).  The powers take registers, so FP64 keeps the plain recurrence.
template <typename real> struct ReadoutBlock { static constexpr int M = 4; };
template <> struct ReadoutBlock<double> { static constexpr int M = 2; };
static_assert(kT % ReadoutBlock<float>::M == 0, "a chunk holds whole readout blocks");

// 16-byte LDS vectors of the readout step factors
template <typename real> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int V = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int V = 2; };

// A device pointer of StepArgs as a pointer into global memory.  The batched
// kernel reads its arguments from a request record, and the compiler cannot
// tell where such pointers point: without this it accesses them with flat
// instructions, and an outstanding flat store also holds up every later wait
// for LDS data.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// A value of a partial-sum row: each is written once and read once, by the
// finalize after the whole launch, so the store is nontemporal (a slice's
// rows are far larger than the caches and would only displace what the
// step kernel reads again).
template <typename T, typename V>
__device__ __forceinline__ void put_partial(__attribute__((address_space(1))) T* p, V v) {
    __builtin_nontemporal_store((T)v, p);
}

constexpr double kLog2e = 1.4426950408889634073599246810019;
constexpr double kInv2Pi = 0.15915494309189533576888376337251;

// ---------------------------------------------------------------------------
// precision-dependent helpers
// ---------------------------------------------------------------------------
template <typename real> struct Math;

template <> struct Math<float> {
    // exp(-t r) for t, r >= 0: the base-2 exponent is formed in FP64 and split
    // into an exact integer part and a fraction in [-1/2, 1/2], so rounding of
    // a large exponent does not turn into a relative error of the result.
    static __device__ __forceinline__ float expneg(double t, double r) {
        double a = fmax(-t * r * kLog2e, -250.0);
        double i = rint(a);
        float f = (float)(a - i);
        return ldexpf(__builtin_amdgcn_exp2f(f), (int)i);
    }
    // 1 - exp(-x), x = t r >= 0, formed without cancellation (for x << 1 the
    // FP32 difference 1 - exp(-x) would keep only a few significant bits):
    // below 1/2 the Taylor series of 1 - e^-x to x^8 (truncation below
    // 1.5e-8 relative), above it 1 - 2^(-x log2 e) from the hardware exp2
    // (e^-x <= 0.61 there, so its error stays relative).  Both are cheaper
    // than the library expm1f, which handles the whole range.
    static __device__ __forceinline__ float one_minus_expneg(double t, double r) {
        const float x = (float)(t * r);
        float p = fmaf(x, -1.0f / 40320.0f, 1.0f / 5040.0f);
        p = fmaf(x, -p, 1.0f / 720.0f);
        p = fmaf(x, -p, 1.0f / 120.0f);
        p = fmaf(x, -p, 1.0f / 24.0f);
        p = fmaf(x, -p, 1.0f / 6.0f);
        p = fmaf(x, -p, 0.5f);
        p = fmaf(x, -p, 1.0f);
        p *= x;
        const float q = 1.0f - __builtin_amdgcn_exp2f(-x * (float)kLog2e);
        return x < 0.5f ? p : q;
    }
    // cos and sin of 2 pi c for a phase c in revolutions (FP64), reduced to
    // [-1/2, 1/2] in FP64 before rounding to FP32, then evaluated by the
    // hardware sine/cosine, which take revolutions.  Measured on gfx950 over
    // [-1/2, 1/2]: max abs error 1.25e-7 with zero mean (FP64 reference).
    static __device__ __forceinline__ void cis(double c, float& co, float& si) {
        const float f = (float)(c - rint(c));
        co = __builtin_amdgcn_cosf(f);
        si = __builtin_amdgcn_sinf(f);
    }
};

template <> struct Math<double> {
    static __device__ __forceinline__ double expneg(double t, double r) { return exp(-t * r); }
    static __device__ __forceinline__ double one_minus_expneg(double t, double r) { return -expm1(-t * r); }
    static __device__ __forceinline__ void cis(double c, double& co, double& si) {
        double f = c - rint(c);
        sincospi(2.0 * f, &si, &co);
    }
};

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Tables of the matrix-core readout held by each lane (one spin per lane;
// see the file comment).  MFMA q (q = 0 .. 31) of a tile takes the spins of
// lanes q and q + 32; lane l supplies operand A[i][k] with i = l & 15 (row
// (b, p) = (i >> 1, i & 1)) and k = l >> 4 (spin lane q + 32 (k >> 1),
// component c = k & 1), and operand B[k][j] with j = l & 15:
//   A = row (b, p), slot c of a_b: Re a_b for p == c, -Im a_b for
//       (p, c) = (0, 1), Im a_b for (1, 0);
//   bq[q] = component c of z^j of that spin.
// (wr, wi)[b] = z^(16 b) (b = 1 .. 7) and (zr, zi) = z^128 belong to the
// lane's own spin.
template <bool On> struct MatrixTables {};
template <> struct MatrixTables<true> {
    float bq[32];
    float wr[8], wi[8];
    float zr, zi;
};
// The A-operand tile of a wave in LDS: rows (h, b, v) for the spins of
// lanes 32 h .. 32 h + 31 (v = 0: Re a_b, 1: Im a_b, 2: -Im a_b), 32 columns
// (one per spin); column q is stored at q ^ (4 (row & 7)), which keeps each
// 4-column group contiguous and spreads the 16 rows a 16-lane read touches
// over the LDS banks.
constexpr int kMatrixARows = 2 * 8 * 3;

// ---------------------------------------------------------------------------
// wave-wide transpose-reduce of 64 values per lane -> 1 value per lane
// (lane l ends with the sum over all 64 lanes of input value l)
// ---------------------------------------------------------------------------
// The patterns used here (row mirrors, quad permutes) read a valid lane for
// every lane, so bound_ctrl changes no value; set, it lets the compiler fold
// the move into the consuming add (one v_add_f32 with a DPP source).
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL, int BIT, int HALF, int N>
__device__ __forceinline__ void dpp_stage(float (&v)[N], int lane) {
    const bool upper = (lane & BIT) != 0;
#pragma unroll
    for (int i = 0; i < HALF; ++i) {
        const float lo = v[i] + dpp<CTRL>(v[i]);             // both lanes of a pair sum value i
        const float hi = v[i + HALF] + dpp<CTRL>(v[i + HALF]);
        v[i] = upper ? hi : lo;
    }
}

__device__ __forceinline__ float wave_reduce64(float (&v)[64], int lane) {
    // lanes l and l^32: swap halves of the wave
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 32]),
                                                  false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    // lanes l and l^16: swap odd and even 16-lane rows
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 16]),
                                                  false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    dpp_stage<0x140, 8, 8>(v, lane);  // row_mirror: l <-> 15 - l within a row
    dpp_stage<0x141, 4, 4>(v, lane);  // row_half_mirror: l <-> 7 - l within 8
    dpp_stage<0x4E, 2, 2>(v, lane);   // quad_perm [2,3,0,1]: l <-> l ^ 2
    dpp_stage<0xB1, 1, 1>(v, lane);   // quad_perm [1,0,3,2]: l <-> l ^ 1
    return v[0];
}

// Readout form of the same reduction, for a chunk of 32 samples produced
// as four quarters of 8: each quarter's 16 values (v[2 s + c] = component c
// of its sample s) are halved twice right away, across lane bits 5 and 4,
// so that only 4 values per quarter stay live; the 16 values left then go
// through lane bits 3 .. 0.  Lane l ends with the wave sum of component
// l & 1 of chunk sample readout_sample_of_lane(l).
__device__ __forceinline__ int readout_sample_of_lane(int lane) {
    return ((lane >> 1) & 1) | (((lane >> 4) & 1) << 1) | (((lane >> 5) & 1) << 2) |
           (((lane >> 2) & 1) << 3) | (((lane >> 3) & 1) << 4);
}

template <int H>
__device__ __forceinline__ void perm32_stage(float (&v)[16]) {   // value i vs i + H across lanes l, l ^ 32
#pragma unroll
    for (int i = 0; i < H; ++i) {
        auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + H]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
}

template <int H>
__device__ __forceinline__ void perm16_stage(float (&v)[16]) {   // value i vs i + H across lanes l, l ^ 16
#pragma unroll
    for (int i = 0; i < H; ++i) {
        auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + H]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
}

__device__ __forceinline__ void quarter_reduce(float (&v)[16], int) {
    perm32_stage<8>(v);
    perm16_stage<4>(v);
}

__device__ __forceinline__ float reduce16(float (&v)[16], int lane) {
    dpp_stage<0x140, 8, 8>(v, lane);
    dpp_stage<0x141, 4, 4>(v, lane);
    dpp_stage<0x4E, 2, 2>(v, lane);
    dpp_stage<0xB1, 1, 1>(v, lane);
    return v[0];
}

// value i vs i + H across lanes l, l ^ D (FP64)
template <int D, int H, int N>
__device__ __forceinline__ void xor_stage_h(double (&v)[N], int lane) {
    const bool upper = (lane & D) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        double send = upper ? v[i] : v[i + H];
        double keep = upper ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, D, 64);
    }
}

// The FP64 readout butterfly takes the same lane exchanges as the FP32 one,
// each applied to the two 32-bit halves of a value (lane swaps and DPP
// moves are pure data movement), so lane l ends with the same sample.
__device__ __forceinline__ double join_halves(uint32_t lo, uint32_t hi) {
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | (uint64_t)lo));
}

template <int H>
__device__ __forceinline__ void perm32_stage(double (&v)[16]) {   // value i vs i + H across lanes l, l ^ 32
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const uint64_t a = (uint64_t)__double_as_longlong(v[i]), b = (uint64_t)__double_as_longlong(v[i + H]);
        auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
        auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
        v[i] = join_halves(lo[0], hi[0]) + join_halves(lo[1], hi[1]);
    }
}

template <int H>
__device__ __forceinline__ void perm16_stage(double (&v)[16]) {   // value i vs i + H across lanes l, l ^ 16
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const uint64_t a = (uint64_t)__double_as_longlong(v[i]), b = (uint64_t)__double_as_longlong(v[i + H]);
        auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)b, false, false);
        auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
        v[i] = join_halves(lo[0], hi[0]) + join_halves(lo[1], hi[1]);
    }
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return join_halves(lo, hi);
}

template <int CTRL, int BIT, int HALF>
__device__ __forceinline__ void dpp_stage(double (&v)[16], int lane) {
    const bool upper = (lane & BIT) != 0;
#pragma unroll
    for (int i = 0; i < HALF; ++i) {
        const double lo = v[i] + dpp<CTRL>(v[i]);
        const double hi = v[i + HALF] + dpp<CTRL>(v[i + HALF]);
        v[i] = upper ? hi : lo;
    }
}

__device__ __forceinline__ void quarter_reduce(double (&v)[16], int) {
    perm32_stage<8>(v);
    perm16_stage<4>(v);
}

__device__ __forceinline__ double reduce16(double (&v)[16], int lane) {
    dpp_stage<0x140, 8, 8>(v, lane);
    dpp_stage<0x141, 4, 4>(v, lane);
    dpp_stage<0x4E, 2, 2>(v, lane);
    dpp_stage<0xB1, 1, 1>(v, lane);
    return v[0];
}

template <int D>
__device__ __forceinline__ void xor_stage(double (&v)[64], int lane) {
    const bool upper = (lane & D) != 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double send = upper ? v[i] : v[i + D];
        double keep = upper ? v[i + D] : v[i];
        v[i] = keep + __shfl_xor(send, D, 64);
    }
}

__device__ __forceinline__ double wave_reduce64(double (&v)[64], int lane) {
    xor_stage<32>(v, lane);
    xor_stage<16>(v, lane);
    xor_stage<8>(v, lane);
    xor_stage<4>(v, lane);
    xor_stage<2>(v, lane);
    xor_stage<1>(v, lane);
    return v[0];
}

// ---------------------------------------------------------------------------
// the stepper
// ---------------------------------------------------------------------------
// Waves that share their spins during readouts (see the file comment):
// the readout works on G * S spins per lane.
template <int S>
struct ReadoutShare {
    static constexpr int G = S <= 2 ? 4 : (S == 4 ? 2 : 1);
};

// Readout step factors of a spin, as complex numbers c = 0 .. NC - 1:
// z^(c + 1) for c < M (one sample to a block of M), then z^(32 g) for
// g = 1 .. G - 1 (the chunk offsets of a wave group), then W = z^(32 G)
// (the stride of a wave's chunks); NF reals, padded to whole LDS vectors.
template <typename real, int S>
struct StepFactors {
    static constexpr int M = ReadoutBlock<real>::M;
    static constexpr int G = ReadoutShare<S>::G;
    static constexpr int V = Vec16<real>::V;
    static constexpr int kZ = 0, kZg = M, kW = M + G - 1, NC = M + G;
    static constexpr int NF = (2 * NC + V - 1) / V * V;
};

int64_t rows_per_block_of(int spins_per_lane) {
    switch (spins_per_lane) {
        case 1: return kWaves / ReadoutShare<1>::G;
        case 2: return kWaves / ReadoutShare<2>::G;
        case 4: return kWaves / ReadoutShare<4>::G;
        default: return kWaves / ReadoutShare<8>::G;
    }
}

template <typename real, int S>
struct Spins {
    float x[S], y[S], z[S], dw[S], m0[S];
    double r1[S], r2[S];     // 1/T1, 1/T2 (0 for +inf)
    real ar[S], ai[S], az[S];  // anchors: Mxy_a = ar + j ai, Mz_a = az
};

// A wave-uniform FP64 value (read from LDS into vector registers) moved to
// scalar registers.
__device__ __forceinline__ double uniform(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(lo | (hi << 32)));
}

// Phase of a spin in revolutions: k.x + (dw / 2 pi) t.
__device__ __forceinline__ double phase_rev(const double* k, double t, float x, float y, float z,
                                            float dw) {
    return fma(k[0], (double)x, fma(k[1], (double)y, fma(k[2], (double)z, (double)dw * kInv2Pi * t)));
}

// Relaxation factors of the lane's spin kept for the time they were last
// formed for (the matrix-only kernel, one spin per lane): a sequence that
// repeats its timing (every repetition of a Cartesian scan) forms them once.
// A kept factor is the one the same computation gives, so results do not
// change.  The keys are the times' bit patterns, compared on the scalar unit
// (it has no FP64 compare).
template <bool On> struct DecayCache {};
template <> struct DecayCache<true> {
    uint64_t t1_key = ~0ull, t2_key = ~0ull;  // bit patterns of wave-uniform times (a NaN: no time yet)
    float d1 = 0.0f, e2 = 0.0f;              // 1 - exp(-t1 / T1), exp(-t2 / T2) for those times
};

template <typename real, int S, bool C>
__device__ __forceinline__ real one_minus_e1(const Spins<real, S>& sp, int s, double t, DecayCache<C>* dc) {
    if constexpr (C) {
        const uint64_t key = (uint64_t)__double_as_longlong(t);
        if (key != dc->t1_key) {
            dc->d1 = Math<real>::one_minus_expneg(t, sp.r1[s]);
            dc->t1_key = key;
        }
        return dc->d1;
    } else {
        return Math<real>::one_minus_expneg(t, sp.r1[s]);
    }
}

template <typename real, int S, bool C>
__device__ __forceinline__ real e2_of(const Spins<real, S>& sp, int s, double t, DecayCache<C>* dc) {
    if constexpr (C) {
        const uint64_t key = (uint64_t)__double_as_longlong(t);
        if (key != dc->t2_key) {
            dc->e2 = Math<real>::expneg(t, sp.r2[s]);
            dc->t2_key = key;
        }
        return dc->e2;
    } else {
        return Math<real>::expneg(t, sp.r2[s]);
    }
}

// Magnetisation at the instant described by (k, txy, tz) from the anchors.
template <typename real, int S, bool C = false>
__device__ __forceinline__ void evaluate(const Spins<real, S>& sp, const Op& op, bool mxy_zero,
                                         real (&mx)[S], real (&my)[S], real (&mz)[S],
                                         DecayCache<C>* dc = nullptr) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
        // T1 recovery over tz as Mz_a + (M0 - Mz_a)(1 - E1): in a saturated
        // steady state Mz << M0, and M0 + (Mz_a - M0) E1 would cancel, turning
        // the rounding of E1 into a bias that is the same for this spin in
        // every repetition.
        const real d1 = one_minus_e1<real, S, C>(sp, s, uniform(op.tz), dc);
        const real m0 = (real)sp.m0[s];
        mz[s] = fma(m0 - sp.az[s], d1, sp.az[s]);
        if (mxy_zero) {
            mx[s] = 0; my[s] = 0;
        } else {
            real e2 = e2_of<real, S, C>(sp, s, uniform(op.txy), dc);
            real c, sn;
            Math<real>::cis(phase_rev(op.k, op.txy, sp.x[s], sp.y[s], sp.z[s], sp.dw[s]), c, sn);
            // (ar + j ai) (c - j sn)
            mx[s] = e2 * (sp.ar[s] * c + sp.ai[s] * sn);
            my[s] = e2 * (sp.ai[s] * c - sp.ar[s] * sn);
        }
    }
}

template <typename real>
__device__ __forceinline__ const real* rot_of(const Op& op);
template <> __device__ __forceinline__ const float* rot_of<float>(const Op& op) { return op.u.r32; }
template <> __device__ __forceinline__ const double* rot_of<double>(const Op& op) { return op.u.r64; }

// Hard pulse (eq. 3.19) applied as M <- M + D M with D = R - I (host-built
// without cancellation): a near-identity rotation then loses nothing to the
// rounding of cos(alpha) ~ 1, and the rounding that is left is the final
// addition, which differs from spin to spin instead of biasing them all.
template <typename real, int S>
__device__ __forceinline__ void rotate(const real* D, real (&mx)[S], real (&my)[S], real (&mz)[S]) {
    const real d00 = D[0], d01 = D[1], d02 = D[2], d10 = D[3], d11 = D[4], d12 = D[5],
               d20 = D[6], d21 = D[7], d22 = D[8];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        real a = mx[s], b = my[s], c = mz[s];
        mx[s] = fma(d00, a, fma(d01, b, fma(d02, c, a)));
        my[s] = fma(d10, a, fma(d11, b, fma(d12, c, b)));
        mz[s] = fma(d20, a, fma(d21, b, fma(d22, c, c)));
    }
}

// Precession + T2 decay factor of one sub-step minus one, u - 1 with
// u = E2(tau) exp(-j 2 pi c), formed in FP64 without cancellation:
// Re(u - 1) = expm1(-tau/T2) - 2 E2 sin^2(pi c), Im(u - 1) = -E2 sin(2 pi c).
template <typename real>
__device__ __forceinline__ void step_delta(double c, double tau, double r2, real& dr, real& di) {
    const double f = c - rint(c);
    double s1, c1;
    sincospi(f, &s1, &c1);
    const double em1 = expm1(-tau * r2);
    const double e2 = 1.0 + em1;
    dr = (real)(em1 - 2.0 * e2 * s1 * s1);
    di = (real)(-2.0 * e2 * s1 * c1);
}

// LDS of a step workgroup outside the dynamic part (s_ops, s_x below).
template <typename real, int S, int VAR = STEP_GENERAL>
struct MatrixReadout {
    static constexpr bool on = std::is_same<real, float>::value && S == 1 && VAR != STEP_VECTOR_ONLY;
    static constexpr int LW = on ? kWaves : 1;   // LDS extents (1 when off)
};

template <typename real, int S, int VAR = STEP_GENERAL>
constexpr size_t static_lds_bytes() {
    constexpr int G = ReadoutShare<S>::G;
    constexpr int NF = StepFactors<real, S>::NF;
    // the matrix-core arrays exist only where that readout does (the
    // compiler drops the placeholders of the other kernels)
    constexpr size_t matrix = MatrixReadout<real, S, VAR>::on
                                  ? sizeof(float) * kWaves * kMatrixARows * 32 + sizeof(float4) * 4 * kWaves * 64
                                  : 0;
    return sizeof(Op) * kOpChunk + sizeof(real) * 2 * (G > 1 ? kWaves : 1) * (G > 1 ? S : 1) * 64 * 2 +
           sizeof(real) * S * NF * kBlock + sizeof(real) * (G > 1 ? kWaves : 1) * 64 + matrix;
}

// Shaped-pulse propagator of every spin of this lane (see ps_ops.h): the
// sub-steps of the direct path are applied in FP64 to the three columns of
// the identity (the linear part A) and to the zero vector with the T1 source
// term (the offset b), and the result is stored, narrowed to real, into the
// lane's slot entries: entry k of spin s at cache[(k * S + s) * kBlock].
// Calls f(std::integral_constant<int, I>()) for I = B .. E-1: a loop whose
// index is a compile-time constant even where the body holds a run-time loop
// (an unroll pragma may leave such a loop rolled, and a run-time index into
// the per-lane spin arrays would move them to scratch memory).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>());
        static_for<B + 1, E>(f);
    }
}

template <typename real, int S, typename RowPtr>
__device__ __forceinline__ void shape_fill(const Spins<real, S>& sp, const Op& op, RowPtr rows, int n_sub,
                                           real* cache) {
    const double tau = op.u.shape.tau;
    static_for<0, S>([&](auto si) {
        constexpr int s = decltype(si)::value;
        double dur, dui;
        step_delta<double>(phase_rev(op.u.shape.mu, tau, sp.x[s], sp.y[s], sp.z[s], sp.dw[s]), tau, sp.r2[s],
                           dur, dui);
        const double d1 = -expm1(-tau * sp.r1[s]);
        const double m0d = (double)sp.m0[s];
        // vectors 0..2: columns of A; vector 3: b
        double vx[4] = {1.0, 0.0, 0.0, 0.0}, vy[4] = {0.0, 1.0, 0.0, 0.0}, vz[4] = {0.0, 0.0, 1.0, 0.0};
        for (int q = 0; q < n_sub; ++q) {
            double r[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) r[e] = rows[9 * q + e];
            rotate<double, 4>(r, vx, vy, vz);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double a_ = vx[v], b_ = vy[v];
                vx[v] = fma(a_, dur, fma(-b_, dui, a_));
                vy[v] = fma(a_, dui, fma(b_, dur, b_));
                vz[v] = fma(v == 3 ? m0d - vz[v] : -vz[v], d1, vz[v]);
            }
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            cache[((0 + v) * S + s) * kBlock] = (real)vx[v];   // A[0][v]
            cache[((3 + v) * S + s) * kBlock] = (real)vy[v];   // A[1][v]
            cache[((6 + v) * S + s) * kBlock] = (real)vz[v];   // A[2][v]
        }
        cache[(9 * S + s) * kBlock] = (real)vx[3];
        cache[(10 * S + s) * kBlock] = (real)vy[3];
        cache[(11 * S + s) * kBlock] = (real)vz[3];
    });
}

// M <- Rz(phi) (A Rz(-phi) M + b) with (cos phi, sin phi) = (c, sn), from
// the lane's slot entries; turn == false means phi = 0.  With mxy_zero the
// magnetisation is (0, 0, Mz), which Rz(-phi) leaves alone and on which only
// the third column of A acts.
template <typename real, int S>
__device__ __forceinline__ void shape_apply(const real* cache, bool turn, real c, real sn, bool mxy_zero,
                                            real (&mx)[S], real (&my)[S], real (&mz)[S]) {
    if (mxy_zero) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const real z = mz[s];
            const real* e = cache + s * kBlock;
            real nx = fma(e[2 * S * kBlock], z, e[9 * S * kBlock]);
            real ny = fma(e[5 * S * kBlock], z, e[10 * S * kBlock]);
            mz[s] = fma(e[8 * S * kBlock], z, e[11 * S * kBlock]);
            if (turn) {
                const real x0 = nx;
                nx = fma(c, x0, -sn * ny);
                ny = fma(c, ny, sn * x0);
            }
            mx[s] = nx;
            my[s] = ny;
        }
        return;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        real x = mx[s], y = my[s];
        if (turn) {
            const real x0 = x;
            x = fma(c, x0, sn * y);
            y = fma(c, y, -sn * x0);
        }
        const real z = mz[s];
        const real* e = cache + s * kBlock;
        real nx = fma(e[0 * S * kBlock], x, fma(e[1 * S * kBlock], y, fma(e[2 * S * kBlock], z, e[9 * S * kBlock])));
        real ny = fma(e[3 * S * kBlock], x, fma(e[4 * S * kBlock], y, fma(e[5 * S * kBlock], z, e[10 * S * kBlock])));
        mz[s] = fma(e[6 * S * kBlock], x, fma(e[7 * S * kBlock], y, fma(e[8 * S * kBlock], z, e[11 * S * kBlock])));
        if (turn) {
            const real x0 = nx;
            nx = fma(c, x0, -sn * ny);
            ny = fma(c, ny, sn * x0);
        }
        mx[s] = nx;
        my[s] = ny;
    }
}

// Matrix-core readout tables of the lane (MatrixTables) for the per-sample
// step (mu, tau): every factor from its own FP64 phase, the other spins'
// parameters (for the B operand) fetched by lane shuffles.
__device__ __forceinline__ void matrix_tables(const Spins<float, 1>& sp, const double (&mu)[3], double tau, int lane,
                                              MatrixTables<true>& mt) {
    const int j = lane & 15;                 // B: sample inside the block
    const int c = (lane >> 4) & 1;           // contraction slot: component of the spin
    const int half = lane >> 5;
    // the per-sample phase of the lane's own spin (FP64); the B operand takes
    // the other spins' from their lanes
    const double ph = phase_rev(mu, tau, sp.x[0], sp.y[0], sp.z[0], sp.dw[0]);
    {
        auto power = [&](double e, float& re, float& im) {   // z^e of the lane's own spin
            float co, sn;
            Math<float>::cis(ph * e, co, sn);
            const float m = Math<float>::expneg(tau * e, sp.r2[0]);
            re = m * co;
            im = -m * sn;
        };
        mt.wr[0] = 1.0f;
        mt.wi[0] = 0.0f;
#pragma unroll
        for (int b = 1; b < 8; ++b) power(16.0 * b, mt.wr[b], mt.wi[b]);
        power((double)kMatrixTile, mt.zr, mt.zi);
    }
    static_for<0, 32>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const int src = q + 32 * half;
        const double ph_q = __shfl(ph, src), r2 = __shfl(sp.r2[0], src);
        float co, sn;
        Math<float>::cis(ph_q * (double)j, co, sn);
        const float e = Math<float>::expneg(tau * (double)j, r2);
        mt.bq[q] = c == 0 ? e * co : -e * sn;           // component c of z^j
    });
}

// Matrix-core readout of one ADC operation (n samples) for one receive coil
// (weight (wx, wy) when weighted): tiles of kMatrixTile samples; m starts
// each tile from an FP64 phase every kMatrixReanchor tiles and is stepped by
// z^128 in between.  s_a is the wave's A-operand tile; out points at the
// coil's first sample of this operation in the workgroup's row (2 reals per
// sample).  Every wave of the workgroup takes part (one barrier per tile,
// or per pair of tiles inside the readout).
constexpr int kMatrixReanchor = 8;

template <bool C>
__device__ __forceinline__ void matrix_readout(const Spins<float, 1>& sp, const Op& op, const double (&mu)[3],
                                               double tau, int n, bool weighted, float wx, float wy,
                                               const MatrixTables<true>& mt, float* s_a, float4* s_md,
                                               int& m_pass, int wave, int lane,
                                               __attribute__((address_space(1))) float* out, DecayCache<C>* dc) {
    const int n_tiles = (n + kMatrixTile - 1) / kMatrixTile;
    const int half = lane >> 5;
    const int col = lane & 31;
    // this lane's A operand: row (h, b, v) with v from (p, c) (see MatrixTables)
    const int p = lane & 1, c = (lane >> 4) & 1;
    const int a_row = (half * 8 + ((lane & 15) >> 1)) * 3 + (p == c ? 0 : (p == 1 ? 1 : 2));
    const float* a_src = s_a + a_row * 32;
    const int a_swz = 4 * (a_row & 7);
    float mr = 0.0f, mi = 0.0f;
    for (int tile = 0; tile < n_tiles; ++tile) {
        if (tile % kMatrixReanchor == 0) {
            // value at sample s0 from the anchors, as in the vector path
            // (at s0 = 0 the moment and time are the operation's own, exactly)
            double t = uniform(op.txy);
            double k[3] = {uniform(op.k[0]), uniform(op.k[1]), uniform(op.k[2])};
            if (tile > 0) {
                const double s0 = (double)(tile * kMatrixTile);
                t += s0 * tau;
                k[0] += s0 * mu[0];
                k[1] += s0 * mu[1];
                k[2] += s0 * mu[2];
            }
            const float e2 = e2_of<float, 1, C>(sp, 0, t, dc);
            float co, sn;
            Math<float>::cis(phase_rev(k, t, sp.x[0], sp.y[0], sp.z[0], sp.dw[0]), co, sn);
            const float pr = e2 * (sp.ar[0] * co + sp.ai[0] * sn);
            const float pi = e2 * (sp.ai[0] * co - sp.ar[0] * sn);
            if (weighted) {
                mr = fmaf(wx, pr, wy * pi);
                mi = fmaf(wx, pi, -wy * pr);
            } else {
                mr = pr;
                mi = pi;
            }
        } else {
            const float t_ = mr * mt.zr - mi * mt.zi;
            mi = mr * mt.zi + mi * mt.zr;
            mr = t_;
        }
        // this spin's a_b = m z^(16 b) into the wave's tile; LDS operations
        // of a wave complete in order, so the reads below see these writes
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            float re = mr, im = mi, nim = -mi;
            if (b > 0) {
                const float t2 = mi * mt.wr[b], t1 = mi * mt.wi[b];
                re = fmaf(mr, mt.wr[b], -t1);
                im = fmaf(mr, mt.wi[b], t2);
                nim = fmaf(-mr, mt.wi[b], -t2);
            }
            const int r0 = (half * 8 + b) * 3;
            s_a[(r0 + 0) * 32 + (col ^ (4 * ((r0 + 0) & 7)))] = re;
            s_a[(r0 + 1) * 32 + (col ^ (4 * ((r0 + 1) & 7)))] = im;
            s_a[(r0 + 2) * 32 + (col ^ (4 * ((r0 + 2) & 7)))] = nim;
        }
        // the eight operand reads (the compiler issues each just before its
        // four products at this register budget; holding more in flight
        // measured no faster), then one accumulation chain of 32 products
        float4 av[8];
        static_for<0, 8>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            av[g] = *reinterpret_cast<const float4*>(a_src + ((4 * g) ^ a_swz));
        });
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        static_for<0, 8>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].x, mt.bq[4 * g + 0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].y, mt.bq[4 * g + 1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].z, mt.bq[4 * g + 2], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].w, mt.bq[4 * g + 3], acc, 0, 0, 0);
        });
        // lane l holds rows 4 (l >> 4) + r (r = 0 .. 3) of column l & 15,
        // i.e. (re, im) of samples 32 (l >> 4) + (l & 15) and 16 more.  The
        // results go to a ring of four slots; the first tile of a pair inside
        // the readout waits for the second's barrier, after which wave 0
        // sums the first and wave 1 the second.  Barriers come at least
        // every two tiles, so a slot is written again only after a barrier
        // that its readers reached once they had read it.
        const int slot = m_pass % 4;
        ++m_pass;
        s_md[(slot * kWaves + wave) * 64 + lane] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        const bool first_of_pair = (tile & 1) == 0 && tile + 1 < n_tiles;
        if (first_of_pair) continue;
        __syncthreads();
        auto store_tile = [&](int sl, int t) {
            const float4* md = s_md + sl * kWaves * 64;
            float4 v = md[lane];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) {
                const float4 u = md[w * 64 + lane];
                v.x += u.x; v.y += u.y; v.z += u.z; v.w += u.w;
            }
            const int smp = t * kMatrixTile + 32 * (lane >> 4) + (lane & 15);
            if (smp < n) {
                put_partial(out + 2 * (int64_t)smp, v.x);
                put_partial(out + 2 * (int64_t)smp + 1, v.y);
            }
            if (smp + 16 < n) {
                put_partial(out + 2 * (int64_t)(smp + 16), v.z);
                put_partial(out + 2 * (int64_t)(smp + 16) + 1, v.w);
            }
        };
        if ((tile & 1) == 1) {
            // a pair: the first tile in the previous slot
            if (wave == 0) store_tile((slot + 3) % 4, tile - 1);
            else if (wave == 1) store_tile(slot, tile);
        } else if (wave < 2) {
            // a single last tile: waves 0 and 1 each store one of its halves
            const float2* md = reinterpret_cast<const float2*>(s_md + slot * kWaves * 64);
            float2 v = md[lane * 2 + wave];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) {
                const float2 u = md[(w * 64 + lane) * 2 + wave];
                v.x += u.x;
                v.y += u.y;
            }
            const int smp = tile * kMatrixTile + 32 * (lane >> 4) + 16 * wave + (lane & 15);
            if (smp < n) {
                put_partial(out + 2 * (int64_t)smp, v.x);
                put_partial(out + 2 * (int64_t)smp + 1, v.y);
            }
        }
    }
}

// One workgroup tile of one request: spins [blk * 256 S, (blk + 1) * 256 S)
// through the slice's operations, partial sums into the tile's rows.
// VAR: the kernel variant (StepVariant).  The matrix-only kernel (MO: FP32,
// S = 1) runs programs whose readouts are all marked OPF_MATRIX, none
// tabulated, all with the step (a.mx_mu, a.mx_tau): it is built without the
// vector and trajectory readouts and builds the tables once, before the
// operations, so that they are loop-invariant and keep their registers
// (tables rebuilt inside the loop make the register allocator move them at
// every readout).  The vector-only kernel (FP32, S = 1) is built without
// the matrix-core readout and sums every readout with the vector path.
template <typename real, int S, int VAR = STEP_GENERAL>
__device__ __forceinline__ void step_body(const StepArgs& a, const int64_t blk, const int rep, const int n_rep) {
    constexpr bool MO = VAR == STEP_MATRIX_ONLY;
    constexpr int G = ReadoutShare<S>::G;
    constexpr int R = G * S;                 // spins per lane inside readouts
    using SF = StepFactors<real, S>;
    constexpr int M = SF::M;
    constexpr int NF = SF::NF;               // step factors per spin (re, im pairs)
    constexpr int V = SF::V;
    using vec_t = typename Vec16<real>::type;
    __shared__ Op s_ops[MO ? 1 : kOpChunk];
    // readout sample-0 values (re, im) handed over inside wave groups, in two
    // buffers used by alternate readout passes
    __shared__ __align__(16) real s_x[2][G > 1 ? kWaves : 1][G > 1 ? S : 1][64][2];
    // readout step factors of every spin of the tile for the (mu, tau) of
    // the last ADC operation (StepFactors), written by the spin's own lane
    // and read by the lanes of its wave group, one 16-byte vector per lane
    __shared__ __align__(16) real s_stepf[S][NF / V][kBlock][V];
    __shared__ real s_red[G > 1 ? kWaves : 1][64];   // chunk sums of waves sharing a chunk
    // matrix-core readout: each wave's A-operand tile, and the waves'
    // 16 x 16 results of a tile, in a ring of four slots (see matrix_readout)
    constexpr bool kMatrix = MatrixReadout<real, S, VAR>::on;
    static_assert(!MO || kMatrix, "the matrix-only kernel is FP32 at one spin per lane");
    constexpr int LW = MatrixReadout<real, S, VAR>::LW;
    constexpr int LR = kMatrix ? kMatrixARows * 32 : 1;
    __shared__ __align__(16) float s_ta[LW][LR];
    __shared__ __align__(16) float4 s_md[4][LW][64];
    extern __shared__ __align__(16) unsigned char s_dyn[];
    // shaped-pulse deltas, FP64: staged in LDS, except in the matrix-only
    // kernel, which reads them (wave-uniform) through the scalar cache and
    // keeps its LDS for a third workgroup per CU
    double* s_rows = reinterpret_cast<double*>(s_dyn);
    const auto c_rows = reinterpret_cast<__attribute__((address_space(4))) const double*>(
        reinterpret_cast<uintptr_t>(a.rows));
    // then the propagator cache: a.n_cache_slots slots of kShapeCacheReals x S
    // x kBlock reals; every lane reads only the entries it wrote itself
    real* s_cache = reinterpret_cast<real*>(s_rows + (MO ? 0 : 9 * a.n_shape_rows));

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t base = (blk * kWaves + wave) * 64 * S;
    __syncthreads();                         // LDS of a previous tile is no longer in use

    Spins<real, S> sp;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t i = base + s * 64 + lane;
        if (i < a.n_spins) {
            sp.x[s] = gmem(a.x)[i]; sp.y[s] = gmem(a.y)[i]; sp.z[s] = gmem(a.z)[i];
            sp.m0[s] = gmem(a.m0)[i]; sp.dw[s] = gmem(a.dw)[i];
            sp.r1[s] = 1.0 / (double)gmem(a.t1)[i];
            sp.r2[s] = 1.0 / (double)gmem(a.t2)[i];
            if (a.load_state) {
                const auto st = gmem(reinterpret_cast<const real*>(a.state)) +
                                (int64_t)(3 * (a.anchor_parity ^ 1)) * a.n_spins;
                sp.ar[s] = st[i]; sp.ai[s] = st[a.n_spins + i]; sp.az[s] = st[2 * a.n_spins + i];
            } else {
                sp.ar[s] = 0; sp.ai[s] = 0; sp.az[s] = (real)sp.m0[s];
            }
        } else {  // padding spin: contributes exactly zero
            sp.x[s] = 0.f; sp.y[s] = 0.f; sp.z[s] = 0.f; sp.m0[s] = 0.f; sp.dw[s] = 0.f;
            sp.r1[s] = 0.0; sp.r2[s] = 0.0;
            sp.ar[s] = 0; sp.ai[s] = 0; sp.az[s] = 0;
        }
    }

    // Propagators filled in an earlier time slice: back from the state into
    // this lane's own cache entries (each lane reads only what it wrote).
    if (a.cache_load) {
        const auto st = gmem(reinterpret_cast<const real*>(a.state));
        for (int slot = 0; slot < kShapeSlots; ++slot) {
            if (!((a.cache_load >> slot) & 1u)) continue;
            real* cache = s_cache + slot * (kShapeCacheReals * S * kBlock) + tid;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int64_t i = base + s * 64 + lane;
#pragma unroll
                for (int e = 0; e < kShapeCacheReals; ++e)
                    cache[(e * S + s) * kBlock] =
                        i < a.n_spins ? st[(kStateSlot0 + kShapeCacheReals * slot + e) * a.n_spins + i] : (real)0;
            }
        }
    }

    // shaped-pulse rotation rows -> LDS (made visible by the first barrier below)
    if constexpr (!MO) {
        const auto rows = gmem(reinterpret_cast<const double*>(a.rows));
        for (int i = tid; i < a.n_shape_rows * 9; i += kBlock) s_rows[i] = rows[i];
    }

    const int wg = wave % G;                 // position inside the wave group
    double step_mu[3] = {0.0, 0.0, 0.0}, step_tau = 0.0;
    int adc_seen = 0;                        // readouts met so far (replica split)
    int x_pass = 0;                          // readout passes met so far (s_x buffer)
    bool step_valid = false;
    DecayCache<MO> dc;                       // relaxation factors kept across repetitions
    MatrixTables<kMatrix> mt;                // valid for (mt_mu, mt_tau) when mt_valid
    double mt_mu[3] = {0.0, 0.0, 0.0}, mt_tau = 0.0;
    bool mt_valid = false;
    int m_pass = 0;                          // matrix tiles met so far (s_md buffer)
    const auto partial = gmem(reinterpret_cast<real*>(a.partial)) +
                    (blk * (kWaves / G) + wave / G) * a.row_stride;
    if constexpr (MO) {
        const double mu0[3] = {a.mx_mu[0], a.mx_mu[1], a.mx_mu[2]};
        matrix_tables(sp, mu0, a.mx_tau, lane, mt);
    }

    // Operation records: staged in LDS a chunk at a time, except in the
    // matrix-only kernel, which loads each (wave-uniform) record through the
    // scalar cache straight into scalar registers: no vector instructions to
    // make its fields uniform, no staging barriers.
    const auto c_ops = reinterpret_cast<__attribute__((address_space(4))) const uint32_t*>(
        reinterpret_cast<uintptr_t>(a.ops));
    for (int c0 = 0; c0 < a.n_ops; c0 += (MO ? a.n_ops : kOpChunk)) {
        const int cn = MO ? a.n_ops : min(kOpChunk, a.n_ops - c0);
        if constexpr (!MO) {
            __syncthreads();
            {
                const auto src = gmem(reinterpret_cast<const uint32_t*>(a.ops + c0));
                uint4* dst = reinterpret_cast<uint4*>(s_ops);
                for (int i = tid; i < cn * 8; i += kBlock)
                    dst[i] = make_uint4(src[4 * i], src[4 * i + 1], src[4 * i + 2], src[4 * i + 3]);
            }
            __syncthreads();
        }

        for (int j = 0; j < cn; ++j) {
            Op op_copy;
            if constexpr (MO) {
                uint32_t* w = reinterpret_cast<uint32_t*>(&op_copy);
#pragma unroll
                for (int i = 0; i < (int)(sizeof(Op) / 4); ++i) w[i] = c_ops[(c0 + j) * (int)(sizeof(Op) / 4) + i];
            }
            const Op& op = MO ? op_copy : s_ops[j];
            const uint32_t kind = __builtin_amdgcn_readfirstlane(op.kind);
            const bool mxy_zero = (__builtin_amdgcn_readfirstlane(op.flags) & OPF_MXY_ZERO) != 0;

            if (kind == OP_RF) {
                real mx[S], my[S], mz[S];
                evaluate<real, S, MO>(sp, op, mxy_zero, mx, my, mz, &dc);
                const real* D = rot_of<real>(op);
                if (mxy_zero) {              // (0, 0, Mz): only the third column of D acts
                    const real d02 = D[2], d12 = D[5], d22 = D[8];
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        sp.ar[s] = d02 * mz[s]; sp.ai[s] = d12 * mz[s]; sp.az[s] = fma(d22, mz[s], mz[s]);
                    }
                    continue;
                }
                rotate<real, S>(D, mx, my, mz);
#pragma unroll
                for (int s = 0; s < S; ++s) { sp.ar[s] = mx[s]; sp.ai[s] = my[s]; sp.az[s] = mz[s]; }
            } else if (kind == OP_SPOIL) {
#pragma unroll
                for (int s = 0; s < S; ++s) { sp.ar[s] = 0; sp.ai[s] = 0; }
            } else if (kind == OP_SNAP) {
                // magnetisation of every spin at this instant (section 7.2);
                // the anchors are left as they are; replica 0 stores it
                if (rep != 0) continue;
                real mx[S], my[S], mz[S];
                evaluate<real, S, MO>(sp, op, mxy_zero, mx, my, mz, &dc);
                const auto out = gmem(reinterpret_cast<real*>(a.snaps)) +
                            (int64_t)__builtin_amdgcn_readfirstlane(op.aux) * 3 * a.n_spins;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const int64_t i = base + s * 64 + lane;
                    if (i < a.n_spins) {
                        out[i] = mx[s]; out[a.n_spins + i] = my[s]; out[2 * a.n_spins + i] = mz[s];
                    }
                }
            } else if (kind == OP_SHAPE) {
                // Shaped pulse (eq. 3.23): n_sub sub-steps, each a hard
                // sub-pulse, precession/decay by u and T1 recovery, all in
                // "operator minus identity" form (see rotate).  The sub-step
                // state is carried in FP64: each sub-step adds a small
                // increment to every component, and in FP32 the roundings of
                // these many small additions are correlated and drift.  With
                // packed FP32 unused, an FP64 FMA issues at the FP32 rate.
                // The rows hold the shape's own phases; the event's RF phase
                // conjugates the whole pulse by Rz (see ps_ops.h).
                real ex[S], ey[S], ez[S];
                evaluate<real, S, MO>(sp, op, mxy_zero, ex, ey, ez, &dc);
                const uint32_t mode = __builtin_amdgcn_readfirstlane(op.u.shape.mode);
                const int n_sub = (int)__builtin_amdgcn_readfirstlane(op.n);
                const int row0 = 9 * (int)__builtin_amdgcn_readfirstlane(op.aux);
                // rows: LDS, or the constant address space in the matrix-only kernel
                auto shaped = [&](auto rows) {
                if (mode != SHAPE_DIRECT) {
                    real* cache = s_cache +
                                  (int)__builtin_amdgcn_readfirstlane(op.u.shape.slot) * (kShapeCacheReals * S * kBlock) +
                                  tid;
                    if (mode == SHAPE_FILL) shape_fill<real, S>(sp, op, rows, n_sub, cache);
                    const double rc = op.u.shape.rot[0], rs = op.u.shape.rot[1];
                    shape_apply<real, S>(cache, rc != 1.0 || rs != 0.0, (real)rc, (real)rs, mxy_zero, ex, ey, ez);
#pragma unroll
                    for (int s = 0; s < S; ++s) { sp.ar[s] = ex[s]; sp.ai[s] = ey[s]; sp.az[s] = ez[s]; }
                    return;
                }
                double mx[S], my[S], mz[S];
                const double tau = op.u.shape.tau;
                const double rc = op.u.shape.rot[0], rs = op.u.shape.rot[1];
                const bool turn = rc != 1.0 || rs != 0.0;
                double dur[S], dui[S], d1[S], m0d[S];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    mx[s] = ex[s]; my[s] = ey[s]; mz[s] = ez[s];
                    if (turn) {                  // Rz(-phi)
                        const double x0 = mx[s];
                        mx[s] = fma(rc, x0, rs * my[s]);
                        my[s] = fma(rc, my[s], -rs * x0);
                    }
                    step_delta<double>(phase_rev(op.u.shape.mu, tau, sp.x[s], sp.y[s], sp.z[s], sp.dw[s]), tau,
                                       sp.r2[s], dur[s], dui[s]);
                    d1[s] = -expm1(-tau * sp.r1[s]);
                    m0d[s] = (double)sp.m0[s];
                }
                for (int q = 0; q < n_sub; ++q) {
                    double r[9];
#pragma unroll
                    for (int e = 0; e < 9; ++e) r[e] = rows[9 * q + e];
                    rotate<double, S>(r, mx, my, mz);
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        const double a_ = mx[s], b_ = my[s];
                        mx[s] = fma(a_, dur[s], fma(-b_, dui[s], a_));
                        my[s] = fma(a_, dui[s], fma(b_, dur[s], b_));
                        mz[s] = fma(m0d[s] - mz[s], d1[s], mz[s]);
                    }
                }
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (turn) {                  // Rz(phi)
                        const double x0 = mx[s];
                        mx[s] = fma(rc, x0, -rs * my[s]);
                        my[s] = fma(rc, my[s], rs * x0);
                    }
                    sp.ar[s] = (real)mx[s]; sp.ai[s] = (real)my[s]; sp.az[s] = (real)mz[s];
                }
                };
                if constexpr (MO) shaped(c_rows + row0);
                else shaped(s_rows + row0);
            } else if (!MO && kind == OP_ADCT) {     // (no tabulated readouts reach MO)
                // Readout at tabulated instants (non-uniform trajectories):
                // every sample is evaluated directly from the anchors,
                //   p_s = Mxy_a E2(t_s) exp(-j 2 pi (k_s . x + dw t_s / 2 pi)).
                // FP64 evaluates the phase from the absolute (k_s, t_s) rows.
                // FP32 splits each 32-sample chunk into blocks of 8: a block's
                // first row gives every spin an FP64 phase and decay, and
                // the block's samples add FP32 offsets (k_s - k_b, t_s - t_b)
                // that the workgroup stages in LDS once per chunk; the
                // offsets stay small, so FP32 keeps the phase to ~1e-7 of a
                // revolution.  FP32 wave groups share their spins (below);
                // otherwise each wave sums its own spins over a chunk and a
                // wave group's waves add their chunk sums in LDS in wave order.
                if (n_rep > 1 && (adc_seen++ % n_rep) != rep) continue;
                const int n = (int)__builtin_amdgcn_readfirstlane(op.n);
                const int aux = (int)__builtin_amdgcn_readfirstlane(op.aux);
                const uint64_t row_u = op.u.tab.row;
                const int64_t row0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(row_u >> 32)) << 32) |
                                               (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)row_u));
                const auto table = gmem(a.traj) + 4 * row0;
                const int n_chunks = (n + kT - 1) / kT;
                real* red = &s_x[0][0][0][0][0];      // G x 64 chunk sums (s_x is free here)
                // FP32 staging of a chunk's rows in the step-factor area, whose
                // cached factors are then no longer valid
                constexpr int kTB = 8;                 // samples per FP64-anchored block
                float4* s_trow = reinterpret_cast<float4*>(&s_stepf[0][0][0][0]);
                double* s_tanc = reinterpret_cast<double*>(s_trow + kT);   // [kT / kTB][4]
                static_assert(sizeof(float4) * kT + sizeof(double) * 4 * (kT / kTB) <= sizeof(s_stepf),
                              "trajectory staging fits the step-factor area");
                step_valid = false;
                float dwf[S], r2l[S];                 // dw / 2 pi and log2(e) / T2 in FP32
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    dwf[s] = (float)((double)sp.dw[s] * kInv2Pi);
                    r2l[s] = (float)(sp.r2[s] * kLog2e);
                }
                const int n_passes = a.n_coils > 0 ? a.n_coils : 1;
                for (int coil = 0; coil < n_passes; ++coil) {
                    real wr[S], wi[S];               // coil-weighted anchors
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        wr[s] = sp.ar[s]; wi[s] = sp.ai[s];
                        if (a.n_coils > 0) {
                            const int64_t i = base + s * 64 + lane;
                            real sx = 0, sy = 0;
                            if (i < a.n_spins) {
                                sx = (real)gmem(a.s_x)[coil * a.n_spins + i];
                                sy = (real)gmem(a.s_y)[coil * a.n_spins + i];
                            }
                            wr[s] = fma(sx, sp.ar[s], sy * sp.ai[s]);
                            wi[s] = fma(sx, sp.ai[s], -sy * sp.ar[s]);
                        }
                    }
                    const auto partial_c = partial + coil * a.coil_stride;
                    if (std::is_same<real, float>::value && G > 1 &&
                        (__builtin_amdgcn_readfirstlane(op.flags) & OPF_EVEN_T) != 0) {
                        // Instants on a regular raster (every fixed-dwell
                        // readout): the wave group shares its G * S spins, as
                        // in the Cartesian readout: wave wg of the group
                        // evaluates chunk round * G + wg for all of them, so
                        // each lane sums 8 spins per sample, the butterfly is
                        // shared by them and no chunk sums are added across
                        // waves.  Every spin's parameters and weighted anchor
                        // go through LDS once per pass; rows of G chunks are
                        // staged per round.  The T2 decay inside a block of 8
                        // samples is stepped by one factor per sample.
                        // Uneven instants take the per-wave path below.
                        constexpr int RT = G * S;
                        float4* g_row = s_trow;                                        // [G * kT]
                        double* g_anc = reinterpret_cast<double*>(g_row + G * kT);      // [G * kT / kTB][4]
                        float* g_par = reinterpret_cast<float*>(g_anc + 4 * (G * kT / kTB));   // [kWaves][S][8][64]
                        static_assert(sizeof(float4) * G * kT + sizeof(double) * 4 * (G * kT / kTB) +
                                          sizeof(float) * kWaves * S * 8 * 64 <= sizeof(s_stepf),
                                      "shared trajectory staging fits the step-factor area");
                        __syncthreads();     // earlier readers of these areas are done
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            float* q = g_par + ((wave * S + s) * 8) * 64 + lane;
                            const double r2 = sp.r2[s];
                            const uint64_t r2b = (uint64_t)__double_as_longlong(r2);
                            q[0 * 64] = sp.x[s]; q[1 * 64] = sp.y[s]; q[2 * 64] = sp.z[s]; q[3 * 64] = sp.dw[s];
                            q[4 * 64] = __uint_as_float((uint32_t)r2b);
                            q[5 * 64] = __uint_as_float((uint32_t)(r2b >> 32));
                            q[6 * 64] = wr[s]; q[7 * 64] = wi[s];
                        }
                        const int w0 = (wave / G) * G;
                        const int smp_lane = readout_sample_of_lane(lane);
                        const int n_rounds = (n_chunks + G - 1) / G;
                        const float dt_even = (float)uniform(op.u.tab.dt);
                        for (int round = 0; round < n_rounds; ++round) {
                            __syncthreads();     // parameters visible; previous round's rows read
                            if (tid < G * kT) {  // rows past n are never stored
                                const int c = tid / kT, t = tid % kT;
                                const int j = round * G + c;
                                const auto row = table + 4 * min(j * kT + t, n - 1);
                                const auto blk_row = table + 4 * min(j * kT + (t & ~(kTB - 1)), n - 1);
                                g_row[tid] = make_float4((float)(row[0] - blk_row[0]), (float)(row[1] - blk_row[1]),
                                                         (float)(row[2] - blk_row[2]), (float)(row[3] - blk_row[3]));
                                if ((t & (kTB - 1)) == 0) {
#pragma unroll
                                    for (int k = 0; k < 4; ++k) g_anc[(tid / kTB) * 4 + k] = blk_row[k];
                                }
                            }
                            __syncthreads();
                            const int j = round * G + wg;
                            if (j >= n_chunks) continue;
                            // the group's spins: x, y, z, dw and log2(e) / T2 for
                            // the samples; 1 / T2 and the anchor are read again
                            // per block (fewer live registers)
                            auto par = [&](int q) {
                                return g_par + (((w0 + q / S) * S + q % S) * 8) * 64 + lane;
                            };
                            auto rate = [&](const float* src) {
                                return __longlong_as_double((long long)(((uint64_t)__float_as_uint(src[5 * 64]) << 32) |
                                                                        (uint64_t)__float_as_uint(src[4 * 64])));
                            };
                            // pdec: the decay over one spacing, 2^(-dt log2(e) / T2)
                            float px[RT], py[RT], pz[RT], pdw[RT], pdec[RT];
#pragma unroll
                            for (int q = 0; q < RT; ++q) {
                                const float* src = par(q);
                                px[q] = src[0 * 64]; py[q] = src[1 * 64]; pz[q] = src[2 * 64]; pdw[q] = src[3 * 64];
                                pdec[q] = __builtin_amdgcn_exp2f(-dt_even * (float)(rate(src) * kLog2e));
                            }
                            float red16[16];
#pragma unroll
                            for (int b = 0; b < kT / kTB; ++b) {
                                // keep the blocks apart: interleaving them
                                // would keep several blocks' anchors live
                                __builtin_amdgcn_sched_barrier(0);
                                const double* anc = g_anc + (wg * (kT / kTB) + b) * 4;
                                const double kb[3] = {anc[0], anc[1], anc[2]};
                                const double tb = anc[3];
                                float c0[RT], br[RT], bi[RT];
#pragma unroll
                                for (int q = 0; q < RT; ++q) {
                                    const float* src = par(q);
                                    const double ph = phase_rev(kb, tb, px[q], py[q], pz[q], pdw[q]);
                                    c0[q] = (float)(ph - rint(ph));
                                    const float eb = Math<float>::expneg(tb, rate(src));
                                    br[q] = eb * src[6 * 64]; bi[q] = eb * src[7 * 64];
                                }
                                float vq[16];
                                // the block's decay E2(t - t_b) is pdec^(sample),
                                // stepped by one product per sample folded into
                                // (br, bi)
#pragma unroll
                                for (int t = 0; t < kTB; ++t) {
                                    const float4 d = g_row[wg * kT + b * kTB + t];
                                    const float dt_rev = d.w * (float)kInv2Pi;   // dw dt / 2 pi = dw * dt_rev
                                    float sr = 0, si = 0;
#pragma unroll
                                    for (int q = 0; q < RT; ++q) {
                                        const float f = c0[q] + fmaf(d.x, px[q], fmaf(d.y, py[q], fmaf(d.z, pz[q], pdw[q] * dt_rev)));
                                        const float c = __builtin_amdgcn_cosf(f);
                                        const float sn = __builtin_amdgcn_sinf(f);
                                        sr = fmaf(br[q], c, fmaf(bi[q], sn, sr));
                                        si = fmaf(bi[q], c, fmaf(-br[q], sn, si));
                                        br[q] *= pdec[q]; bi[q] *= pdec[q];
                                    }
                                    vq[2 * t] = sr; vq[2 * t + 1] = si;
                                }
                                quarter_reduce(vq, lane);
#pragma unroll
                                for (int i = 0; i < 4; ++i) red16[4 * b + i] = vq[i];
                            }
                            const float v = reduce16(red16, lane);
                            if (j * kT + smp_lane < n)
                                put_partial(partial_c + 2 * (int64_t)(aux + j * kT + smp_lane) + (lane & 1), v);
                        }
                        continue;
                    }
                    for (int j = 0; j < n_chunks; ++j) {
                        real v;
                        int smp_lane;                // chunk sample whose component lane & 1 this lane ends with
                        if constexpr (std::is_same<real, float>::value) {
                            static_assert(kTB == 8, "a block is one butterfly quarter");
                            __syncthreads();         // earlier readers of the staging area are done
                            if (tid < kT) {          // rows past n are never stored
                                const auto row = table + 4 * min(j * kT + tid, n - 1);
                                const auto blk_row = table + 4 * min(j * kT + (tid & ~(kTB - 1)), n - 1);
                                s_trow[tid] = make_float4((float)(row[0] - blk_row[0]), (float)(row[1] - blk_row[1]),
                                                          (float)(row[2] - blk_row[2]), (float)(row[3] - blk_row[3]));
                                if ((tid & (kTB - 1)) == 0) {
#pragma unroll
                                    for (int c = 0; c < 4; ++c) s_tanc[(tid / kTB) * 4 + c] = blk_row[c];
                                }
                            }
                            __syncthreads();
                            float red16[16];
#pragma unroll
                            for (int b = 0; b < kT / kTB; ++b) {
                                const double kb[3] = {s_tanc[b * 4], s_tanc[b * 4 + 1], s_tanc[b * 4 + 2]};
                                const double tb = s_tanc[b * 4 + 3];
                                float c0[S], br[S], bi[S];   // block phase, weighted magnetisation
#pragma unroll
                                for (int s = 0; s < S; ++s) {
                                    const double ph = phase_rev(kb, tb, sp.x[s], sp.y[s], sp.z[s], sp.dw[s]);
                                    c0[s] = (float)(ph - rint(ph));
                                    const float eb = Math<float>::expneg(tb, sp.r2[s]);
                                    br[s] = eb * wr[s]; bi[s] = eb * wi[s];
                                }
                                float q[16];
#pragma unroll
                                for (int t = 0; t < kTB; ++t) {
                                    const float4 d = s_trow[b * kTB + t];
                                    float sr = 0, si = 0;
#pragma unroll
                                    for (int s = 0; s < S; ++s) {
                                        const float f = c0[s] + fmaf(d.x, sp.x[s], fmaf(d.y, sp.y[s],
                                                                fmaf(d.z, sp.z[s], dwf[s] * d.w)));
                                        const float c = __builtin_amdgcn_cosf(f);
                                        const float sn = __builtin_amdgcn_sinf(f);
                                        const float ed = __builtin_amdgcn_exp2f(-d.w * r2l[s]);
                                        sr = fmaf(ed, fmaf(br[s], c, bi[s] * sn), sr);
                                        si = fmaf(ed, fmaf(bi[s], c, -br[s] * sn), si);
                                    }
                                    q[2 * t] = sr; q[2 * t + 1] = si;
                                }
                                quarter_reduce(q, lane);
#pragma unroll
                                for (int i = 0; i < 4; ++i) red16[4 * b + i] = q[i];
                            }
                            v = reduce16(red16, lane);
                            smp_lane = readout_sample_of_lane(lane);
                        } else {
                            real acc[2 * kT];
#pragma unroll
                            for (int t = 0; t < kT; ++t) {
                                const int smp = min(j * kT + t, n - 1);   // rows past n are never stored
                                const auto row = table + 4 * smp;
                                const double kx = row[0], ky = row[1], kz = row[2], tt = row[3];
                                real sr = 0, si = 0;
#pragma unroll
                                for (int s = 0; s < S; ++s) {
                                    const double ph = fma(kx, (double)sp.x[s], fma(ky, (double)sp.y[s],
                                                      fma(kz, (double)sp.z[s], (double)sp.dw[s] * kInv2Pi * tt)));
                                    real c, sn;
                                    Math<real>::cis(ph, c, sn);
                                    const real e2 = Math<real>::expneg(tt, sp.r2[s]);
                                    sr += e2 * fma(wr[s], c, wi[s] * sn);
                                    si += e2 * fma(wi[s], c, -wr[s] * sn);
                                }
                                acc[2 * t] = sr; acc[2 * t + 1] = si;
                            }
                            v = wave_reduce64(acc, lane);
                            smp_lane = lane >> 1;
                        }
                        if constexpr (G > 1) {
                            __syncthreads();             // earlier readers of red are done
                            red[wave * 64 + lane] = v;
                            __syncthreads();
                            if (wg == 0) {
                                v = red[wave * 64 + lane];
#pragma unroll
                                for (int g = 1; g < G; ++g) v += red[(wave + g) * 64 + lane];
                            }
                        }
                        if (wg == 0 && j * kT + smp_lane < n)
                            put_partial(partial_c + 2 * (int64_t)(aux + j * kT + smp_lane) + (lane & 1), v);
                    }
                }
                __syncthreads();                     // the staging area is free again
            } else if (kind == OP_ADC) {
                // A readout changes no spin state, so replicas of this tile
                // share the slice's readouts round-robin and skip the others.
                if (n_rep > 1 && (adc_seen++ % n_rep) != rep) continue;
                const int n = (int)__builtin_amdgcn_readfirstlane(op.n);
                const int aux = (int)__builtin_amdgcn_readfirstlane(op.aux);
                const double tau = uniform(op.u.adc.tau);
                const double mu[3] = {uniform(op.u.adc.mu[0]), uniform(op.u.adc.mu[1]), uniform(op.u.adc.mu[2])};
                if constexpr (kMatrix) {
                    if (MO || (__builtin_amdgcn_readfirstlane(op.flags) & OPF_MATRIX)) {
                        if (!MO && !(mt_valid && mu[0] == mt_mu[0] && mu[1] == mt_mu[1] && mu[2] == mt_mu[2] &&
                                     tau == mt_tau)) {
                            matrix_tables(sp, mu, tau, lane, mt);
                            mt_mu[0] = mu[0]; mt_mu[1] = mu[1]; mt_mu[2] = mu[2];
                            mt_tau = tau;
                            mt_valid = true;
                        }
                        if (a.n_coils == 0) {
                            matrix_readout(sp, op, mu, tau, n, false, 1.0f, 0.0f, mt, s_ta[wave < LW ? wave : 0],
                                           &s_md[0][0][0], m_pass, wave, lane, partial + 2 * (int64_t)aux, &dc);
                            continue;
                        }
                        for (int coil = 0; coil < a.n_coils; ++coil) {
                            // coil weight (S_x - j S_y) at the spin
                            const int64_t i = base + lane;
                            float wx = 0.0f, wy = 0.0f;
                            if (i < a.n_spins) {
                                wx = gmem(a.s_x)[coil * a.n_spins + i];
                                wy = gmem(a.s_y)[coil * a.n_spins + i];
                            }
                            matrix_readout(sp, op, mu, tau, n, true, wx, wy, mt, s_ta[wave < LW ? wave : 0],
                                           &s_md[0][0][0], m_pass, wave, lane,
                                           partial + coil * a.coil_stride + 2 * (int64_t)aux, &dc);
                        }
                        continue;
                    }
                }
                // Per spin: the sample-0 value p0 and the step factors
                // (StepFactors), all from FP64 phases.  Step factors depend
                // only on (mu, tau) and the spin; successive readouts of a
                // sequence usually share them, so they are kept (in LDS, off
                // the register budget) from the previous ADC operation when
                // (mu, tau) is unchanged.
                const bool same_step = step_valid && mu[0] == step_mu[0] && mu[1] == step_mu[1] &&
                                       mu[2] == step_mu[2] && tau == step_tau;
                // the step factors of spin s (StepFactors), each from its own
                // FP64 phase
                auto step_factors = [&](int s, real* f) {
                    const double ph = phase_rev(mu, tau, sp.x[s], sp.y[s], sp.z[s], sp.dw[s]);
                    auto put = [&](int c, double mult) {
                        real co, sn;
                        const real e = Math<real>::expneg(tau * mult, sp.r2[s]);
                        Math<real>::cis(ph * mult, co, sn);
                        f[2 * c] = e * co; f[2 * c + 1] = -e * sn;
                    };
#pragma unroll
                    for (int m = 1; m <= M; ++m) put(SF::kZ + m - 1, (double)m);
#pragma unroll
                    for (int g = 1; g < G; ++g) put(SF::kZg + g - 1, (double)(kT * g));
                    put(SF::kW, (double)(kT * G));
#pragma unroll
                    for (int k = 2 * SF::NC; k < NF; ++k) f[k] = 0;
                };
                // complex factor c of the spin in slot ss of lane ln
                auto factor = [&](int ss, int ln, int c, real& re, real& im) {
                    re = s_stepf[ss][(2 * c) / V][ln][(2 * c) % V];
                    im = s_stepf[ss][(2 * c) / V][ln][(2 * c) % V + 1];
                };
                if (!same_step) {
                    // other waves of the group may still read the factors of
                    // the previous readout
                    if constexpr (G > 1) __syncthreads();
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        real f[NF];
                        step_factors(s, f);
#pragma unroll
                        for (int v = 0; v < NF / V; ++v) {
                            vec_t w;
                            if constexpr (V == 4) w = make_float4(f[4 * v], f[4 * v + 1], f[4 * v + 2], f[4 * v + 3]);
                            else w = make_double2(f[2 * v], f[2 * v + 1]);
                            *reinterpret_cast<vec_t*>(&s_stepf[s][v][tid][0]) = w;
                        }
                    }
                    step_mu[0] = mu[0]; step_mu[1] = mu[1]; step_mu[2] = mu[2];
                    step_tau = tau;
                    step_valid = true;
                }
                // sample-0 magnetisation of this lane's spins
                real p0r[S], p0i[S];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    real e2 = Math<real>::expneg(op.txy, sp.r2[s]);
                    real c, sn;
                    Math<real>::cis(phase_rev(op.k, op.txy, sp.x[s], sp.y[s], sp.z[s], sp.dw[s]), c, sn);
                    p0r[s] = e2 * (sp.ar[s] * c + sp.ai[s] * sn);
                    p0i[s] = e2 * (sp.ai[s] * c - sp.ar[s] * sn);
                }
                // Receive coils: each coil's pass starts from the sample-0
                // magnetisation weighted by (S_x - j S_y) of that coil at the
                // spin; the spins' stepping above is shared by all coils.
                const int n_passes = a.n_coils > 0 ? a.n_coils : 1;
                for (int coil = 0; coil < n_passes; ++coil) {
                real ap[S][2];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (a.n_coils > 0) {
                        const int64_t i = base + s * 64 + lane;
                        real sx = 0, sy = 0;
                        if (i < a.n_spins) {
                            sx = (real)gmem(a.s_x)[coil * a.n_spins + i];
                            sy = (real)gmem(a.s_y)[coil * a.n_spins + i];
                        }
                        ap[s][0] = fma(sx, p0r[s], sy * p0i[s]);
                        ap[s][1] = fma(sx, p0i[s], -sy * p0r[s]);
                    } else {
                        ap[s][0] = p0r[s];
                        ap[s][1] = p0i[s];
                    }
                }
                const auto partial_c = partial + coil * a.coil_stride;
                // the wave group's G * S spins (LDS hand-over when G > 1)
                const int w0 = (wave / G) * G;
                const int n_chunks = (n + kT - 1) / kT;
                const int smp_of_lane = readout_sample_of_lane(lane);
                int xb = 0;
                if constexpr (G > 1) {
                    // Two buffers for alternate passes: the writers of this
                    // pass's buffer have passed the barrier below of the
                    // previous pass, which every reader of this buffer's
                    // previous contents had reached after reading it.
                    xb = x_pass++ & 1;
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        s_x[xb][wave][s][lane][0] = ap[s][0];
                        s_x[xb][wave][s][lane][1] = ap[s][1];
                    }
                    __syncthreads();
                }
                // A readout of fewer chunks than the group has waves would
                // leave waves idle: then n_share = G / n_chunks waves share
                // each chunk, each taking 1 / n_share of the group's spins,
                // and add their chunk sums in LDS in wave order (one chunk
                // per wave).
                int n_share = 1;
                if constexpr (G > 1) {
                    if (4 * n_chunks <= G) n_share = 4;
                    else if (2 * n_chunks <= G) n_share = 2;
                }
                auto run = [&](auto p_c) {
                    constexpr int P = decltype(p_c)::value;     // waves per chunk
                    constexpr int RS = R / P;                    // spins per lane in this readout
                    const int sub = wg % P;                      // which RS of the group's spins
                    const int j0 = wg / P;                       // first chunk
                    // zr/zi[q][m - 1] = z^m of spin q for m = 1 .. M (W, the
                    // stride of G chunks, is read from LDS when it is used)
                    real pr[RS], pi[RS], zr[RS][M], zi[RS][M];
#pragma unroll
                    for (int q = 0; q < RS; ++q) {
                        const int qq = sub * RS + q;
                        const int sw = w0 + qq / S, ss = qq % S;
                        const int ln = sw * 64 + lane;
                        real p_r, p_i;
                        if constexpr (G > 1) {
                            p_r = s_x[xb][sw][ss][lane][0]; p_i = s_x[xb][sw][ss][lane][1];
                        } else {
                            p_r = ap[ss][0]; p_i = ap[ss][1];
                        }
#pragma unroll
                        for (int m = 0; m < M; ++m) factor(ss, ln, SF::kZ + m, zr[q][m], zi[q][m]);
                        if (j0 > 0) {            // start at chunk j0: p0 z^(32 j0)
                            real Zr_, Zi_;
                            factor(ss, ln, SF::kZg + j0 - 1, Zr_, Zi_);
                            const real t = p_r * Zr_ - p_i * Zi_;
                            p_i = p_r * Zi_ + p_i * Zr_;
                            p_r = t;
                        }
                        pr[q] = p_r; pi[q] = p_i;
                    }
                    // With P > 1, P n_chunks == G: each sub-group has exactly
                    // the one chunk j0.  Saying so lets the compiler drop the
                    // loop; otherwise it hoists the (loop-invariant) products
                    // out of it and copies them before every in-place lane
                    // swap of the reduction.
                    const int j_end = P == 1 ? n_chunks : j0 + 1;
                    for (int j = j0; j < j_end; j += G / P) {
                        real qr[RS], qi[RS];
#pragma unroll
                        for (int q = 0; q < RS; ++q) { qr[q] = pr[q]; qi[q] = pi[q]; }
                        real red[16];
#pragma unroll
                        for (int h = 0; h < kT / 8; ++h) {     // quarters of 8 samples
                            real v[16];
#pragma unroll
                            for (int b = 0; b < 8; b += M) {
                                // sample t: the sum of the spins; samples
                                // t + m: the sum of the spins times z^m, as
                                // multiply-accumulates
                                const int t = 8 * h + b;
                                real sr = qr[0], si = qi[0];
#pragma unroll
                                for (int q = 1; q < RS; ++q) { sr += qr[q]; si += qi[q]; }
                                v[2 * b] = sr; v[2 * b + 1] = si;
#pragma unroll
                                for (int m = 1; m < M; ++m) {
                                    real ur = qr[0] * zr[0][m - 1], ui = qr[0] * zi[0][m - 1];
                                    ur = fma(-qi[0], zi[0][m - 1], ur);
                                    ui = fma(qi[0], zr[0][m - 1], ui);
#pragma unroll
                                    for (int q = 1; q < RS; ++q) {
                                        ur = fma(qr[q], zr[q][m - 1], ur);
                                        ur = fma(-qi[q], zi[q][m - 1], ur);
                                        ui = fma(qr[q], zi[q][m - 1], ui);
                                        ui = fma(qi[q], zr[q][m - 1], ui);
                                    }
                                    v[2 * (b + m)] = ur; v[2 * (b + m) + 1] = ui;
                                }
                                if (t + M < kT) {
#pragma unroll
                                    for (int q = 0; q < RS; ++q) {
                                        const real a_ = qr[q], b_ = qi[q];
                                        qr[q] = a_ * zr[q][M - 1] - b_ * zi[q][M - 1];
                                        qi[q] = a_ * zi[q][M - 1] + b_ * zr[q][M - 1];
                                    }
                                }
                            }
                            quarter_reduce(v, lane);
#pragma unroll
                            for (int i = 0; i < 4; ++i) red[4 * h + i] = v[i];
                        }
                        if constexpr (P == 1) {
                            if (j + G < j_end) {           // this wave has another chunk
#pragma unroll
                                for (int q = 0; q < RS; ++q) {     // advance G chunks from the anchor
                                    real w_r, w_i;
                                    factor(q % S, (w0 + q / S) * 64 + lane, SF::kW, w_r, w_i);
                                    const real a_ = pr[q], b_ = pi[q];
                                    pr[q] = a_ * w_r - b_ * w_i;
                                    pi[q] = a_ * w_i + b_ * w_r;
                                }
                            }
                        }
                        real v = reduce16(red, lane);
                        if constexpr (P > 1) {
                            // every wave of the group runs exactly this one
                            // chunk; the readers of s_red below are done
                            // before they reach the next readout's barrier
                            s_red[wave][lane] = v;
                            __syncthreads();
                            if (sub == 0)
                                for (int k = 1; k < P; ++k) v += s_red[wave + k][lane];
                        }
                        if (sub == 0 && j * kT + smp_of_lane < n)
                            put_partial(partial_c + 2 * (int64_t)(aux + j * kT + smp_of_lane) + (lane & 1), v);
                    }
                };
                if (__builtin_expect(n_share == 1, 1)) {
                    run(std::integral_constant<int, 1>());
                } else if constexpr (G >= 2) {
                    if (n_share == 2) run(std::integral_constant<int, 2>());
                    else if constexpr (G >= 4) run(std::integral_constant<int, 4>());
                }
                }   // coil passes
            }
        }
    }

    if (a.save_state && rep == 0) {
        const auto st = gmem(reinterpret_cast<real*>(a.state));
        const auto sa = st + (int64_t)(3 * a.anchor_parity) * a.n_spins;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t i = base + s * 64 + lane;
            if (i < a.n_spins) {
                sa[i] = sp.ar[s]; sa[a.n_spins + i] = sp.ai[s]; sa[2 * a.n_spins + i] = sp.az[s];
            }
        }
        for (int slot = 0; slot < kShapeSlots; ++slot) {
            if (!((a.cache_save >> slot) & 1u)) continue;
            const real* cache = s_cache + slot * (kShapeCacheReals * S * kBlock) + tid;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int64_t i = base + s * 64 + lane;
                if (i < a.n_spins) {
#pragma unroll
                    for (int e = 0; e < kShapeCacheReals; ++e)
                        st[(kStateSlot0 + kShapeCacheReals * slot + e) * a.n_spins + i] = cache[(e * S + s) * kBlock];
                }
            }
        }
    }
}

// Waves per SIMD the register allocation is held to: for FP32, two at 1
// and 2 spins per lane (at 1 the matrix-core readout keeps 50 table
// registers live next to the vector readout's; at 2 the readout is tuned to
// fit 256 registers, and a second wave hides the latency of its LDS and
// transcendental operations) and three in the matrix-only kernel (its
// spills are on cold paths: the prologue, the table build and the
// shaped-pulse fill); else whatever the code needs.
template <typename real, int S, int VAR = STEP_GENERAL>
struct StepOccupancy {
    static constexpr int kWavesPerEU = !std::is_same<real, float>::value ? 1
                                       : S == 1 && VAR != STEP_GENERAL ? 3
                                       : S <= 2 ? 2 : 1;
};

// Workgroup b < n_whole runs tile b whole; later workgroups run the tiles
// from n_whole on, b' = b - n_whole being tile n_whole + b' % (n_tiles -
// n_whole) as readout replica b' / (n_tiles - n_whole).  The whole tiles
// come first, so the split ones fill the end of the launch.
template <typename real, int S, int VAR = STEP_GENERAL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(StepOccupancy<real, S, VAR>::kWavesPerEU)))
void step_kernel(StepArgs a) {
    const int64_t b = blockIdx.x;
    int64_t tile = b;
    int rep = 0, n_rep = 1;
    if (b >= a.n_whole) {
        const int64_t bs = b - a.n_whole, nt = a.n_tiles - a.n_whole;
        tile = a.n_whole + bs % nt;
        rep = (int)(bs / nt);
        n_rep = a.n_replicas;
    }
    step_body<real, S, VAR>(a, tile, rep, n_rep);
}

// Persistent form: workgroups take (request, tile, readout replica) items
// from a queue until it is empty.  Items are numbered request by request
// (BatchItem.item_begin is the prefix sum of the requests' item counts, a
// request's items being its tiles times its replicas, replica-major).  Every
// item writes only its own rows and samples, so which workgroup runs it
// never changes a result.
template <typename real, int S, int VAR = STEP_GENERAL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(StepOccupancy<real, S, VAR>::kWavesPerEU)))
void batch_step_kernel(const BatchItem* __restrict__ reqs, int32_t n_req, int64_t total,
                       unsigned long long* counter) {
    __shared__ unsigned long long s_item;
    for (;;) {
        __syncthreads();                     // every wave is done reading s_item
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t item = (int64_t)s_item;
        if (item >= total) break;            // every wave of the group sees the same value
        int lo = 0, hi = n_req - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (reqs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
        }
        const StepArgs a = reqs[lo].args;
        const int64_t local = item - reqs[lo].item_begin;   // replica-major over the tiles
        step_body<real, S, VAR>(a, local % a.n_tiles, (int)(local / a.n_tiles), a.n_replicas);
    }
}

// Cross-workgroup sum (FP64, fixed order): partial rows are summed in groups
// of kRowGroup consecutive rows (pass 1), then the group sums in group order
// (pass 2); with at most kRowGroup rows pass 1 writes the output directly.
constexpr int64_t kRowGroup = 64;

// A pass-1 thread sums kFinVals consecutive values of its row group with
// one 16-byte (FP32) or two 16-byte (FP64) loads per row: the host pads
// row_stride and every coil block to a multiple of kFinVals values, so the
// loads are aligned and stay inside the rows (values past n_vals in the
// padding are read but never stored).  Each value is still summed over the
// rows in row order.  The partial rows are read once, so the loads are
// nontemporal, as are the step kernels' stores of them (put_partial).

__device__ __forceinline__ void load_fin(const float* p, double (&v)[kFinVals]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 q = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}
__device__ __forceinline__ void load_fin(const double* p, double (&v)[kFinVals]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 a = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
    const d2 b = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p) + 1);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

// Sum of rows r0 .. r1 - 1 at values j .. j + kFinVals - 1 into out[j ..],
// the values below n_vals only.
template <typename real>
__device__ __forceinline__ void sum_rows(const real* partial, int64_t r0, int64_t r1, int64_t row_stride, int64_t j,
                                         int64_t n_vals, double* out) {
    double s[kFinVals] = {0.0, 0.0, 0.0, 0.0};
    // eight rows' loads in flight before their adds (still in row order)
    constexpr int kU = 8;
    int64_t r = r0;
    for (; r + kU <= r1; r += kU) {
        double v[kU][kFinVals];
#pragma unroll
        for (int u = 0; u < kU; ++u) load_fin(partial + (r + u) * row_stride + j, v[u]);
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int k = 0; k < kFinVals; ++k) s[k] += v[u][k];
    }
    for (; r < r1; ++r) {
        double v[kFinVals];
        load_fin(partial + r * row_stride + j, v);
#pragma unroll
        for (int k = 0; k < kFinVals; ++k) s[k] += v[k];
    }
#pragma unroll
    for (int k = 0; k < kFinVals; ++k)
        if (j + k < n_vals) out[j + k] = s[k];
}

template <typename real>
__global__ void finalize_rows_kernel(const real* __restrict__ partial, int64_t n_rows, int64_t row_stride,
                                     int64_t n_vals, double* __restrict__ out) {
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kFinVals;
    if (j >= n_vals) return;
    const int64_t r0 = (int64_t)blockIdx.y * kRowGroup;
    const int64_t r1 = min(n_rows, r0 + kRowGroup);
    sum_rows(partial, r0, r1, row_stride, j, n_vals, out + (int64_t)blockIdx.y * n_vals);
}

// Sum of the group sums of value j in group order; eight groups' loads in
// flight before their adds (a thread per value leaves few workgroups, so
// each must keep several loads outstanding).
template <typename P>
__device__ __forceinline__ double sum_groups(P mid, int64_t n_groups, int64_t n_vals, int64_t j) {
    constexpr int kU = 8;
    double s = 0.0;
    int64_t g = 0;
    for (; g + kU <= n_groups; g += kU) {
        double v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = mid[(g + u) * n_vals + j];
#pragma unroll
        for (int u = 0; u < kU; ++u) s += v[u];
    }
    for (; g < n_groups; ++g) s += mid[g * n_vals + j];
    return s;
}

__global__ void finalize_groups_kernel(const double* __restrict__ mid, int64_t n_groups, int64_t n_vals,
                                       double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_vals) return;
    out[j] = sum_groups(mid, n_groups, n_vals, j);
}

// Batched finalize: pass 1 over (request, row group, value tile), pass 2
// over (request, value tile) for requests with more than one row group.
__device__ __forceinline__ int find_desc(const FinDesc* d, int n, int64_t t, bool pass2) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((pass2 ? d[mid].tile_begin2 : d[mid].tile_begin1) <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename real>
__global__ void batch_finalize_pass1(const FinDesc* __restrict__ d, int32_t n) {
    const int64_t t = blockIdx.x;
    const FinDesc& f = d[find_desc(d, n, t, false)];
    const int64_t jt = finalize_tiles(f.n_vals);
    const int64_t local = t - f.tile_begin1;
    const int64_t g = local / jt;
    const int64_t j = ((local % jt) * 256 + threadIdx.x) * kFinVals;
    if (j >= f.n_vals) return;
    const int64_t r0 = g * kRowGroup, r1 = min(f.n_rows, r0 + kRowGroup);
    sum_rows(reinterpret_cast<const real*>(f.partial), r0, r1, f.row_stride, j, f.n_vals,
             f.n_groups > 1 ? f.mid + g * f.n_vals : f.out);
}

__global__ void batch_finalize_pass2(const FinDesc* __restrict__ d, int32_t n) {
    const int64_t t = blockIdx.x;
    const FinDesc& f = d[find_desc(d, n, t, true)];
    const int64_t j = (t - f.tile_begin2) * 256 + threadIdx.x;
    if (f.n_groups <= 1 || j >= f.n_vals) return;
    gmem(f.out)[j] = sum_groups(gmem(f.mid), f.n_groups, f.n_vals, j);
}

__global__ void fill_zero_kernel(double* __restrict__ out, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[j] = 0.0;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename real, int S, int VAR = STEP_GENERAL>
static size_t dyn_lds_t(int32_t n_shape_rows, int32_t n_cache_slots) {
    return (VAR == STEP_MATRIX_ONLY ? 0 : (size_t)n_shape_rows * 9 * sizeof(double)) +
           (size_t)n_cache_slots * kShapeCacheReals * S * kBlock * sizeof(real);
}

// LDS the matrix-only kernel declares: A-operand tiles and result buffers
// (it reads its operations through the scalar cache, and the vector path's
// arrays are not in it).
constexpr size_t matrix_only_static_lds_bytes() {
    return sizeof(float) * kWaves * kMatrixARows * 32 + sizeof(float4) * 4 * kWaves * 64;
}

// Calls f(real_tag, S_tag, V_tag) for the kernel instance the arguments
// select; returns false for a combination that has none.
template <typename F>
static bool dispatch_step(int precision, int spins_per_lane, int variant, F&& f) {
    using std::integral_constant;
    if (precision == 64) {
        switch (spins_per_lane) {
            case 1: f(double(), integral_constant<int, 1>(), integral_constant<int, STEP_GENERAL>()); return true;
            case 2: f(double(), integral_constant<int, 2>(), integral_constant<int, STEP_GENERAL>()); return true;
            default: return false;
        }
    }
    switch (spins_per_lane) {
        case 1:
            if (variant == STEP_MATRIX_ONLY)
                f(float(), integral_constant<int, 1>(), integral_constant<int, STEP_MATRIX_ONLY>());
            else if (variant == STEP_VECTOR_ONLY)
                f(float(), integral_constant<int, 1>(), integral_constant<int, STEP_VECTOR_ONLY>());
            else
                f(float(), integral_constant<int, 1>(), integral_constant<int, STEP_GENERAL>());
            return true;
        case 2: f(float(), integral_constant<int, 2>(), integral_constant<int, STEP_GENERAL>()); return true;
        case 4: f(float(), integral_constant<int, 4>(), integral_constant<int, STEP_GENERAL>()); return true;
        case 8: f(float(), integral_constant<int, 8>(), integral_constant<int, STEP_GENERAL>()); return true;
        default: return false;
    }
}

size_t step_dyn_lds_bytes(int precision, int spins_per_lane, int32_t n_shape_rows, int32_t n_cache_slots,
                          int variant) {
    size_t out = 0;
    // (an unsupported spins_per_lane sizes as S = 8, the largest)
    if (!dispatch_step(precision, precision == 64 ? std::min(spins_per_lane, 2) : spins_per_lane, variant,
                       [&](auto r, auto sc, auto vc) {
                           out = dyn_lds_t<decltype(r), decltype(sc)::value, decltype(vc)::value>(n_shape_rows,
                                                                                                 n_cache_slots);
                       }))
        out = dyn_lds_t<float, 8>(n_shape_rows, n_cache_slots);
    return out;
}

int step_workgroups_per_cu(int precision, int spins_per_lane, int variant, size_t dyn_lds) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    dispatch_step(precision, precision == 64 ? std::min(spins_per_lane, 2) : spins_per_lane, variant,
                  [&](auto r, auto sc, auto vc) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, step_kernel<decltype(r), decltype(sc)::value, decltype(vc)::value>, kBlock, dyn_lds);
    });
    return e == hipSuccess && n > 0 ? n : 1;
}

int shape_cache_slots_fitting(int precision, int spins_per_lane, int32_t n_shape_rows, int variant) {
    // FP32: keep a workgroup's LDS within half of a CU's 160 KiB so that two
    // workgroups (8 waves, the register-bound occupancy at S = 2) stay
    // resident per CU.  At S = 1 registers allow three; slots that push a
    // workgroup past a third of the LDS trade the third for fewer sub-step
    // evaluations, which cost far more.  FP64 kernels run one workgroup per
    // CU anyway.
    const size_t kBudget = (precision == 64 ? 160 : 80) * 1024;
    // The matrix-only kernel reads its shaped-pulse rows from memory: with one
    // slot (12 KiB) it stays within a third of the CU's LDS, the three
    // workgroups per CU its registers allow.
    size_t fixed = static_lds_bytes<float, 8>();
    if (precision != 64 && spins_per_lane == 1 && variant == STEP_MATRIX_ONLY)
        fixed = matrix_only_static_lds_bytes();
    else
        dispatch_step(precision, spins_per_lane, variant, [&](auto r, auto sc, auto vc) {
            fixed = static_lds_bytes<decltype(r), decltype(sc)::value, decltype(vc)::value>();
        });
    int n = 0;
    while (n < kShapeSlots &&
           fixed + step_dyn_lds_bytes(precision, spins_per_lane, n_shape_rows, n + 1, variant) <= kBudget)
        ++n;
    return n;
}

template <typename real, int S, int VAR = STEP_GENERAL>
static hipError_t launch_step_t(const StepArgs& a, int64_t n_blocks, hipStream_t st) {
    const size_t dyn = dyn_lds_t<real, S, VAR>(a.n_shape_rows, a.n_cache_slots);
    StepArgs b = a;
    b.n_tiles = n_blocks;
    if (b.n_replicas < 1) b.n_replicas = 1;
    if (b.n_whole < 0 || b.n_whole > n_blocks) return hipErrorInvalidValue;
    if (b.n_whole == n_blocks) b.n_replicas = 1;
    const int64_t grid = b.n_whole + (n_blocks - b.n_whole) * b.n_replicas;
    hipLaunchKernelGGL((step_kernel<real, S, VAR>), dim3((unsigned)grid), dim3(kBlock), dyn, st, b);
    return hipGetLastError();
}

template <typename real, int S, int VAR = STEP_GENERAL>
static hipError_t launch_batch_t(const BatchItem* reqs, int32_t n_req, int64_t total, unsigned long long* counter,
                                 size_t dyn, int n_cu, hipStream_t st) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_step_kernel<real, S, VAR>, kBlock, dyn) !=
            hipSuccess || per_cu < 1)
        per_cu = 1;
    const int64_t grid = std::min<int64_t>(total, (int64_t)per_cu * n_cu);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((batch_step_kernel<real, S, VAR>), dim3((unsigned)grid), dim3(kBlock), dyn, st, reqs, n_req,
                       total, counter);
    return hipGetLastError();
}

hipError_t launch_batch_step(const BatchItem* reqs, int32_t n_req, int64_t total, unsigned long long* counter,
                             size_t dyn_lds, int precision, int spins_per_lane, int n_cu, hipStream_t st,
                             int variant) {
    hipError_t e = hipErrorInvalidValue;
    dispatch_step(precision, spins_per_lane, variant, [&](auto r, auto sc, auto vc) {
        e = launch_batch_t<decltype(r), decltype(sc)::value, decltype(vc)::value>(reqs, n_req, total, counter,
                                                                                   dyn_lds, n_cu, st);
    });
    return e;
}

hipError_t launch_batch_finalize(const FinDesc* d, int32_t n, int64_t tiles1, int64_t tiles2, int precision,
                                 hipStream_t st) {
    if (tiles1 > 0) {
        if (precision == 64)
            hipLaunchKernelGGL(batch_finalize_pass1<double>, dim3((unsigned)tiles1), dim3(256), 0, st, d, n);
        else
            hipLaunchKernelGGL(batch_finalize_pass1<float>, dim3((unsigned)tiles1), dim3(256), 0, st, d, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (tiles2 > 0) {
        hipLaunchKernelGGL(batch_finalize_pass2, dim3((unsigned)tiles2), dim3(256), 0, st, d, n);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipKernelNodeParams KernelNode::params() {
    argv[0] = &a0; argv[1] = &a1; argv[2] = &a2; argv[3] = &a3;
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(func);
    p.gridDim = grid;
    p.blockDim = block;
    p.sharedMemBytes = (unsigned int)shmem;
    p.kernelParams = argv;
    p.extra = nullptr;
    return p;
}

hipError_t KernelNode::launch(hipStream_t st) {
    const hipKernelNodeParams p = params();
    return hipLaunchKernel(p.func, p.gridDim, p.blockDim, p.kernelParams, p.sharedMemBytes, st);
}

template <typename real, int S, int VAR = STEP_GENERAL>
static hipError_t batch_node_t(const BatchItem* reqs, int32_t n_req, int64_t total, unsigned long long* counter,
                               size_t dyn, int n_cu, std::vector<KernelNode>* out) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_step_kernel<real, S, VAR>, kBlock, dyn) !=
            hipSuccess || per_cu < 1)
        per_cu = 1;
    const int64_t grid = std::min<int64_t>(total, (int64_t)per_cu * n_cu);
    if (grid <= 0) return hipSuccess;
    KernelNode k;
    k.func = reinterpret_cast<const void*>(&batch_step_kernel<real, S, VAR>);
    k.grid = dim3((unsigned)grid);
    k.block = dim3(kBlock);
    k.shmem = dyn;
    k.n_args = 4;
    k.a0 = reqs; k.a1 = n_req; k.a2 = total; k.a3 = counter;
    out->push_back(k);
    return hipSuccess;
}

hipError_t batch_step_nodes(const BatchItem* reqs, int32_t n_req, int64_t total, unsigned long long* counter,
                            size_t dyn_lds, int precision, int spins_per_lane, int n_cu, std::vector<KernelNode>* out,
                            int variant) {
    hipError_t e = hipErrorInvalidValue;
    dispatch_step(precision, spins_per_lane, variant, [&](auto r, auto sc, auto vc) {
        e = batch_node_t<decltype(r), decltype(sc)::value, decltype(vc)::value>(reqs, n_req, total, counter, dyn_lds,
                                                                                 n_cu, out);
    });
    return e;
}

hipError_t batch_finalize_nodes(const FinDesc* d, int32_t n, int64_t tiles1, int64_t tiles2, int precision,
                                std::vector<KernelNode>* out) {
    if (tiles1 > 0) {
        KernelNode k;
        k.func = precision == 64 ? reinterpret_cast<const void*>(&batch_finalize_pass1<double>)
                                 : reinterpret_cast<const void*>(&batch_finalize_pass1<float>);
        k.grid = dim3((unsigned)tiles1);
        k.n_args = 2;
        k.a0 = d; k.a1 = n;
        out->push_back(k);
    }
    if (tiles2 > 0) {
        KernelNode k;
        k.func = reinterpret_cast<const void*>(&batch_finalize_pass2);
        k.grid = dim3((unsigned)tiles2);
        k.n_args = 2;
        k.a0 = d; k.a1 = n;
        out->push_back(k);
    }
    return hipSuccess;
}

int64_t spins_per_block_of(int spins_per_lane) { return (int64_t)kBlock * spins_per_lane; }

// Device memory of the allocation-free entry point: op and shaped-pulse
// tables, partial-sum rows, finalize row-group sums and slice state of one
// request at a time.  Every GPU the library runs on holds its own copy from
// module load to process end.  Host code must not pass `scratch` itself to a
// kernel or a copy (in host code the name stands for a host-side shadow, not
// a device address): it uses the address hipGetSymbolAddress returns for the
// current device, kept per device by noalloc_scratch.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// ---------------------------------------------------------------------------
// K-t simulation (section 5.1.2, eq. 4.19): the object's spatial-frequency
// function at the configurations' lattice positions, superposed per sample
// ---------------------------------------------------------------------------
// Spectrum: one workgroup per (tissue, block of up to 32 pairs, tile of up to
// kKtTile spins of that tissue).  Every lane holds kKtSpl spins and forms,
// for each pair p of the block, sum over its spins of
// m0 exp(-2 pi j k_p . x) (phase in FP64 revolutions, reduced to one
// revolution, then the hardware sine / cosine in FP32, or FP64 sincospi);
// the 64 sums (32 pairs x re / im) are reduced across the wave's lanes by
// the transpose-reduce, the four waves' results added in wave order, and
// the tile's row written to partial[item].
template <typename real>
__global__ __launch_bounds__(kBlock) void kt_spectrum_kernel(const KtItem* __restrict__ items,
                                                             const double* __restrict__ pair_k,
                                                             const float* __restrict__ x,
                                                             const float* __restrict__ y,
                                                             const float* __restrict__ z,
                                                             const float* __restrict__ m0,
                                                             real* __restrict__ partial) {
    __shared__ double s_k[kKtPairs][3];
    __shared__ real s_red[kWaves][64];
    const KtItem it = items[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < 3 * kKtPairs; i += kBlock)
        s_k[i / 3][i % 3] = i / 3 < it.n_pairs ? pair_k[3 * (it.pair_begin + i / 3) + i % 3] : 0.0;
    double px[kKtSpl], py[kKtSpl], pz[kKtSpl];
    real w[kKtSpl];
#pragma unroll
    for (int s = 0; s < kKtSpl; ++s) {
        const int64_t j = (int64_t)(wave * kKtSpl + s) * 64 + lane;   // coalesced rows of 64
        const bool in = j < it.n_spins;
        const int64_t i = it.spin_begin + (in ? j : 0);
        px[s] = in ? (double)x[i] : 0.0;
        py[s] = in ? (double)y[i] : 0.0;
        pz[s] = in ? (double)z[i] : 0.0;
        w[s] = in ? (real)m0[i] : (real)0;
    }
    __syncthreads();
    real v[64];
#pragma unroll
    for (int p = 0; p < kKtPairs; ++p) {
        const double k0 = s_k[p][0], k1 = s_k[p][1], k2 = s_k[p][2];
        real re = 0, im = 0;
#pragma unroll
        for (int s = 0; s < kKtSpl; ++s) {
            real c, sn;
            Math<real>::cis(fma(k0, px[s], fma(k1, py[s], k2 * pz[s])), c, sn);
            re = fma(w[s], c, re);
            im = fma(-w[s], sn, im);
        }
        v[2 * p] = re;
        v[2 * p + 1] = im;
    }
    real r = wave_reduce64(v, lane);       // lane l: component l & 1 of pair l >> 1
    s_red[wave][lane] = r;
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int g = 1; g < kWaves; ++g) r += s_red[g][lane];
        partial[(int64_t)blockIdx.x * 64 + lane] = r;
    }
}

// S(pair) = sum over the tiles of its tissue of the tiles' partial sums, in
// tile order, FP64.
template <typename real>
__global__ void kt_pair_sum_kernel(const KtPairSum* __restrict__ ps, int64_t n_pairs, const real* __restrict__ partial,
                                   double* __restrict__ spec) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_pairs) return;
    const KtPairSum q = ps[u];
    double re = 0.0, im = 0.0;
    for (int32_t t = 0; t < q.n_tiles; ++t) {
        const real* row = partial + (q.item0 + t) * 64 + 2 * q.slot;
        re += (double)row[0];
        im += (double)row[1];
    }
    spec[2 * u] = re;
    spec[2 * u + 1] = im;
}

// signal[n] = sum over the sample's entries of a_e S(pair_e) (eq. 4.19).
__global__ void kt_combine_kernel(const KtEntry* __restrict__ entries, const int64_t* __restrict__ offsets,
                                  int64_t n_samples, const double* __restrict__ spec, double* __restrict__ signal) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_samples) return;
    double re = 0.0, im = 0.0;
    for (int64_t e = offsets[n]; e < offsets[n + 1]; ++e) {
        const KtEntry q = entries[e];
        const double sr = spec[2 * q.pair], si = spec[2 * q.pair + 1];
        re += q.a_re * sr - q.a_im * si;
        im += q.a_re * si + q.a_im * sr;
    }
    signal[2 * n] = re;
    signal[2 * n + 1] = im;
}

hipError_t launch_kt(const KtItem* items, int64_t n_items, const double* pair_k, const KtPairSum* pair_sums,
                     int64_t n_pairs, const KtEntry* entries, const int64_t* offsets, int64_t n_samples,
                     const float* x, const float* y, const float* z, const float* m0, void* partial, double* spec,
                     double* signal, int precision, hipStream_t st) {
    if (n_samples <= 0) return hipSuccess;
    if (n_items > 0) {
        if (n_items > 0x7fffffffll) return hipErrorInvalidValue;
        if (precision == 64)
            hipLaunchKernelGGL(kt_spectrum_kernel<double>, dim3((unsigned)n_items), dim3(kBlock), 0, st, items,
                               pair_k, x, y, z, m0, reinterpret_cast<double*>(partial));
        else
            hipLaunchKernelGGL(kt_spectrum_kernel<float>, dim3((unsigned)n_items), dim3(kBlock), 0, st, items,
                               pair_k, x, y, z, m0, reinterpret_cast<float*>(partial));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const unsigned g = (unsigned)((n_pairs + 255) / 256);
        if (precision == 64)
            hipLaunchKernelGGL(kt_pair_sum_kernel<double>, dim3(g), dim3(256), 0, st, pair_sums, n_pairs,
                               reinterpret_cast<const double*>(partial), spec);
        else
            hipLaunchKernelGGL(kt_pair_sum_kernel<float>, dim3(g), dim3(256), 0, st, pair_sums, n_pairs,
                               reinterpret_cast<const float*>(partial), spec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kt_combine_kernel, dim3((unsigned)((n_samples + 255) / 256)), dim3(256), 0, st, entries,
                       offsets, n_samples, spec, signal);
    return hipGetLastError();
}

hipError_t noalloc_scratch(int device, void** ptr) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes the device current
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_step(const StepArgs& a, int precision, int spins_per_lane, int64_t n_blocks,
                       hipStream_t st, int variant) {
    if (n_blocks <= 0) return hipSuccess;
    hipError_t e = hipErrorInvalidValue;
    dispatch_step(precision, spins_per_lane, variant, [&](auto r, auto sc, auto vc) {
        e = launch_step_t<decltype(r), decltype(sc)::value, decltype(vc)::value>(a, n_blocks, st);
    });
    return e;
}

int64_t row_group_size() { return kRowGroup; }

int64_t finalize_scratch_doubles(int64_t n_rows, int64_t n_vals) {
    const int64_t groups = (n_rows + kRowGroup - 1) / kRowGroup;
    return groups > 1 ? groups * n_vals : 0;
}

hipError_t launch_finalize(const void* partial, int precision, int64_t n_rows, int64_t row_stride,
                           int64_t n_vals, double* out, double* scratch, hipStream_t st) {
    if (n_vals <= 0) return hipSuccess;
    const int threads = 256;
    if (row_stride % kFinVals != 0 || reinterpret_cast<uintptr_t>(partial) % 16 != 0) return hipErrorInvalidValue;
    const int64_t gx = finalize_tiles(n_vals);
    const int64_t groups = (n_rows + kRowGroup - 1) / kRowGroup;
    double* dst = groups > 1 ? scratch : out;
    if (groups > 1 && !scratch) return hipErrorInvalidValue;
    const dim3 grid((unsigned)gx, (unsigned)std::max<int64_t>(groups, 1));
    if (precision == 64)
        hipLaunchKernelGGL(finalize_rows_kernel<double>, grid, dim3(threads), 0, st,
                           reinterpret_cast<const double*>(partial), n_rows, row_stride, n_vals, dst);
    else
        hipLaunchKernelGGL(finalize_rows_kernel<float>, grid, dim3(threads), 0, st,
                           reinterpret_cast<const float*>(partial), n_rows, row_stride, n_vals, dst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || groups <= 1) return e;
    hipLaunchKernelGGL(finalize_groups_kernel, dim3((unsigned)((n_vals + threads - 1) / threads)), dim3(threads), 0,
                       st, scratch, groups, n_vals, out);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    const int64_t grid = (n + threads - 1) / threads;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)grid), dim3(threads), 0, st, out, n);
    return hipGetLastError();
}

}  // namespace ps
