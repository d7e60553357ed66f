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
// Per-sample superposition (eq. 3.32): each lane first sums its S spins,
// then a butterfly over 32 consecutive samples (64 reals) reduces the 64
// lanes with permlane32/16 swaps and DPP, leaving lane l with sample l/2,
// component l%2; the 4 waves are added in LDS in a fixed order and the
// workgroup writes one partial per sample.  A second kernel sums the
// workgroup partials in FP64 in workgroup order.  Every order is fixed, so
// results are bitwise reproducible for a given tiling.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ps_kernels.h"
#include "ps_ops.h"

namespace ps {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kOpChunk = 32;
constexpr int kT = 32;  // samples per reduction chunk (64 reals -> 64 lanes)

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
    // 1 - exp(-t r), formed without cancellation (for t r << 1 the FP32
    // difference 1 - exp(-t r) would keep only a few significant bits).
    static __device__ __forceinline__ float one_minus_expneg(double t, double r) {
        return (float)(-expm1(-t * r));
    }
    // cos and sin of 2 pi c for a phase c in revolutions (FP64), reduced to
    // [-1/2, 1/2] in FP64 before rounding to FP32.
    static __device__ __forceinline__ void cis(double c, float& co, float& si) {
        float f = (float)(c - rint(c));
        sincospif(2.0f * f, &si, &co);
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

// ---------------------------------------------------------------------------
// wave-wide transpose-reduce of 64 values per lane -> 1 value per lane
// (lane l ends with the sum over all 64 lanes of input value l)
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL, int BIT, int HALF>
__device__ __forceinline__ void dpp_stage(float (&v)[64], int lane) {
    const bool upper = (lane & BIT) != 0;
#pragma unroll
    for (int i = 0; i < HALF; ++i) {
        float send = upper ? v[i] : v[i + HALF];
        float keep = upper ? v[i + HALF] : v[i];
        v[i] = keep + dpp<CTRL>(send);
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
template <typename real, int S>
struct Spins {
    float x[S], y[S], z[S], dw[S], m0[S];
    double r1[S], r2[S];     // 1/T1, 1/T2 (0 for +inf)
    real ar[S], ai[S], az[S];  // anchors: Mxy_a = ar + j ai, Mz_a = az
};

// Phase of a spin in revolutions: k.x + (dw / 2 pi) t.
__device__ __forceinline__ double phase_rev(const double* k, double t, float x, float y, float z,
                                            float dw) {
    return fma(k[0], (double)x, fma(k[1], (double)y, fma(k[2], (double)z, (double)dw * kInv2Pi * t)));
}

// Magnetisation at the instant described by (k, txy, tz) from the anchors.
template <typename real, int S>
__device__ __forceinline__ void evaluate(const Spins<real, S>& sp, const Op& op, bool mxy_zero,
                                         real (&mx)[S], real (&my)[S], real (&mz)[S]) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
        real e1 = Math<real>::expneg(op.tz, sp.r1[s]);
        real m0 = (real)sp.m0[s];
        mz[s] = m0 + (sp.az[s] - m0) * e1;
        if (mxy_zero) {
            mx[s] = 0; my[s] = 0;
        } else {
            real e2 = Math<real>::expneg(op.txy, sp.r2[s]);
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

template <typename real, int S>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs a) {
    __shared__ Op s_ops[kOpChunk];
    __shared__ real s_red[2][kWaves][64];
    extern __shared__ __align__(16) unsigned char s_dyn[];
    real* s_rows = reinterpret_cast<real*>(s_dyn);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t base = ((int64_t)blockIdx.x * kWaves + wave) * 64 * S;

    Spins<real, S> sp;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t i = base + s * 64 + lane;
        if (i < a.n_spins) {
            sp.x[s] = a.x[i]; sp.y[s] = a.y[i]; sp.z[s] = a.z[i];
            sp.m0[s] = a.m0[i]; sp.dw[s] = a.dw[i];
            sp.r1[s] = 1.0 / (double)a.t1[i];
            sp.r2[s] = 1.0 / (double)a.t2[i];
            if (a.load_state) {
                const real* st = reinterpret_cast<const real*>(a.state);
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

    // shaped-pulse rotation rows -> LDS (made visible by the first barrier below)
    {
        const real* rows = reinterpret_cast<const real*>(a.rows);
        for (int i = tid; i < a.n_rows * 9; i += kBlock) s_rows[i] = rows[i];
    }

    real* partial = reinterpret_cast<real*>(a.partial) + (int64_t)blockIdx.x * a.row_stride;
    int red_buf = 0;

    for (int c0 = 0; c0 < a.n_ops; c0 += kOpChunk) {
        const int cn = min(kOpChunk, a.n_ops - c0);
        __syncthreads();
        {
            const uint4* src = reinterpret_cast<const uint4*>(a.ops + c0);
            uint4* dst = reinterpret_cast<uint4*>(s_ops);
            for (int i = tid; i < cn * 8; i += kBlock) dst[i] = src[i];
        }
        __syncthreads();

        for (int j = 0; j < cn; ++j) {
            const Op& op = s_ops[j];
            const uint32_t kind = __builtin_amdgcn_readfirstlane(op.kind);
            const bool mxy_zero = (__builtin_amdgcn_readfirstlane(op.flags) & OPF_MXY_ZERO) != 0;

            if (kind == OP_RF) {
                real mx[S], my[S], mz[S];
                evaluate<real, S>(sp, op, mxy_zero, mx, my, mz);
                rotate<real, S>(rot_of<real>(op), mx, my, mz);
#pragma unroll
                for (int s = 0; s < S; ++s) { sp.ar[s] = mx[s]; sp.ai[s] = my[s]; sp.az[s] = mz[s]; }
            } else if (kind == OP_SPOIL) {
#pragma unroll
                for (int s = 0; s < S; ++s) { sp.ar[s] = 0; sp.ai[s] = 0; }
            } else if (kind == OP_SHAPE) {
                real mx[S], my[S], mz[S];
                evaluate<real, S>(sp, op, mxy_zero, mx, my, mz);
                // every sub-step: hard sub-pulse, then precession/decay by u and
                // T1 recovery, all in "operator minus identity" form (see rotate)
                const double tau = op.u.adc.tau;
                real dur[S], dui[S], d1[S], m0r[S];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    step_delta<real>(phase_rev(op.u.adc.mu, tau, sp.x[s], sp.y[s], sp.z[s], sp.dw[s]), tau,
                                     sp.r2[s], dur[s], dui[s]);
                    d1[s] = Math<real>::one_minus_expneg(tau, sp.r1[s]);
                    m0r[s] = (real)sp.m0[s];
                }
                const int n_sub = (int)__builtin_amdgcn_readfirstlane(op.n);
                const real* rows = s_rows + 9 * (int)__builtin_amdgcn_readfirstlane(op.aux);
                for (int q = 0; q < n_sub; ++q) {
                    rotate<real, S>(rows + 9 * q, mx, my, mz);
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        real a_ = mx[s], b_ = my[s];
                        mx[s] = fma(a_, dur[s], fma(-b_, dui[s], a_));
                        my[s] = fma(a_, dui[s], fma(b_, dur[s], b_));
                        mz[s] = fma(m0r[s] - mz[s], d1[s], mz[s]);
                    }
                }
#pragma unroll
                for (int s = 0; s < S; ++s) { sp.ar[s] = mx[s]; sp.ai[s] = my[s]; sp.az[s] = mz[s]; }
            } else if (kind == OP_ADC) {
                const int n = (int)__builtin_amdgcn_readfirstlane(op.n);
                const int aux = (int)__builtin_amdgcn_readfirstlane(op.aux);
                const double tau = op.u.adc.tau;
                real pr[S], pi[S], zr[S], zi[S], Zr[S], Zi[S], cr[S], ci[S];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    // sample 0
                    real e2 = Math<real>::expneg(op.txy, sp.r2[s]);
                    real c, sn;
                    Math<real>::cis(phase_rev(op.k, op.txy, sp.x[s], sp.y[s], sp.z[s], sp.dw[s]), c, sn);
                    pr[s] = e2 * (sp.ar[s] * c + sp.ai[s] * sn);
                    pi[s] = e2 * (sp.ai[s] * c - sp.ar[s] * sn);
                    cr[s] = pr[s]; ci[s] = pi[s];
                    // one sample step and kT sample steps
                    const double ph = phase_rev(op.u.adc.mu, tau, sp.x[s], sp.y[s], sp.z[s], sp.dw[s]);
                    real ez = Math<real>::expneg(tau, sp.r2[s]);
                    Math<real>::cis(ph, c, sn);
                    zr[s] = ez * c; zi[s] = -ez * sn;
                    real eZ = Math<real>::expneg(tau * kT, sp.r2[s]);
                    Math<real>::cis(ph * kT, c, sn);
                    Zr[s] = eZ * c; Zi[s] = -eZ * sn;
                }
                for (int n0 = 0; n0 < n; n0 += kT) {
                    real acc[2 * kT];
#pragma unroll
                    for (int t = 0; t < kT; ++t) {
                        real sr = pr[0], si = pi[0];
#pragma unroll
                        for (int s = 1; s < S; ++s) { sr += pr[s]; si += pi[s]; }
                        acc[2 * t] = sr; acc[2 * t + 1] = si;
                        if (t + 1 < kT) {
#pragma unroll
                            for (int s = 0; s < S; ++s) {
                                real a_ = pr[s], b_ = pi[s];
                                pr[s] = a_ * zr[s] - b_ * zi[s];
                                pi[s] = a_ * zi[s] + b_ * zr[s];
                            }
                        }
                    }
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        real a_ = cr[s], b_ = ci[s];
                        cr[s] = a_ * Zr[s] - b_ * Zi[s];
                        ci[s] = a_ * Zi[s] + b_ * Zr[s];
                        pr[s] = cr[s]; pi[s] = ci[s];
                    }
                    const real v = wave_reduce64(acc, lane);
                    s_red[red_buf][wave][lane] = v;
                    __syncthreads();
                    if (wave == 0) {
                        real sum = s_red[red_buf][0][lane];
#pragma unroll
                        for (int w = 1; w < kWaves; ++w) sum += s_red[red_buf][w][lane];
                        if (n0 + (lane >> 1) < n) partial[2 * (int64_t)(aux + n0) + lane] = sum;
                    }
                    red_buf ^= 1;
                }
            }
        }
    }

    if (a.save_state) {
        real* st = reinterpret_cast<real*>(a.state);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t i = base + s * 64 + lane;
            if (i < a.n_spins) {
                st[i] = sp.ar[s]; st[a.n_spins + i] = sp.ai[s]; st[2 * a.n_spins + i] = sp.az[s];
            }
        }
    }
}

template <typename real>
__global__ void finalize_kernel(const real* __restrict__ partial, int64_t n_blocks, int64_t row_stride,
                                int64_t n_vals, double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_vals) return;
    double s = 0.0;
    for (int64_t b = 0; b < n_blocks; ++b) s += (double)partial[b * row_stride + j];
    out[j] = s;
}

__global__ void fill_zero_kernel(double* __restrict__ out, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[j] = 0.0;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename real, int S>
static hipError_t launch_step_t(const StepArgs& a, int64_t n_blocks, hipStream_t st) {
    const size_t dyn = (size_t)a.n_rows * 9 * sizeof(real);
    hipLaunchKernelGGL((step_kernel<real, S>), dim3((unsigned)n_blocks), dim3(kBlock), dyn, st, a);
    return hipGetLastError();
}

int64_t spins_per_block_of(int spins_per_lane) { return (int64_t)kBlock * spins_per_lane; }

hipError_t launch_step(const StepArgs& a, int precision, int spins_per_lane, int64_t n_blocks,
                       hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    if (precision == 64) {
        switch (spins_per_lane) {
            case 1: return launch_step_t<double, 1>(a, n_blocks, st);
            case 2: return launch_step_t<double, 2>(a, n_blocks, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (spins_per_lane) {
        case 1: return launch_step_t<float, 1>(a, n_blocks, st);
        case 2: return launch_step_t<float, 2>(a, n_blocks, st);
        case 4: return launch_step_t<float, 4>(a, n_blocks, st);
        case 8: return launch_step_t<float, 8>(a, n_blocks, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize(const void* partial, int precision, int64_t n_blocks, int64_t row_stride,
                           int64_t n_vals, double* out, hipStream_t st) {
    if (n_vals <= 0) return hipSuccess;
    const int threads = 256;
    const int64_t grid = (n_vals + threads - 1) / threads;
    if (precision == 64)
        hipLaunchKernelGGL(finalize_kernel<double>, dim3((unsigned)grid), dim3(threads), 0, st,
                           reinterpret_cast<const double*>(partial), n_blocks, row_stride, n_vals, out);
    else
        hipLaunchKernelGGL(finalize_kernel<float>, dim3((unsigned)grid), dim3(threads), 0, st,
                           reinterpret_cast<const float*>(partial), n_blocks, row_stride, n_vals, out);
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
