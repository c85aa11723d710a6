// F-stage on the GPU (Sec. 2.3; Sec. 4: 8-bit real ADC samples, 2-tap
// 8192-point polyphase filter bank, 4+4-bit requantisation, a contiguous run
// of channels).  The output is the X-stage input, [channel][spectrum][input]
// CI4 bytes, so the X-stage can run on it directly.
//
// Spectrum m of an input: y[j] = sum_p h[p N + j] x[(m + p) N + j] (N = 8192),
// X[k] = sum_j y[j] e^{-2 pi i jk/N} for the channels k < N/2; then
// v = gain * X[k], each component rounded half to even and saturated to
// [-7, 7].  The real transform runs as one 4096-point complex transform of
// z[n] = y[2n] + i y[2n+1] and a split into the even and odd halves.
//
// Work: a workgroup (256 threads) takes 16 inputs x a run of spectra and
// transforms them one after another.  The 4096-point transform is three
// radix-16 passes (4096 = 16^3) with the data in registers (16 points per
// thread) and two LDS exchanges between them; thread t keeps the filter
// coefficients of the samples it loads in registers for the whole workgroup,
// and the 4-bit results of its 16 channels for the 16 inputs in 64
// registers, so every channel goes out as one 16-byte store of 16 inputs.
// Twiddle factors are LDS tables built once per workgroup in double
// precision.  fp32 arithmetic throughout; bound by VALU work (about 36
// flops per sample against 1.5 bytes of HBM traffic).
#include "xcorr_fstage.h"

namespace xcorr {
namespace {

constexpr int kN = 8192;            // real transform length
constexpr int kThreads = 256;
constexpr int kG = 16;              // inputs per workgroup
constexpr int kSpectra = 8;         // spectra per workgroup
constexpr int kRow = 272;           // LDS row (float2) of a 16 x 256 pass layout
constexpr int kBuf = 16 * kRow;     // 4352 float2

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// 4-point forward DFT in place: (a, b, c, d) -> (X0, X1, X2, X3)
__device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d)
{
    const float2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = csub(b, d);
    a = cadd(s0, s1);
    c = csub(s0, s1);
    b = make_float2(d0.x + d1.y, d0.y - d1.x);    // d0 - i d1
    d = make_float2(d0.x - d1.y, d0.y + d1.x);    // d0 + i d1
}

// W16^m = e^{-2 pi i m / 16} for the products j0 * k0 of the 4 x 4 split
constexpr float kC1 = 0.92387953251128674f;   // cos(pi / 8)
constexpr float kS1 = 0.38268343236508977f;   // sin(pi / 8)
constexpr float kR2 = 0.70710678118654752f;   // cos(pi / 4)

template <int M>
__device__ __forceinline__ float2 w16(float2 v)
{
    if constexpr (M == 0) return v;
    else if constexpr (M == 1) return cmul(v, make_float2(kC1, -kS1));
    else if constexpr (M == 2) return make_float2(kR2 * (v.x + v.y), kR2 * (v.y - v.x));
    else if constexpr (M == 3) return cmul(v, make_float2(kS1, -kC1));
    else if constexpr (M == 4) return make_float2(v.y, -v.x);
    else if constexpr (M == 6) return make_float2(kR2 * (v.y - v.x), -kR2 * (v.x + v.y));
    else return cmul(v, make_float2(-kC1, kS1));  // M == 9
}

// 16-point forward DFT of v[0..15]; the result for frequency k is left in
// v[4 (k % 4) + k / 4] (index j = 4 j1 + j0, k = k0 + 4 k1)
__device__ __forceinline__ void dft16(float2 (&v)[16])
{
#pragma unroll
    for (int j0 = 0; j0 < 4; ++j0) dft4(v[j0], v[4 + j0], v[8 + j0], v[12 + j0]);
    // v[4 k0 + j0] now holds the k0-th output of the j0-th column
    v[5] = w16<1>(v[5]);  v[6] = w16<2>(v[6]);  v[7] = w16<3>(v[7]);
    v[9] = w16<2>(v[9]);  v[10] = w16<4>(v[10]); v[11] = w16<6>(v[11]);
    v[13] = w16<3>(v[13]); v[14] = w16<6>(v[14]); v[15] = w16<9>(v[15]);
#pragma unroll
    for (int k0 = 0; k0 < 4; ++k0) dft4(v[4 * k0], v[4 * k0 + 1], v[4 * k0 + 2], v[4 * k0 + 3]);
}

__device__ __forceinline__ constexpr int slot_of(int k) { return 4 * (k % 4) + k / 4; }

// e^{-2 pi i r / n} in double precision, rounded to float
__device__ __forceinline__ float2 twiddle(int r, int n)
{
    double s, c;
    sincospi(2.0 * r / n, &s, &c);
    return make_float2((float)c, (float)-s);
}

__device__ __forceinline__ uint32_t nibble_pair(float re, float im)
{
    const int qr = (int)fminf(fmaxf(__builtin_rintf(re), -7.0f), 7.0f);
    const int qi = (int)fminf(fmaxf(__builtin_rintf(im), -7.0f), 7.0f);
    return ((uint32_t)(qr & 0xF) << 4) | (uint32_t)(qi & 0xF);
}

template <int P, int OUT>
__global__ void __launch_bounds__(kThreads, 2) fstage_kernel(FstageArgs a)
{
    __shared__ float2 L[kBuf];          // pass exchanges; then Z[k] at k + k / 16
    __shared__ float2 T1[16 * 256];     // [k0][t]  W4096^(t k0)
    __shared__ float2 T2[256];          // [k1][n0] W256^(n0 k1)
    __shared__ float2 TB[16];           // W8192^j

    const int t = threadIdx.x;
    const int n_groups = (a.n_inputs + kG - 1) / kG;
    const int g = blockIdx.x % n_groups;
    const int m0 = (blockIdx.x / n_groups) * kSpectra;
    const int a0 = g * kG;
    const int m1 = min(m0 + kSpectra, a.n_spectra);

#pragma unroll
    for (int k0 = 0; k0 < 16; ++k0) T1[k0 * 256 + t] = twiddle((t * k0) & 4095, 4096);
    T2[t] = twiddle(((t & 15) * (t >> 4)) & 255, 256);
    if (t < 16) TB[t] = twiddle(t, kN);
    const float2 ta = twiddle(16 * t, kN);       // W8192^(16 t)

    // prototype-filter coefficients of the samples this thread loads,
    // h[p N + 512 n2 + 2 t + e]; re-read (from cache) for every transform
    const float2* hc = (const float2*)(a.coeff + 2 * t);

    const int k_first = 16 * t;                  // this thread's channels k_first .. k_first + 15
    const bool full = a0 + kG <= a.n_inputs && (a.n_inputs % 16) == 0;
    __syncthreads();

    for (int m = m0; m < m1; ++m) {
        uint32_t st[16][4];                      // 4-bit results: channel j, inputs 4 w .. 4 w + 3
#pragma unroll
        for (int j = 0; j < 16; ++j)
#pragma unroll
            for (int w = 0; w < 4; ++w) st[j][w] = 0;

        for (int s = 0; s < kG; ++s) {
            const int ai = a0 + s;
            uint32_t q[16];
            if (ai < a.n_inputs) {
                // ---- filter bank: z[256 n2 + t] = y[2n] + i y[2n + 1]
                const uint16_t* x = (const uint16_t*)(a.adc + ai * a.adc_stride + (int64_t)m * kN);
                // an opaque zero keeps the coefficient loads inside the loop
                // (held in registers for the whole workgroup they would not
                // leave room for the 4-bit results)
                int zero;
                asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
                const float2* hz = hc + zero;
                float2 v[16];
#pragma unroll
                for (int n2 = 0; n2 < 16; ++n2) {
                    float re = 0.f, im = 0.f;
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const uint32_t u = x[p * (kN / 2) + 256 * n2 + t];
                        const float2 hh = hz[p * (kN / 2) + 256 * n2];
                        re = fmaf(hh.x, (float)(int8_t)(u & 0xFF), re);
                        im = fmaf(hh.y, (float)(int8_t)(u >> 8), im);
                    }
                    v[n2] = make_float2(re, im);
                    // bound the loads in flight (and their registers)
                    if ((n2 & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                }
                // ---- pass 1 over n2 (thread t = n_lo), twiddle W4096^(n_lo k0)
                dft16(v);
                __syncthreads();                 // previous transform's reads of L are done
#pragma unroll
                for (int k0 = 0; k0 < 16; ++k0) {
                    const float2 y = v[slot_of(k0)];
                    L[k0 * kRow + t] = k0 ? cmul(y, T1[k0 * 256 + t]) : y;
                }
                __syncthreads();
                // ---- pass 2 over n1 (thread = (k0, n0)), twiddle W256^(n0 k1)
                {
                    const int k0 = t >> 4, n0 = t & 15;
#pragma unroll
                    for (int n1 = 0; n1 < 16; ++n1) v[n1] = L[k0 * kRow + 16 * n1 + n0];
                    dft16(v);
                    __syncthreads();
#pragma unroll
                    for (int k1 = 0; k1 < 16; ++k1) {
                        const float2 y = v[slot_of(k1)];
                        L[k0 * kRow + 17 * k1 + n0] = k1 ? cmul(y, T2[k1 * 16 + n0]) : y;
                    }
                }
                __syncthreads();
                // ---- pass 3 over n0 (thread = (k0, k1)): Z[k0 + 16 k1 + 256 k2]
                {
                    const int k0 = t >> 4, k1 = t & 15;
#pragma unroll
                    for (int n0 = 0; n0 < 16; ++n0) v[n0] = L[k0 * kRow + 17 * k1 + n0];
                    dft16(v);
                    __syncthreads();
#pragma unroll
                    for (int k2 = 0; k2 < 16; ++k2) {
                        const int k = k0 + 16 * k1 + 256 * k2;
                        L[k + (k >> 4)] = v[slot_of(k2)];
                    }
                }
                __syncthreads();
                // ---- real split, equalise, requantise this thread's channels
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int k = k_first + j;
                    const int kk = (4096 - k) & 4095;
                    const float2 zk = L[k + (k >> 4)];
                    const float2 zc = L[kk + (kk >> 4)];
                    // E = (Z[k] + conj Z[-k]) / 2, O = -i (Z[k] - conj Z[-k]) / 2
                    const float2 e = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y - zc.y));
                    const float2 o = make_float2(0.5f * (zk.y + zc.y), -0.5f * (zk.x - zc.x));
                    const float2 X = cadd(e, cmul(o, cmul(ta, TB[j])));
                    const int c = k - a.chan_begin;
                    q[j] = 0;
                    if (c >= 0 && c < a.n_chan) {
                        const float gn = a.gain[(int64_t)ai * a.n_chan + c];
                        if constexpr (OUT == 0) {
                            q[j] = nibble_pair(gn * X.x, gn * X.y);
                        } else {
                            float2* o32 = (float2*)a.out;
                            o32[((int64_t)c * a.n_spectra + m) * a.n_inputs + ai] = make_float2(gn * X.x, gn * X.y);
                        }
                    }
                    if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 16; ++j) q[j] = 0;
            }
            if constexpr (OUT == 0) {
                // shift input s's byte in at the top: after 16 inputs input s
                // sits in byte s % 4 of word s / 4
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    st[j][0] = __builtin_amdgcn_alignbit(st[j][1], st[j][0], 8);
                    st[j][1] = __builtin_amdgcn_alignbit(st[j][2], st[j][1], 8);
                    st[j][2] = __builtin_amdgcn_alignbit(st[j][3], st[j][2], 8);
                    st[j][3] = __builtin_amdgcn_alignbit(q[j], st[j][3], 8);
                }
            }
        }
        if constexpr (OUT == 0) {
            uint8_t* o8 = (uint8_t*)a.out;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int c = k_first + j - a.chan_begin;
                if (c < 0 || c >= a.n_chan) continue;
                uint8_t* dst = o8 + ((int64_t)c * a.n_spectra + m) * a.n_inputs + a0;
                if (full) {
                    *(uint4*)dst = make_uint4(st[j][0], st[j][1], st[j][2], st[j][3]);
                } else {
#pragma unroll
                    for (int s = 0; s < kG; ++s)   // constant indices keep st in registers
                        if (a0 + s < a.n_inputs) dst[s] = (uint8_t)(st[j][s >> 2] >> (8 * (s & 3)));
                }
            }
        }
    }
}

template <int P>
hipError_t launch_p(const FstageArgs& a, dim3 grid, hipStream_t s)
{
    if (a.out_kind == 0) hipLaunchKernelGGL((fstage_kernel<P, 0>), grid, dim3(kThreads), 0, s, a);
    else                 hipLaunchKernelGGL((fstage_kernel<P, 1>), grid, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fstage(const FstageArgs& a, hipStream_t s)
{
    if (a.n_spectra <= 0) return hipSuccess;
    const int64_t n_groups = (a.n_inputs + kG - 1) / kG;
    const int64_t blocks = n_groups * ((a.n_spectra + kSpectra - 1) / kSpectra);
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks);
    return a.n_taps == 1 ? launch_p<1>(a, grid, s) : launch_p<2>(a, grid, s);
}

}  // namespace xcorr
