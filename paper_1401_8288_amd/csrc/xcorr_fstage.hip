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
// Work: a workgroup (256 threads) takes one input and a run of spectra and
// transforms them one after another.  The 4096-point transform is three
// radix-16 passes (4096 = 16^3) with the data in registers (16 points per
// thread) and LDS exchanges between them.  Thread t keeps the filter
// coefficients of the samples it loads and the input's gains for its 16
// channels in registers for the whole run, and the next spectrum's samples
// load while the current one is transformed.  Its 16 channels' codes go out
// as one 16-byte store, input-major; a second, HBM-bound kernel transposes
// them into X-stage order, chunk by chunk beside the next chunk's transform.
// Twiddle factors are built once per workgroup in double precision (LDS
// tables for the passes, registers for the real split).  fp32 arithmetic
// throughout; bound by VALU work (about 36 flops per sample against 2.5
// bytes of HBM traffic, the transpose included).
#include "xcorr_fstage.h"

#include <algorithm>
#include <mutex>

namespace xcorr {
namespace {

constexpr int kN = 8192;            // real transform length
constexpr int kThreads = 256;
constexpr int kSpectra = 32;        // spectra per workgroup
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

// LDS writes visible, then a workgroup barrier; global loads stay in flight
// (__syncthreads would also wait for them)
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// raw 16-bit pairs (samples 2n, 2n + 1, n = 256 n2 + t) of the P frames of spectrum m
template <int P>
__device__ __forceinline__ void load_frames(uint32_t (&xr)[P][16], const uint16_t* x, int t)
{
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) xr[p][n2] = x[p * (kN / 2) + 256 * n2 + t];
}

// One workgroup: one input, spectra m0 .. m0 + kSpectra - 1.
// OUT 0: 4-bit codes in input-major order, work[m][a][cp] with channel
//        k at cp = k - base (base = chan_begin rounded down to 16), one
//        16-byte store per thread (channels outside the selection get 0);
// OUT 1: equalised values, float2 out[c][m][a].
template <int P, int OUT>
__global__ void __launch_bounds__(kThreads, 2) fstage_kernel(FstageArgs a)
{
    __shared__ float2 L[kBuf];          // pass exchanges; then Z[k] at k + k / 16
    __shared__ float2 T1[16 * 256];     // [k0][t]  W4096^(t k0)
    __shared__ float2 T2[256];          // [k1][n0] W256^(n0 k1)

    const int t = threadIdx.x;
    const int ai = blockIdx.x % a.n_inputs;
    const int m0 = a.m_begin + (blockIdx.x / a.n_inputs) * kSpectra;
    const int m1 = min(m0 + kSpectra, a.m_end);
    const int k_first = 16 * t;                  // this thread's channels k_first .. k_first + 15
    const int base = a.chan_begin & ~15;

    const uint16_t* xa = (const uint16_t*)(a.adc + ai * a.adc_stride);
    uint32_t xr[P][16];
    load_frames<P>(xr, xa + (int64_t)m0 * (kN / 2), t);

#pragma unroll
    for (int k0 = 0; k0 < 16; ++k0) T1[k0 * 256 + t] = twiddle((t * k0) & 4095, 4096);
    T2[t] = twiddle(((t & 15) * (t >> 4)) & 255, 256);
    // W8192^k for this thread's channels k = 16 t + j: W^(16 t) times
    // powers of W^1, multiplied out in double precision, then rounded
    float2 wk[16];
    {
        double br, bi, sr, si;
        sincospi(2.0 * (16 * t) / kN, &bi, &br);
        sincospi(2.0 / kN, &si, &sr);
        bi = -bi;
        si = -si;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            wk[j] = make_float2((float)br, (float)bi);
            const double nr = br * sr - bi * si, ni = br * si + bi * sr;
            br = nr;
            bi = ni;
        }
    }

    // prototype-filter coefficients of this thread's samples,
    // h[p N + 512 n2 + 2 t + e], and the input's gains for its channels
    float2 h[P][16];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) h[p][n2] = *(const float2*)(a.coeff + p * kN + 512 * n2 + 2 * t);
    float gh[16];                                // gain / 2 (the split's 1/2 folded in)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int c = k_first + j - a.chan_begin;
        gh[j] = (c >= 0 && c < a.n_chan) ? 0.5f * a.gain[(int64_t)ai * a.n_chan + c] : 0.0f;
    }
    const bool writes = k_first + 16 > a.chan_begin && k_first < a.chan_begin + a.n_chan;
    __syncthreads();

    for (int m = m0; m < m1; ++m) {
        // ---- filter bank: z[256 n2 + t] = y[2n] + i y[2n + 1]
        float2 v[16];
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                re = fmaf(h[p][n2].x, (float)(int8_t)(xr[p][n2] & 0xFF), re);
                im = fmaf(h[p][n2].y, (float)(int8_t)(xr[p][n2] >> 8), im);
            }
            v[n2] = make_float2(re, im);
        }
        // the next spectrum's samples load while this one is transformed
        if (m + 1 < m1) load_frames<P>(xr, xa + (int64_t)(m + 1) * (kN / 2), t);

        // ---- pass 1 over n2 (thread t = n_lo), twiddle W4096^(n_lo k0)
        dft16(v);
        // the twiddles are read before the barrier, so that their latency
        // overlaps the wait (the float-output kernel has no registers for it)
        float2 tw[16];
        if constexpr (OUT == 0) {
#pragma unroll
            for (int k0 = 1; k0 < 16; ++k0) tw[k0] = T1[k0 * 256 + t];
        }
        lds_barrier();                           // previous transform's reads of L are done
#pragma unroll
        for (int k0 = 0; k0 < 16; ++k0) {
            const float2 y = v[slot_of(k0)];
            L[k0 * kRow + t] = k0 ? cmul(y, OUT == 0 ? tw[k0] : T1[k0 * 256 + t]) : y;
        }
        lds_barrier();
        // ---- pass 2 over n1 (thread = (k0, n0)), twiddle W256^(n0 k1)
        {
            const int k0 = t >> 4, n0 = t & 15;
#pragma unroll
            for (int n1 = 0; n1 < 16; ++n1) v[n1] = L[k0 * kRow + 16 * n1 + n0];
            dft16(v);
            float2 tw2[16];
            if constexpr (OUT == 0) {
#pragma unroll
                for (int k1 = 1; k1 < 16; ++k1) tw2[k1] = T2[k1 * 16 + n0];
            }
            lds_barrier();
#pragma unroll
            for (int k1 = 0; k1 < 16; ++k1) {
                const float2 y = v[slot_of(k1)];
                L[k0 * kRow + 17 * k1 + n0] = k1 ? cmul(y, OUT == 0 ? tw2[k1] : T2[k1 * 16 + n0]) : y;
            }
        }
        lds_barrier();
        // ---- pass 3 over n0 (thread = (k0, k1)): Z[k0 + 16 k1 + 256 k2]
        {
            const int k0 = t >> 4, k1 = t & 15;
#pragma unroll
            for (int n0 = 0; n0 < 16; ++n0) v[n0] = L[k0 * kRow + 17 * k1 + n0];
            dft16(v);
            lds_barrier();
#pragma unroll
            for (int k2 = 0; k2 < 16; ++k2) {
                const int k = k0 + 16 * k1 + 256 * k2;
                L[k + (k >> 4)] = v[slot_of(k2)];
            }
        }
        lds_barrier();
        // ---- real split, equalise, requantise this thread's channels
        if (writes) {
            uint32_t q[4] = {0, 0, 0, 0};
            // Z[-k] for k = 16 t + j sits at 4351 - 17 t - j (j > 0) and
            // at 4352 - 17 t (j = 0, t > 0) of the padded layout
            const float2* zc_lo = L + (4336 - 17 * t);
            const int zc0 = t ? 4352 - 17 * t : 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int k = k_first + j;
                const float2 zk = L[k + (k >> 4)];
                const float2 zc = j ? zc_lo[15 - j] : L[zc0];
                // X = (s - i W8192^k d) / 2 with s = Z[k] + conj Z[-k] and
                // d = Z[k] - conj Z[-k] (the even- and odd-sample transforms)
                const float sx = zk.x + zc.x, sy = zk.y - zc.y, dx = zk.x - zc.x, dy = zk.y + zc.y;
                const float2 w = wk[j];
                const float vr = gh[j] * fmaf(w.x, dy, fmaf(w.y, dx, sx));
                const float vi = gh[j] * fmaf(-w.x, dx, fmaf(w.y, dy, sy));
                if constexpr (OUT == 0) {
                    // clamp to [-7, 7], then round half to even by adding
                    // 1.5 * 2^23: the integer is left in the low mantissa
                    // bits, two's complement
                    const uint32_t br = __float_as_uint(__builtin_amdgcn_fmed3f(vr, -7.0f, 7.0f) + 12582912.0f);
                    const uint32_t bi = __float_as_uint(__builtin_amdgcn_fmed3f(vi, -7.0f, 7.0f) + 12582912.0f);
                    q[j >> 2] |= (((br & 0xFu) << 4) | (bi & 0xFu)) << (8 * (j & 3));
                } else {
                    const int c = k - a.chan_begin;
                    if (c >= 0 && c < a.n_chan)
                        ((float2*)a.out)[((int64_t)c * a.n_spectra + m) * a.n_inputs + ai] = make_float2(vr, vi);
                }
            }
            if constexpr (OUT == 0)
                *(uint4*)((uint8_t*)a.work + ((int64_t)m * a.n_inputs + ai) * a.cp + (k_first - base)) =
                    make_uint4(q[0], q[1], q[2], q[3]);
        }
    }
}

// work[m][a][cp] -> out[c][m][a] (c = cp - (chan_begin - base)), bytes.  A
// workgroup moves 128-input x 128-channel tiles of one spectrum each (a
// grid smaller than the tile count loops over them): 16-byte loads along
// channels, 4 x 4 byte transposes in registers, an LDS tile of
// [input / 4][channel] dwords, and 16-byte stores along inputs, eight lanes
// to a 128-byte row on both sides.
__global__ void __launch_bounds__(kThreads) fstage_transpose_kernel(FstageArgs a)
{
    __shared__ uint32_t T[32][128 + 4];
    const int t = threadIdx.x;
    const int n_ct = (a.cp + 127) / 128;
    // spectra vary fastest over the tiles: workgroups running together touch
    // neighbouring rows of both buffers (few pages)
    const int n_m = a.m_end - a.m_begin;
    const int n_tiles = n_ct * ((a.n_inputs + 127) / 128) * n_m;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        int b = tile;
        const int m = a.m_begin + b % n_m;  b /= n_m;
        const int ct = b % n_ct;
        const int at = b / n_ct;
        const int cp0 = ct * 128, a0 = at * 128;
        const int off = a.chan_begin - (a.chan_begin & ~15);
        const uint8_t* w = (const uint8_t*)a.work;

        {
            // 16-byte loads: lane (c16, aq) reads channels cp0 + 16 c16 .. + 15
            // of inputs a0 + 4 aq .. + 3; eight lanes cover a 128-byte row
            const int c16 = t & 7, aq = t >> 3;
            const int cp = cp0 + 16 * c16;
            uint4 r[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ar = a0 + 4 * aq + k;
                r[k] = (ar < a.n_inputs && cp < a.cp)
                           ? *(const uint4*)(w + ((int64_t)m * a.n_inputs + ar) * a.cp + cp) : make_uint4(0, 0, 0, 0);
            }
            const uint32_t* rr[4] = {&r[0].x, &r[1].x, &r[2].x, &r[3].x};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // 4 x 4 byte transpose of channels 4 j .. + 3: column cc holds
                // the four inputs of channel 4 j + cc
                const uint32_t r0 = rr[0][j], r1 = rr[1][j], r2 = rr[2][j], r3 = rr[3][j];
                const uint32_t t0 = __builtin_amdgcn_perm(r1, r0, 0x05010400u);
                const uint32_t t1 = __builtin_amdgcn_perm(r1, r0, 0x07030602u);
                const uint32_t t2 = __builtin_amdgcn_perm(r3, r2, 0x05010400u);
                const uint32_t t3 = __builtin_amdgcn_perm(r3, r2, 0x07030602u);
                uint4 col;
                col.x = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
                col.y = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
                col.z = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
                col.w = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
                *(uint4*)&T[aq][16 * c16 + 4 * j] = col;
            }
        }
        __syncthreads();
        {
            // eight lanes write one channel's 128 inputs: full 128-byte rows
            const int q = t & 7;                     // inputs a0 + 16 q .. + 15
            const int ab = a0 + 16 * q;
#pragma unroll
            for (int pass = 0; pass < 4; ++pass) {
                const int cl = 32 * pass + (t >> 3);
                const int c = cp0 + cl - off;        // output channel
                if (c < 0 || c >= a.n_chan || cp0 + cl >= a.cp || ab >= a.n_inputs) continue;
                const uint4 d = make_uint4(T[4 * q][cl], T[4 * q + 1][cl], T[4 * q + 2][cl], T[4 * q + 3][cl]);
                uint8_t* o = (uint8_t*)a.out + ((int64_t)c * a.n_spectra + m) * a.n_inputs + ab;
                if (ab + 16 <= a.n_inputs && (a.n_inputs & 15) == 0) {
                    *(uint4*)o = d;
                } else {
                    const uint32_t dw[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        if (ab + k < a.n_inputs) o[k] = (uint8_t)(dw[k >> 2] >> (8 * (k & 3)));
                }
            }
        }
        __syncthreads();                         // T is refilled by the next tile
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

int64_t fstage_work_bytes(int n_inputs, int64_t n_spectra, int chan_begin, int n_chan)
{
    const int64_t base = chan_begin & ~15;
    const int64_t cp = (chan_begin + n_chan + 15) / 16 * 16 - base;
    return (int64_t)n_inputs * n_spectra * cp;
}

namespace {

// The transpose of a chunk of spectra runs on a second stream while the next
// chunk is transformed (the transform is bound by the vector ALU, the
// transpose by HBM, and a CU holds two transform workgroups and a transpose
// one at once).  Each caller stream gets a side stream and events of its own
// (per device, created on first use and kept for the process), so that
// calls on different caller streams never wait for each other through a
// shared side stream; past kMaxSides caller streams on a device, or if one
// cannot be created, a call runs its chunks in order on the caller's stream.
// Enqueue sequences on a device are serialised.
constexpr int kChunks = 8;
constexpr int kMaxDevices = 64;
constexpr int kMaxSides = 16;

struct Side {
    hipStream_t caller = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev[kChunks + 1] = {};
};
struct DeviceSides {
    std::mutex mu;
    int n = 0;
    Side side[kMaxSides];
};
DeviceSides g_sides[kMaxDevices];

// The side stream of caller stream s (lock held), or null.
Side* side_of(DeviceSides& d, hipStream_t s)
{
    for (int i = 0; i < d.n; ++i)
        if (d.side[i].caller == s) return &d.side[i];
    if (d.n == kMaxSides) return nullptr;
    Side sd;
    sd.caller = s;
    hipError_t e = hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking);
    for (int k = 0; e == hipSuccess && k <= kChunks; ++k) e = hipEventCreateWithFlags(&sd.ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        for (int k = 0; k <= kChunks; ++k)
            if (sd.ev[k]) (void)hipEventDestroy(sd.ev[k]);
        if (sd.stream) (void)hipStreamDestroy(sd.stream);
        return nullptr;
    }
    d.side[d.n] = sd;
    return &d.side[d.n++];
}

template <int P>
hipError_t launch_transform(FstageArgs a, hipStream_t s)
{
    const int64_t blocks = (int64_t)a.n_inputs * ((a.m_end - a.m_begin + kSpectra - 1) / kSpectra);
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    return launch_p<P>(a, dim3((unsigned)blocks), s);
}

// max_groups > 0 caps the grid (the workgroups then loop over the tiles)
hipError_t launch_transpose(const FstageArgs& a, hipStream_t s, int64_t max_groups = 0)
{
    const int64_t tiles = (int64_t)((a.cp + 127) / 128) * ((a.n_inputs + 127) / 128) * (a.m_end - a.m_begin);
    if (tiles > 0x7fffffff) return hipErrorInvalidConfiguration;
    const int64_t grid = max_groups > 0 ? std::min(tiles, max_groups) : tiles;
    hipLaunchKernelGGL(fstage_transpose_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fstage(FstageArgs a, hipStream_t s)
{
    if (a.n_spectra <= 0) return hipSuccess;
    a.cp = (int32_t)((a.chan_begin + a.n_chan + 15) / 16 * 16 - (a.chan_begin & ~15));
    auto transform = [&](const FstageArgs& c) {
        return a.n_taps == 1 ? launch_transform<1>(c, s) : launch_transform<2>(c, s);
    };
    const int groups = (a.n_spectra + kSpectra - 1) / kSpectra;
    int dev = 0;
    Side* sd = nullptr;
    std::unique_lock<std::mutex> lk;
    if (a.out_kind == 0 && groups >= 4 * kChunks && hipGetDevice(&dev) == hipSuccess && dev >= 0 &&
        dev < kMaxDevices) {
        lk = std::unique_lock<std::mutex>(g_sides[dev].mu);
        sd = side_of(g_sides[dev], s);
        if (!sd) lk.unlock();
    }
    if (!sd) {
        a.m_begin = 0;
        a.m_end = a.n_spectra;
        hipError_t e = transform(a);
        if (e != hipSuccess || a.out_kind != 0) return e;
        return launch_transpose(a, s);
    }
    // chunks of whole workgroup runs; the side stream starts after the work
    // already on s and s continues after the last transpose.  Beside a
    // transform the transposes run as 3 workgroups per CU looping over their
    // tiles: spread over more of the transform's time they slow it less
    // (21.1 ms against 21.4 for the LWA-size stage with one workgroup per
    // tile; 2 per CU: 21.2)
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0) {
        (void)hipGetLastError();
        n_cu = 256;
    }
    const int per = (groups + kChunks - 1) / kChunks;
    for (int c = 0; c < kChunks; ++c) {
        FstageArgs ac = a;
        ac.m_begin = std::min(c * per * kSpectra, a.n_spectra);
        ac.m_end = std::min((c + 1) * per * kSpectra, a.n_spectra);
        if (ac.m_begin >= ac.m_end) break;
        hipError_t e = transform(ac);
        if (e == hipSuccess) e = hipEventRecord(sd->ev[c], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(sd->stream, sd->ev[c], 0);
        if (e == hipSuccess) e = launch_transpose(ac, sd->stream, 3 * (int64_t)n_cu);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(sd->ev[kChunks], sd->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, sd->ev[kChunks], 0);
    return e;
}

}  // namespace xcorr
