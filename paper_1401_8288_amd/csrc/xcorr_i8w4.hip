// int8 MFMA X-stage kernel, one wave per SIMD (tile variant XCORR_TILE_W4).
//
// The same arithmetic as xcorr_i8.hip (Sec. 1, Sec. 2.4: per channel the
// lower triangle of sum_t x x^H; the complex product split into
// v_mfma_i32_16x16x64_i8 contractions over time, Re with one accumulator, Im
// with two), with a different balance of resources: four waves per
// workgroup, one per SIMD, each owning a whole 64x64 tile (16 blocks, 192
// int32 accumulators, kept in the accumulator registers).  Per MFMA a wave
// then reads a third fewer operand bytes from LDS and spends a third fewer
// vector instructions splitting 4-bit samples than with two waves of half
// tiles, at the price of a single instruction stream per SIMD.
//
// Staging is the LDS-DMA scheme: every step of 64 samples, wave s copies
// slot s (64 sample rows x 64 inputs, four 1-KB buffer loads straight into
// LDS, chunk-swizzled so that the transpose reads are free of bank
// conflicts); kDepth buffers are in flight.  The launch is persistent: one
// workgroup per CU walks a static slice of the work items of its XCD and
// copies the next item's first steps before the current item's epilogue.
#include "xcorr_device.h"

#include <utility>

namespace xcorr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kStep = 64;                       // samples per LDS buffer
constexpr int kDepth = 4;                       // LDS buffers (steps in flight)
constexpr int kSlotBytes = kRowBlock * kRowBlock;   // 64 rows of 64 bytes
constexpr int kBufBytes = kSlots * kSlotBytes;

__device__ __forceinline__ int swz(int row)
{
    return ((row >> 2) & 1) | ((((row >> 1) ^ (row >> 4)) & 1) << 1);
}

// Copies of one slot: lane l of copy j writes row 16 j + l / 4, position
// l % 4, i.e. chunk (l % 4) ^ swz(row) of that sample row.
struct Stager {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t vofs[4];
    int lds_ofs;
    int row_bytes;

    __device__ __forceinline__ void init(const LaunchArgs& a, const WaveJob& w, int lane)
    {
        row_bytes = a.row_bytes;
        rsrc = channel_rsrc(a, w.stage_rb, w.stage_ch);
        lds_ofs = w.stage_slot * kSlotBytes;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 16 * j + (lane >> 2);
            const int q = (lane & 3) ^ swz(row);
            const int input = (w.stage_rb < 0 ? 0 : w.stage_rb) * kRowBlock + 16 * q;
            vofs[j] = (uint32_t)row * (uint32_t)a.row_bytes + column_offset(input, a.n_inputs, 1);
        }
    }

    __device__ __forceinline__ void load(uint8_t* buf, int k) const
    {
        typedef __attribute__((address_space(3))) void lds_void;
        const uint32_t step = (uint32_t)(k * kStep) * (uint32_t)row_bytes;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void*)(buf + lds_ofs + 16 * kRowBlock * j), 16,
                                                     (int)(vofs[j] + step), 0, 0, 0);
    }
};

// Operand fragment of block blk of a slot: lane l gets input 16 blk + l % 16
// for samples 16 (l / 16)..+15, from two transpose reads of 8 sample rows.
__device__ __forceinline__ int tr_offset(int slot, int blk, int lane)
{
    const int j = lane & 15;
    const int row = 16 * (lane >> 4) + (j >> 1);
    return slot * kSlotBytes + row * kRowBlock + 16 * (blk ^ swz(row)) + 8 * (j & 1);
}

__device__ __forceinline__ v4i frag_tr(const uint8_t* buf, int ofs)
{
    typedef int v2i __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) v2i lds_v2i;
    const v2i lo = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i*)(buf + ofs));
    const v2i hi = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i*)(buf + ofs + 8 * kRowBlock));
    return v4i{lo.x, lo.y, hi.x, hi.y};
}

// CI4 byte = (re << 4) | (im & 0xF): masking gives 16 re and 16 im as exact int8.
__device__ __forceinline__ v4i hi16(v4i x)
{
    const int m = (int)0xF0F0F0F0u;
    return x & v4i{m, m, m, m};
}
__device__ __forceinline__ v4i lo16(v4i x)
{
    const int m = (int)0xF0F0F0F0u;
    return (x << 4) & v4i{m, m, m, m};
}

struct Acc {
    v4i re[4][4], ab[4][4], ba[4][4];
};
struct Raw {
    v4i ri[4], rj[4];
};
struct Ops {
    v4i ia[4], ib[4], ja[4], jb[4];
};

template <int KIND>
__device__ __forceinline__ constexpr bool diag_kind()
{
    return KIND == KIND_DIAG;
}

template <int KIND>
__device__ __forceinline__ constexpr bool need_i(int b)
{
    return row_on(KIND, b) || (diag_kind<KIND>() && column_on(KIND, b));
}

template <int KIND>
__device__ __forceinline__ constexpr bool need_j(int b)
{
    return column_on(KIND, b) && !diag_kind<KIND>();
}

template <int KIND>
__device__ __forceinline__ void read_raw(const uint8_t* buf, const int* oi, const int* oj, Raw& r)
{
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (need_i<KIND>(b)) r.ri[b] = frag_tr(buf, oi[b]);
        if (need_j<KIND>(b)) r.rj[b] = frag_tr(buf, oj[b]);
    }
}

template <int KIND>
__device__ __forceinline__ void prepare(const Raw& r, Ops& o)
{
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (need_i<KIND>(b)) {
            o.ia[b] = hi16(r.ri[b]);
            o.ib[b] = lo16(r.ri[b]);
        }
        if (need_j<KIND>(b)) {
            o.ja[b] = hi16(r.rj[b]);
            o.jb[b] = lo16(r.rj[b]);
        }
        if (diag_kind<KIND>() && column_on(KIND, b)) {
            o.ja[b] = o.ia[b];
            o.jb[b] = o.ib[b];
        }
    }
}

template <int KIND>
__device__ __forceinline__ constexpr int n_frags()
{
    int n = 0;
    for (int b = 0; b < 4; ++b) n += (need_i<KIND>(b) ? 1 : 0) + (need_j<KIND>(b) ? 1 : 0);
    return n;
}

// The MFMAs of one step, term-major (the two MFMAs into one Re accumulator
// are far apart).
template <int KIND>
__device__ __forceinline__ void mma(const Ops& o, Acc& c)
{
#pragma unroll
    for (int term = 0; term < 4; ++term)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) {
                if (!block_on(KIND, bi, bj)) continue;
                if (term == 0) c.re[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ia[bi], o.ja[bj], c.re[bi][bj], 0, 0, 0);
                if (term == 1) c.ab[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ia[bi], o.jb[bj], c.ab[bi][bj], 0, 0, 0);
                if (term == 2) c.ba[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ib[bi], o.ja[bj], c.ba[bi][bj], 0, 0, 0);
                if (term == 3) c.re[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ib[bi], o.jb[bj], c.re[bi][bj], 0, 0, 0);
            }
}

template <int N>
__device__ __forceinline__ void wait_vm_lgkm()
{
    static_assert(N >= 0 && N < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | (0x7 << 4) | ((N >> 4) << 14));
}

// Barrier without the workgroup fence (which would wait for every LDS-DMA
// copy in flight): own copies older than the newest N and own LDS reads done.
template <int N>
__device__ __forceinline__ void dma_barrier()
{
    __builtin_amdgcn_sched_barrier(0);
    wait_vm_lgkm<N>();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Each LDS buffer is its own variable so that the compiler can tell a copy
// into one from the reads of another.
struct Bufs {
    uint8_t* p[kDepth];
};

// Step k (buffer S = k % kDepth): copy step k + kDepth into buffer S (whose
// fragments were read in step k-1), read the fragments of step k+1, run the
// MFMAs of step k with the splitting of step k+1 in their shadow, wait for
// own copy of step k+2, barrier.
template <int KIND, int S>
__device__ __forceinline__ void step(int k, const Stager& st, const Bufs& L, const int* oi, const int* oj, Ops& ops,
                                     Acc& c)
{
    constexpr int D = kDepth;
    st.load(L.p[S], k + D);
    Ops nx;
    if constexpr (KIND != KIND_NONE) {
        Raw raw;
        read_raw<KIND>(L.p[(S + 1) % D], oi, oj, raw);
        mma<KIND>(ops, c);
        prepare<KIND>(raw, nx);
        constexpr int nm = 4 * __builtin_popcount(kind_mask(KIND));
        constexpr int lead = nm / 4;
        constexpr int n_valu = 12 * n_frags<KIND>();
        constexpr int vpm = (n_valu + (nm - lead) - 1) / (nm - lead);
        __builtin_amdgcn_sched_group_barrier(0x010, 4, 0);                    // copies
        __builtin_amdgcn_sched_group_barrier(0x100, 2 * n_frags<KIND>(), 0);  // fragment reads
        __builtin_amdgcn_sched_group_barrier(0x008, lead, 0);                 // MFMAs while they return
#pragma unroll
        for (int m = lead; m < nm; ++m) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, vpm, 0);
        }
    }
    dma_barrier<4 * (D - 2)>();
    ops = nx;
}

template <int KIND, int... S>
__device__ __forceinline__ void group(int k0, const Stager& st, const Bufs& L, const int* oi, const int* oj, Ops& ops,
                                      Acc& c, std::integer_sequence<int, S...>)
{
    (step<KIND, S>(k0 + S, st, L, oi, oj, ops, c), ...);
}

template <int KIND>
__device__ __forceinline__ void run_tile(const LaunchArgs& a, const WaveJob& w, int lane, const Bufs& L,
                                         const Stager& st, bool has_next, const Stager& nst, bool issue_prologue)
{
    constexpr int D = kDepth;
    const int nk = (a.t_len + kStep - 1) / kStep;
    Acc c;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            if (!block_on(KIND, bi, bj)) continue;
            c.re[bi][bj] = v4i{0, 0, 0, 0};
            c.ab[bi][bj] = v4i{0, 0, 0, 0};
            c.ba[bi][bj] = v4i{0, 0, 0, 0};
        }
    int oi[4], oj[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        oi[b] = tr_offset(w.si, b, lane);
        oj[b] = tr_offset(w.sj, b, lane);
    }
    // Prologue: copies of steps 0..D-1 (unless the previous item issued
    // them), operands of step 0; the second barrier frees buffer 0.
    if (issue_prologue) {
#pragma unroll
        for (int s = 0; s < D; ++s) st.load(L.p[s], s);
    }
    dma_barrier<4 * (D - 1)>();
    Ops ops;
    if constexpr (KIND != KIND_NONE) {
        Raw raw;
        read_raw<KIND>(L.p[0], oi, oj, raw);
        prepare<KIND>(raw, ops);
    }
    dma_barrier<4 * (D - 2)>();
    for (int k0 = 0; k0 < nk; k0 += D)
        group<KIND>(k0, st, L, oi, oj, ops, c, std::make_integer_sequence<int, D>());
    // trailing copies (zeros past the window) land; then the next item's
    // first steps, which overlap this item's epilogue
    wait_vm_lgkm<0>();
    if (has_next) {
#pragma unroll
        for (int s = 0; s < D; ++s) nst.load(L.p[s], s);
    }
    if constexpr (KIND == KIND_NONE) return;

    // Epilogue: 16x16 int32 blocks hold column lane % 16 and rows
    // 4 (lane / 16) + r in register r; products carry the factor 256.
    const int ch = w.tile_ch;
    if (ch >= a.n_channels) return;
    const int i0 = w.rb_i * kRowBlock, j0 = w.rb_j * kRowBlock;
    const int64_t nb = (int64_t)a.n_inputs * (a.n_inputs + 1) / 2;
    const int64_t* src = (const int64_t*)a.src;
    int64_t* dst = (int64_t*)a.dst;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            if (!block_on(KIND, bi, bj)) continue;
            const int j = j0 + 16 * bj + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * bi + 4 * (lane >> 4) + r;
                if (i >= a.n_inputs || j > i) continue;
                int64_t re = ((int64_t)c.re[bi][bj][r]) >> 8;
                int64_t im = ((int64_t)c.ba[bi][bj][r] - (int64_t)c.ab[bi][bj][r]) >> 8;
                const int64_t idx = ((int64_t)ch * nb + (int64_t)i * (i + 1) / 2 + j) * 2;
                if (src) {
                    const longlong2 s = *(const longlong2*)(src + idx);
                    re += s.x;
                    im += s.y;
                }
                longlong2 o;
                o.x = re;
                o.y = im;
                *(longlong2*)(dst + idx) = o;
            }
        }
}

__device__ __forceinline__ void dispatch(const LaunchArgs& a, const WaveJob& w, int lane, const Bufs& L,
                                         const Stager& st, bool has_next, const Stager& nst, bool issue)
{
    switch (w.kind) {
    case KIND_FULL:  run_tile<KIND_FULL>(a, w, lane, L, st, has_next, nst, issue); break;
    case KIND_DIAG:  run_tile<KIND_DIAG>(a, w, lane, L, st, has_next, nst, issue); break;
    case KIND_HALF0: run_tile<KIND_HALF0>(a, w, lane, L, st, has_next, nst, issue); break;
    case KIND_HALF1: run_tile<KIND_HALF1>(a, w, lane, L, st, has_next, nst, issue); break;
    default:         run_tile<KIND_NONE>(a, w, lane, L, st, has_next, nst, issue); break;
    }
}

__device__ __forceinline__ int entry_of(const BatchArgs& ba, int g)
{
    int e = 0;
    while (e + 1 < ba.n_entries && g >= ba.first[e + 1]) ++e;
    return e;
}

// Persistent launch: workgroup j of XCD x takes items slice[x] + j + m P.
__global__ void __launch_bounds__(kThreads, 1) xcorr_i8w4_kernel(BatchArgs ba)
{
    __shared__ __attribute__((aligned(16))) uint8_t b0[kBufBytes], b1[kBufBytes], b2[kBufBytes], b3[kBufBytes];
    static_assert(kDepth == 4, "one LDS variable per buffer");
    const Bufs L{{b0, b1, b2, b3}};
    const int q = ba.xcd_map ? (int)(blockIdx.x & 7) : 0;
    const int j = ba.xcd_map ? (int)(blockIdx.x >> 3) : (int)blockIdx.x;
    const int P = ba.xcd_map ? (int)(gridDim.x >> 3) : (int)gridDim.x;
    const int lo = ba.xcd_map ? ba.slice[q] : ba.slice[0];
    const int hi = ba.xcd_map ? ba.slice[q + 1] : ba.slice[8];
    int g = lo + j;
    if (g >= hi) return;
    const int lane = threadIdx.x & 63;
    int e = entry_of(ba, g);
    WaveJob w = wave_job<kWaves>(ba.e[e], g - ba.first[e]);
    Stager st;
    st.init(ba.e[e], w, lane);
    bool issue = true;
    for (;;) {
        const int gn = g + P;
        const bool has_next = gn < hi;
        int en = e;
        WaveJob wn = w;
        Stager nst = st;
        if (has_next) {
            en = entry_of(ba, gn);
            wn = wave_job<kWaves>(ba.e[en], gn - ba.first[en]);
            nst.init(ba.e[en], wn, lane);
        }
        dispatch(ba.e[e], w, lane, L, st, has_next, nst, issue);
        if (!has_next) break;
        g = gn;
        e = en;
        w = wn;
        st = nst;
        issue = false;
    }
}

}  // namespace

hipError_t launch_i8w4(const BatchArgs& ba, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(xcorr_i8w4_kernel, dim3(grid), dim3(kThreads), 0, s, ba);
    return hipGetLastError();
}

}  // namespace xcorr
