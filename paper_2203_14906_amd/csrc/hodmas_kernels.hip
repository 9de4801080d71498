// Fused HO-DMAS beamforming kernel for gfx950 (MI355X).
//
// One workgroup (4 wave64) forms one pixel tile.  Per pixel and element it
//   1. rebuilds the one-way delay from the tile's float64 anchor (registers),
//   2. gathers the two neighbouring samples from an LDS window that the
//      workgroup staged with coalesced channel-major loads, and interpolates,
//   3. takes the signed k-th root y = sign(s)|s|^(1/k)       (Eq. 2, Eqs. 4-6),
//   4. accumulates the power sums p_j = sum y^j, j = 1..k, with compensated
//      float32 summation (pairwise groups of four, Kahan steps per 32 elements),
// and per pixel recovers the order-k symmetric sum e_k from p_1..p_k with
// Newton's identities (the general form of Eqs. 3, 7, 8 and 9):
//   e_0 = 1,  m e_m = sum_{j=1..m} (-1)^(j-1) e_{m-j} p_j.
// The recovery runs in float32 for k <= 4 and in float64 for k >= 5, where the
// alternating terms cancel more.  y^k is taken as the sample itself (odd k) or
// its magnitude (even k), exactly as the paper's forms use sum s and sum |s|.
//
// Per-element constants are wave-uniform (every lane of a wave works on the same
// element at the same time), so they live in SGPRs via scalar loads; the
// per-pixel state lives in VGPRs.  No MFMA: this is gather + VALU work.
// Template parameter M = 2 pairs each pixel with its mirror image about x = 0
// (one delay serves both; see process_tile).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "hodmas_internal.h"

namespace hodmas {
namespace {

// Read-only tables; wave-uniform indices let the compiler use scalar loads.
using ConstTile = const hodmas_tile_desc* __restrict__;
using ConstEntry = const hodmas_chan_entry* __restrict__;
using ConstStage = const hodmas_stage_entry* __restrict__;

// The tables and work lists are never written by a kernel.  Their elements
// are read through the constant address space, which says so: loads at
// wave-uniform addresses then become scalar loads even after the kernel has
// stored to global memory (the batch kernels store a tile's pixels before
// reading the next tile's entries), and pointers that were themselves read
// from memory are not left as flat pointers.  The copy goes dword by dword
// (every table record is a whole number of dwords).
template <class T>
__device__ __forceinline__ T load_const(const T* base, int64_t index)
{
    static_assert(sizeof(T) % 4 == 0, "table records are whole dwords");
    using CP = const __attribute__((address_space(4))) int*;
    const CP p = (CP)(const void*)(base + index);
    T out;
    int* o = reinterpret_cast<int*>(&out);
#pragma unroll
    for (int i = 0; i < int(sizeof(T) / 4); ++i)
        o[i] = p[i];
    return out;
}

// RF records and images live in global memory; saying so keeps accesses
// through pointers read from a work list global rather than flat (flat loads
// also count against the LDS wait counter).
template <class T>
using Global = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ Global<T> global_ptr(T* p)
{
    return (Global<T>)p;
}

template <int DT> struct Storage;
template <> struct Storage<HODMAS_F32> { using T = float; };
template <> struct Storage<HODMAS_F16> { using T = _Float16; };
template <> struct Storage<HODMAS_I16> { using T = short; };

// Word 3 of a raw (stride 0) buffer resource on gfx950: 32-bit data format,
// no swizzle; with stride 0 an access is in range iff its byte offset is below
// the resource's size.
constexpr int kBufferFlags = 0x00020000;

__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(_Float16 v) { return (float)v; }
__device__ __forceinline__ float widen(short v) { return (float)v; }

// Kahan step: s + x with the running compensation c (true sum ~ s - c).
__device__ __forceinline__ void kahan_add(float& s, float& c, float x)
{
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Where one element's delayed sample sits in the LDS window for this lane's
// pixel: t = delay - floor(anchor delay), its fraction f and the LDS index.
// d^2 - d0^2 comes from one FMA on per-pixel terms; d - d0 = (d^2 - d0^2)/(d + d0).
struct Tap {
    float t, f;
    int addr;    // LDS byte address of the sample before the delay
};

__device__ __forceinline__ Tap locate_at(const hodmas_chan_entry& e, float u2, float q, int off)
{
    Tap p;
    const float num = __builtin_fmaf(u2, e.a, q);
    const float d = __builtin_amdgcn_sqrtf(__builtin_fabsf(e.d0sq + num));
    const float r = __builtin_amdgcn_rcpf(d + e.d0);
    p.t = __builtin_fmaf(num, r, e.frac0);
    // floor(t) as an integer in one instruction (the compiler emits a floor and
    // a conversion), and t - floor(t), which is exact in float32, so fract
    // returns it unchanged
    int fl;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(fl) : "v"(p.t));
    p.f = __builtin_amdgcn_fractf(p.t);
    p.addr = (fl << 2) + off;
    return p;
}

__device__ __forceinline__ Tap locate(const hodmas_chan_entry& e, float u2, float q)
{
    return locate_at(e, u2, q, e.off);
}

// Delays shared along translated pixels.  When the element pitch of a uniform
// linear array is SH pixel columns, the pixel in column x sees element i + 1
// at exactly the delay at which the pixel in column x - SH sees element i
// (Eq. 1 depends on the pixel's x minus the element's x only).  The 16 lanes
// of a tile row are 16 neighbouring columns, so for elements i + s, s = 1..3,
// a lane takes element i's delay from the lane s*SH columns to its left -- or,
// in the row's first s*SH lanes, from F: element i + 3's delay at the pixel
// 16 - 3*SH columns to the left, which is also element i + 4's at the lane's
// own pixel (the next group's first element).  A group of four elements then
// computes one delay per lane instead of four, and passes the others between
// the lanes of a row through 32 entries of an LDS buffer: F in entries [0, 16),
// element i's own delays in [16, 32), so element i + s of lane j is entry
// 16 + j - s*SH.  The shared quantities are 4 floor(delay) as an absolute
// sample index and the fraction; each element adds the byte offset that its
// LDS row gives sample 0.
// Rows' buffers are 48 entries apart: a 64-bit LDS access serves 32 lanes --
// two rows -- at once, and 16 entries of one row fill half the banks, so the
// neighbouring row's entries start half the banks (128 bytes) further on.
constexpr int kRowEntries = 48;

struct alignas(8) XF {     // one 64-bit LDS access per entry
    int x;      // 4 floor(delay), absolute sample index
    float f;    // fraction of the delay
};

struct Shared {
    int x;      // the group's first element at the lane's pixel
    float f;
    int fx;     // F: the next group's first element at the lane's pixel
    float ff;
    XF* buf;    // the lane's entry j of its row's buffer
};

// Orders the LDS accesses of one wave that exchange data between its lanes:
// a wave's LDS instructions complete in issue order, so keeping the compiler
// from moving them across this point is all that is needed.
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Byte offset of sample 0 in the LDS rows of four consecutive staged slots
// (slot, ..., slot + 3 of the chunk whose staging entries start at S): the
// sample at absolute index j of slot m sits at 4 j + ro[m].
__device__ __forceinline__ void load_rowoff(ConstStage S, int slot, int stride, int (&ro)[4])
{
#pragma unroll
    for (int m = 0; m < 4; ++m)
        ro[m] = 4 * ((slot + m) * stride - load_const(S, slot + m).first_sample);
}

// Tiles whose delays may leave the record (CHECK): a delay outside [lo, hi]
// -- before the first sample or past the last -- contributes nothing, so its
// address is pointed at a pair of zeros the staging keeps after the rows
// (`zero`, bytes) and the interpolation yields exactly 0.
__device__ __forceinline__ void redirect(Tap& p, const hodmas_chan_entry& e, int zero)
{
    p.addr = (p.t >= e.lo && p.t <= e.hi) ? p.addr : zero;
}

__device__ __forceinline__ float lds_at(const float* __restrict__ lds, int addr)
{
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(lds) + addr);
}

// Linear interpolation between the two staged samples.  HALF: the LDS words
// hold FP16 samples in their low halves (rows copied straight from an FP16
// record); the mixed-precision FMA widens them, exactly, as it interpolates,
// in the same two instructions.
template <bool HALF = false>
__device__ __forceinline__ float interp(const Tap& p, float s0, float s1)
{
    if constexpr (HALF) {
        const float h0 = (float)__builtin_bit_cast(_Float16, (unsigned short)__builtin_bit_cast(unsigned, s0));
        const float h1 = (float)__builtin_bit_cast(_Float16, (unsigned short)__builtin_bit_cast(unsigned, s1));
        return __builtin_fmaf(p.f, h1, __builtin_fmaf(-p.f, h0, h0));
    } else {
        return __builtin_fmaf(p.f, s1 - s0, s0);
    }
}

// y^1 .. y^K of the signed K-th root of v.
template <int K>
__device__ __forceinline__ void powers(float v, float (&T)[K])
{
    const float a = __builtin_fabsf(v);
    if constexpr (K == 1) {
        T[0] = v;
    } else if constexpr (K == 2) {
        float r = __builtin_amdgcn_sqrtf(a);
        T[0] = __builtin_copysignf(r, v);
        T[1] = a;
    } else if constexpr (K == 4) {
        float r2 = __builtin_amdgcn_sqrtf(a);
        float r = __builtin_amdgcn_sqrtf(r2);
        T[0] = __builtin_copysignf(r, v);
        T[1] = r2;
        T[2] = T[0] * r2;
        T[3] = a;
    } else {
        // |v|^(1/K) = 2^(log2|v| / K); v = 0 gives 2^-inf = 0
        float r = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(a) * (1.0f / K));
        float r2 = r * r;
        T[0] = __builtin_copysignf(r, v);
        T[1] = r2;
        T[2] = T[0] * r2;
        if constexpr (K == 3) {
            T[2] = v;
        } else {
            T[3] = r2 * r2;
            if constexpr (K == 5) {
                T[4] = v;
            } else {
                T[4] = T[2] * r2;
                T[5] = a;
            }
        }
    }
}

// The sums one element feeds: y^1 .. y^K, then -- with coherence-factor
// weighting -- the sample itself and its square.
template <int K, bool CF>
constexpr int n_sums() { return K + (CF ? 2 : 0); }

template <int K, bool CF>
__device__ __forceinline__ void terms(float v, float (&T)[n_sums<K, CF>()])
{
    float Y[K];
    powers<K>(v, Y);
#pragma unroll
    for (int j = 0; j < K; ++j)
        T[j] = Y[j];
    if constexpr (CF) {
        T[K] = v;
        T[K + 1] = v * v;
    }
}

// LDS layout of a staged chunk: rows of window + 2 floats.  Rows [0, nch) hold
// the chunk's slots (row r: slot r's element over its sample window), and the
// two floats after row 0's window are zeros, the target of out-of-record
// delays.  With M == 2 (mirror pairing) rows [nch, 2 nch) hold the mirrored
// elements, n_elements - 1 - element, over the same sample windows: the mirror
// pixel reads them at the same delays, mirror_offset bytes on -- which also
// takes the zeros' address to the same two floats of row nch.
__device__ __forceinline__ int row_stride(int window) { return window + 2; }
__device__ __forceinline__ int zero_offset(int window) { return window * 4; }
__device__ __forceinline__ int mirror_offset(int nch, int window) { return nch * row_stride(window) * 4; }

template <int DT, int M>
__device__ __forceinline__ void stage_chunk(const FrameArgs& A, ConstStage st, int nch, int window,
                                            float* __restrict__ lds, int wave, int nwaves, int lane)
{
    using T = typename Storage<DT>::T;
    constexpr int esz = int(sizeof(T));
    // Each wave stages a contiguous run of rows; lanes run along the window.
    // Latency, not bandwidth, sets the cost here: one vector load brings 64
    // rows' table entries (lane j holds row j), then the sample loads go out
    // kInFlight at a time before any wait.  Each row is read through a buffer
    // resource spanning exactly its channel's record, built in scalar
    // registers from the entry lanes: a sample index outside [0, S) -- before
    // the record, past its end, or negative -- is out of the resource's range
    // and loads as zero in hardware, so no lane clamps or selects.
    constexpr int kInFlight = 16;
    const int rows = M * nch;
    const int per_wave = (rows + nwaves - 1) / nwaves;
    const int s0 = wave * per_wave;
    const int s1 = min(rows, s0 + per_wave);
    const Global<const int> ent = global_ptr(reinterpret_cast<const int*>(st));
    const char* rf = static_cast<const char*>(A.rf);
    const int64_t row_bytes = int64_t(A.stride) * esz;
    const int record_bytes = A.n_samples * esz;
    const int stride = row_stride(window);
    if (wave == 0 && lane < 2 * M)
        lds[(lane >> 1) * nch * stride + window + (lane & 1)] = 0.f;
    for (int c = s0; c < s1; c += 64) {
        const int j = min(c + lane, s1 - 1);
        const bool mirrored = M == 2 && j >= nch;
        const int src = mirrored ? j - nch : j;
        const int elem = ent[2 * src];
        const int my_channel = mirrored ? A.n_elements - 1 - elem : elem;
        const int my_first = ent[2 * src + 1];
        const int cend = min(s1 - c, 64);
        for (int base = 0; base < window; base += 64) {
            const int i = base + lane;
            for (int m0 = 0; m0 < cend; m0 += kInFlight) {
                float v[kInFlight];
#pragma unroll
                for (int m = 0; m < kInFlight; ++m) {
                    const int ch = __builtin_amdgcn_readlane(my_channel, m0 + m);
                    const int first = __builtin_amdgcn_readlane(my_first, m0 + m);
                    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                        const_cast<char*>(rf + ch * row_bytes), (short)0, record_bytes, kBufferFlags);
                    const int off = (first + i) * esz;
                    if constexpr (DT == HODMAS_F32)
                        v[m] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
                    else if constexpr (DT == HODMAS_F16)
                        v[m] = (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0));
                    else
                        v[m] = (float)(short)__builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
                }
#pragma unroll
                for (int m = 0; m < kInFlight; ++m) {
                    const int row = c + m0 + m;
                    if (m0 + m < cend && i < window)
                        lds[row * stride + i] = v[m] * A.in_scale;
                }
            }
        }
    }
}

// FP32 and FP16 tiles whose rows lie inside the record (the plan marks the
// others as tested) copy each row from memory straight into LDS: buffer loads
// that write LDS, one per 64 samples, through one buffer resource over the
// whole frame, with the row's start in the scalar offset.  One vector pass
// forms 64 rows' offsets (lane j: row j), so a row then costs one lane read,
// scalar work and one load per wave -- no vector registers in flight, no
// conversion and no LDS store, where the general staging above spends several
// vector instructions per row.  An FP16 sample lands, zero-extended, in the
// low half of its LDS word (the layout of FP32 rows); the interpolation
// widens it.
template <int DT, int M>
__device__ __forceinline__ void stage_direct(const FrameArgs& A, ConstStage st, int nch, int window,
                                             float* __restrict__ lds, int wave, int nwaves, int lane)
{
    static_assert(DT == HODMAS_F32 || DT == HODMAS_F16, "direct copies move 4- or 2-byte samples");
    constexpr int esz = DT == HODMAS_F32 ? 4 : 2;
    using LdsPtr = __attribute__((address_space(3))) void*;
    const int rows = M * nch;
    const int per_wave = (rows + nwaves - 1) / nwaves;
    const int s0 = wave * per_wave;
    const int s1 = min(rows, s0 + per_wave);
    const int stride = row_stride(window);
    if (wave == 0 && lane < 2 * M)
        lds[(lane >> 1) * nch * stride + window + (lane & 1)] = 0.f;
    const int bytes = A.n_elements * (int)A.stride * esz;   // below 2^31: the plan tests every tile otherwise
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(A.rf), (short)0, bytes, kBufferFlags);
    const Global<const int> ent = global_ptr(reinterpret_cast<const int*>(st));
    for (int c = s0; c < s1; c += 64) {
        const int j = min(c + lane, s1 - 1);
        const bool mirrored = M == 2 && j >= nch;
        const int src = mirrored ? j - nch : j;
        const int elem = ent[2 * src];
        const int ch = mirrored ? A.n_elements - 1 - elem : elem;
        const int my_off = (ch * (int)A.stride + ent[2 * src + 1]) * esz;
        const int cend = __builtin_amdgcn_readfirstlane(min(s1 - c, 64));
        for (int b = 0; b < window; b += 64) {
            if (b + lane < window) {
                for (int m = 0; m < cend; ++m) {
                    const int soff = __builtin_amdgcn_readlane(my_off, m);
                    if constexpr (DT == HODMAS_F32)
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (LdsPtr)(lds + (c + m) * stride + b), 4,
                                                                 (b + lane) * 4, soff, 0, 0);
                    else
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (LdsPtr)(lds + (c + m) * stride + b), 2,
                                                                 (b + lane) * 2, soff, 0, 0);
                }
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);   // the copies are in LDS before the caller's barrier
}

// Workgroups are dealt to the eight XCDs round-robin (workgroup b runs on XCD
// b mod 8).  Give each XCD a contiguous run of tiles -- a band of tile rows --
// so the RF samples an XCD stages come from a narrow range of delays and its
// own L2 holds them, instead of every XCD fetching the whole frame.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n / kXcds, r = n % kXcds;
    const int x = b % kXcds, l = b / kXcds;
    return x * q + min(x, r) + l;
}

// Power-sum accumulation.  Compensated mode: four elements are summed pairwise,
// eight such groups (32 elements) accumulate in a plain float32 partial, and the
// partial enters the running sum with one Kahan step.  The rounding error then
// stays at a few units of the partials' magnitude instead of growing with N.
template <int K>
__device__ __forceinline__ void flush(float (&s)[K], float (&c)[K], float (&P)[K])
{
#pragma unroll
    for (int j = 0; j < K; ++j) {
        kahan_add(s[j], c[j], P[j]);
        P[j] = 0.f;
    }
}

__device__ __forceinline__ void load_group(ConstEntry E, hodmas_chan_entry (&e)[4])
{
#pragma unroll
    for (int m = 0; m < 4; ++m)
        e[m] = load_const(E, m);
}

// One group of four elements: delays and LDS addresses, the four gathers
// issued together, the interpolations, then -- once this group's LDS data is
// in -- the scalar loads of the next group's constants (the LDS/scalar wait
// counter does not order scalar loads, so issuing them earlier would make
// this group's waits also wait for them), then roots, powers and the sums.
// With M == 2 each delay also serves the lane's mirror pixel, whose samples
// sit `moff` bytes further on in the LDS (the mirrored rows).  `zero`: the
// LDS byte address of the zero pair (CHECK).  SH > 0: delays shared along
// translated pixels (see Shared): `sh` holds the group's first element's delay
// on entry and the next group's on return; (u2f, qf) are the lane's pixel
// moved 16 - 3*SH columns to the left; ro / ron: the LDS row offsets of this
// group's slots and, loaded with the next group's constants, of the next.
template <int K, bool CF, bool COMP, bool CHECK, bool HALF, int M, int SH, int NS = n_sums<K, CF>()>
__device__ __forceinline__ void process_group(const hodmas_chan_entry (&e)[4], float u2, float q,
                                              const float* __restrict__ lds, int moff, int zero, float (&s)[M][NS],
                                              float (&P)[M][NS], bool more, ConstEntry En,
                                              hodmas_chan_entry (&en)[4], Shared& sh, float u2f, float qf,
                                              const int (&ro)[4], ConstStage Sn, int slot_n, int stride,
                                              int (&ron)[4])
{
    Tap tp[4];
    float s0[M][4], s1[M][4], v[M][4];
    if constexpr (SH > 0) {
        static_assert(!CHECK && M == 1, "shared delays: untested tiles, one pixel per lane");
        static_assert(4 * SH == 16, "a group of four elements spans one row of 16 lanes");
        // the buffer holds this group's F and first element (written at the
        // end of the previous group, or before the first)
        const XF* b = sh.buf;
        wave_lds_order();
        const XF d1 = b[16 - SH], d2 = b[16 - 2 * SH], d3 = b[16 - 3 * SH];
        tp[0] = Tap{0.f, sh.f, sh.x + ro[0]};
        tp[1] = Tap{0.f, d1.f, d1.x + ro[1]};
        tp[2] = Tap{0.f, d2.f, d2.x + ro[2]};
        tp[3] = Tap{0.f, d3.f, d3.x + ro[3]};
    } else {
#pragma unroll
        for (int m = 0; m < 4; ++m)
            tp[m] = locate(e[m], u2, q);
    }
    if (CHECK) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
            redirect(tp[m], e[m], zero);
    }
#pragma unroll
    for (int mm = 0; mm < M; ++mm) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            s0[mm][m] = lds_at(lds, tp[m].addr + mm * moff);
            s1[mm][m] = lds_at(lds, tp[m].addr + mm * moff + 4);
        }
    }
#pragma unroll
    for (int mm = 0; mm < M; ++mm) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
            v[mm][m] = interp<HALF>(tp[m], s0[mm][m], s1[mm][m]);
    }
    // emits nothing: makes the samples (hence this group's LDS waits)
    // complete before the scalar loads below are issued
#pragma unroll
    for (int mm = 0; mm < M; ++mm)
        asm volatile("" ::"v"(v[mm][0]), "v"(v[mm][1]), "v"(v[mm][2]), "v"(v[mm][3]) : "memory");
    if (more) {
        load_group(En, en);
        if constexpr (SH > 0)
            load_rowoff(Sn, slot_n, stride, ron);
    }
#pragma unroll
    for (int mm = 0; mm < M; ++mm) {
        float T[4][NS];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            terms<K, CF>(v[mm][m], T[m]);
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            if (COMP) {
                P[mm][j] += (T[0][j] + T[1][j]) + (T[2][j] + T[3][j]);
            } else {
                s[mm][j] += T[0][j];
                s[mm][j] += T[1][j];
                s[mm][j] += T[2][j];
                s[mm][j] += T[3][j];
            }
        }
    }
    if constexpr (SH > 0) {
        if (more) {
            // the next group's F -- its last element at the moved pixel --
            // formed here, after this group's arithmetic has been issued, so
            // its latency and that of the next group's constants overlap it;
            // written over this group's entries, whose reads came first
            const Tap tf = locate_at(en[3], u2f, qf, en[3].off - ron[3]);
            XF* b = sh.buf;
            wave_lds_order();
            b[0] = XF{tf.addr, tf.f};
            b[16] = XF{sh.fx, sh.ff};
            sh.x = sh.fx;
            sh.f = sh.ff;
            sh.fx = tf.addr;
            sh.ff = tf.f;
        }
    }
}

template <int NS, bool COMP, int M>
__device__ __forceinline__ void after_group(int& groups, float (&s)[M][NS], float (&c)[M][NS],
                                            float (&P)[M][NS])
{
    if (COMP && (++groups & 7) == 0) {
#pragma unroll
        for (int mm = 0; mm < M; ++mm)
            flush<NS>(s[mm], c[mm], P[mm]);
    }
}

// The n elements of this wave's split group in one staged chunk (their
// constants stored contiguously), four at a time; two constant sets alternate
// so nothing is copied between them.
template <int K, bool CF, bool COMP, bool CHECK, bool HALF, int M, int SH, int NS = n_sums<K, CF>()>
__device__ __forceinline__ void accumulate_chunk(ConstEntry E, int n, float u2, float q,
                                                 const float* __restrict__ lds, int moff, int zero, float (&s)[M][NS],
                                                 float (&c)[M][NS], ConstStage St, int stride, float u2f, float qf,
                                                 XF* shbuf)
{
    float P[M][NS];
#pragma unroll
    for (int mm = 0; mm < M; ++mm) {
#pragma unroll
        for (int j = 0; j < NS; ++j)
            P[mm][j] = 0.f;
    }
    int sl = 0;
    if (n >= 4) {
        hodmas_chan_entry ea[4], eb[4];
        int ra[4] = {0, 0, 0, 0}, rb[4] = {0, 0, 0, 0};
        Shared sh{0, 0.f, 0, 0.f, shbuf};
        load_group(E, ea);
        if constexpr (SH > 0) {
            // slots 0..3 of the chunk: the first element's delay computed in
            // full, and the first group's F
            load_rowoff(St, 0, stride, ra);
            const Tap t0 = locate_at(ea[0], u2, q, ea[0].off - ra[0]);
            const Tap tf = locate_at(ea[3], u2f, qf, ea[3].off - ra[3]);
            sh.x = t0.addr;
            sh.f = t0.f;
            sh.fx = tf.addr;
            sh.ff = tf.f;
            wave_lds_order();
            sh.buf[0] = XF{tf.addr, tf.f};
            sh.buf[16] = XF{t0.addr, t0.f};
        }
        int groups = 0;
        while (true) {
            const bool more_a = sl + 8 <= n;
            process_group<K, CF, COMP, CHECK, HALF, M, SH>(ea, u2, q, lds, moff, zero, s, P, more_a, E + sl + 4, eb,
                                                           sh, u2f, qf, ra, St, sl + 4, stride, rb);
            after_group<NS, COMP, M>(groups, s, c, P);
            sl += 4;
            if (!more_a)
                break;
            const bool more_b = sl + 8 <= n;
            process_group<K, CF, COMP, CHECK, HALF, M, SH>(eb, u2, q, lds, moff, zero, s, P, more_b, E + sl + 4, ea,
                                                           sh, u2f, qf, rb, St, sl + 4, stride, ra);
            after_group<NS, COMP, M>(groups, s, c, P);
            sl += 4;
            if (!more_b)
                break;
        }
    }
    for (; sl < n; ++sl) {
        const hodmas_chan_entry e = load_const(E, sl);
        Tap tp = locate(e, u2, q);
        if (CHECK)
            redirect(tp, e, zero);
#pragma unroll
        for (int mm = 0; mm < M; ++mm) {
            float T[NS];
            const int addr = tp.addr + mm * moff;
            terms<K, CF>(interp<HALF>(tp, lds_at(lds, addr), lds_at(lds, addr + 4)), T);
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                if (COMP)
                    P[mm][j] += T[j];
                else
                    s[mm][j] += T[j];
            }
        }
    }
    if (COMP) {
#pragma unroll
        for (int mm = 0; mm < M; ++mm)
            flush<NS>(s[mm], c[mm], P[mm]);
    }
}

// Newton's identities: e_m = (1/m) sum_{j=1..m} (-1)^(j-1) e_{m-j} p_j.
template <int K, typename R>
__device__ __forceinline__ R newton(const R (&p)[K])
{
    R e[K + 1];
    e[0] = R(1);
#pragma unroll
    for (int m = 1; m <= K; ++m) {
        R acc = R(0);
#pragma unroll
        for (int j = 1; j <= m; ++j) {
            R term = e[m - j] * p[j - 1];
            acc = (j & 1) ? acc + term : acc - term;
        }
        e[m] = acc * (R(1) / R(m));
    }
    return e[K];
}

// One pixel tile of one frame: stage, accumulate, combine, recover, store.
// Every thread of the workgroup calls this with the same (A, tile); all
// branches on tile data are workgroup-uniform, so the barriers inside match.
// With M == 2 the workgroup also forms the mirror tile: the pixel at column
// nx-1-ix of each lane's own pixel at ix.  When the array and the grid are
// symmetric about x = 0 (checked on the host), that pixel's delay to element
// n-1-i equals this pixel's delay to element i, so one delay serves both and
// the mirror pixel gathers from the mirrored rows the staging fills.
template <int K, int DT, bool COMP, bool CF, int M, bool CHECK, int SH = 0>
__device__ __forceinline__ void process_tile(const FrameArgs& A, const hodmas_tile_desc& td,
                                             float* __restrict__ lds)
{
    constexpr int NS = n_sums<K, CF>();
    // rows copied straight into LDS (FP32, FP16) unless the tile is range-tested
    constexpr bool kDirect = !CHECK && (DT == HODMAS_F32 || DT == HODMAS_F16);
    constexpr bool kHalf = kDirect && DT == HODMAS_F16;
    const int tid = threadIdx.x;
    const int npix = A.block / A.split;
    const int nwaves = A.block >> 6;
    const int g = __builtin_amdgcn_readfirstlane(tid / npix);   // npix is a multiple of 64
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int pl = tid - g * npix;
    const int lx = pl % A.tile_x, lz = pl / A.tile_x;
    const bool valid = lx < td.nx && lz < td.nz;
    const int ix = td.ix0 + min(lx, td.nx - 1);
    const int iz = td.iz0 + min(lz, td.nz - 1);
    // the lane's pixel (mm = 0) and, with M == 2, its mirror image; formed
    // where it is stored, so no 64-bit address stays live through the loops
    auto dst = [&](int mm) {
        return global_ptr(A.image + (int64_t)iz * A.nx + (mm == 0 ? ix : A.nx - 1 - ix));
    };

    if (td.n_active < K) {
        // fewer contributing elements than the order: no K-subset exists, e_K = 0 exactly
        if (g == 0 && valid) {
#pragma unroll
            for (int mm = 0; mm < M; ++mm)
                *dst(mm) = 0.f;
        }
        return;
    }

    // pixel offset from the anchor, in float64 once per pixel
    const double u = A.x0s + ix * A.dxs - td.xa;
    const double w = A.z0s + iz * A.dzs - td.za;
    const float u2 = (float)(2.0 * u);
    const float q = (float)(u * u + w * (w + 2.0 * td.za));
    // SH > 0: the same pixel moved 16 - 3*SH columns to the left (the plan
    // keeps every tile 16 columns wide, so no lane's column was clamped)
    float u2f = 0.f, qf = 0.f;
    XF* shbuf = nullptr;
    if constexpr (SH > 0) {
        const double uf = u + (3 * SH - 16) * A.dxs;
        u2f = (float)(2.0 * uf);
        qf = (float)(uf * uf + w * (w + 2.0 * td.za));
        // the row's buffer after the staged rows (pixel row pl / 16 of
        // the workgroup; no lane's column was clamped, see above)
        shbuf = reinterpret_cast<XF*>(reinterpret_cast<char*>(lds) + A.shift_off) + (pl >> 4) * kRowEntries + lx;
    }

    float s[M][NS], c[M][NS];
#pragma unroll
    for (int mm = 0; mm < M; ++mm) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            s[mm][j] = 0.f;
            c[mm][j] = 0.f;
        }
    }
    ConstEntry E = A.entries + td.first_entry;
    ConstStage St = A.stage + td.first_entry;
    for (int c0 = 0; c0 < td.n_active; c0 += A.chunk) {
        const int nch = min(A.chunk, td.n_active - c0);
        __syncthreads();                       // previous readers of the LDS are done
        if constexpr (kDirect)
            stage_direct<DT, M>(A, St + c0, nch, td.window, lds, wave, nwaves, lane);
        else
            stage_chunk<DT, M>(A, St + c0, nch, td.window, lds, wave, nwaves, lane);
        __syncthreads();
        const int moff = mirror_offset(nch, td.window);  // bytes from a slot's row to its mirrored row
        const int zero = zero_offset(td.window);
        // this group's elements of the chunk: slots g, g+split, ..., stored together
        int goff = 0;
        for (int h = 0; h < g; ++h)
            goff += (nch - h + A.split - 1) / A.split;
        const int ng = nch > g ? (nch - g + A.split - 1) / A.split : 0;
        accumulate_chunk<K, CF, COMP, CHECK, kHalf, M, SH>(E + c0 + goff, ng, u2, q, lds, moff, zero, s, c, St + c0,
                                                            row_stride(td.window), u2f, qf, shbuf);
    }

    if (A.split > 1) {
        // fixed-order combination of the groups' partial sums through LDS
        // floats per pixel and group: (sum, compensation) pairs, padded to an
        // odd stride so consecutive lanes fall in different LDS banks
        constexpr int W = 2 * M * NS + 1;
        __syncthreads();
        float* red = lds;
        if (g > 0) {
#pragma unroll
            for (int mm = 0; mm < M; ++mm) {
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    red[((g - 1) * npix + pl) * W + 2 * (mm * NS + j)] = s[mm][j];
                    red[((g - 1) * npix + pl) * W + 2 * (mm * NS + j) + 1] = c[mm][j];
                }
            }
        }
        __syncthreads();
        if (g == 0) {
            for (int gg = 1; gg < A.split; ++gg) {
#pragma unroll
                for (int mm = 0; mm < M; ++mm) {
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        const float so = red[((gg - 1) * npix + pl) * W + 2 * (mm * NS + j)];
                        const float co = red[((gg - 1) * npix + pl) * W + 2 * (mm * NS + j) + 1];
                        if (COMP) {
                            kahan_add(s[mm][j], c[mm][j], so);
                            kahan_add(s[mm][j], c[mm][j], -co);
                        } else {
                            s[mm][j] += so;
                        }
                    }
                }
            }
        }
    }
    if (g != 0 || !valid)
        return;
    using R = typename std::conditional<(K >= 5), double, float>::type;
#pragma unroll
    for (int mm = 0; mm < M; ++mm) {
        R p[K];
#pragma unroll
        for (int j = 0; j < K; ++j)
            p[j] = COMP ? R(s[mm][j]) - R(c[mm][j]) : R(s[mm][j]);
        const R ek = newton<K, R>(p);
        if constexpr (CF) {
            // coherence factor (sum v)^2 / (N sum v^2) of the normalised samples
            const double s1 = COMP ? double(s[mm][K]) - double(c[mm][K]) : double(s[mm][K]);
            const double s2 = COMP ? double(s[mm][K + 1]) - double(c[mm][K + 1]) : double(s[mm][K + 1]);
            const double cf = s2 > 0.0 ? (s1 * s1) / (double(A.n_elements) * s2) : 0.0;
            *dst(mm) = (float)(double(ek) * cf * double(A.out_scale));
        } else {
            *dst(mm) = (float)(ek * R(A.out_scale));
        }
    }
}

// Tiles that reach the record ends take the body with the range test, the
// others the body without it.  The choice is made once per tile, so each body
// is a whole of its own: with the test inside the element loop, or with both
// loop variants in one body, the paired kernels' sums no longer fit their
// registers and the loop's scheduling suffers.
template <int K, int DT, bool COMP, bool CF = false, int M = 1>
__device__ __forceinline__ void form_tile(const FrameArgs& A, int tile, float* __restrict__ lds)
{
    const hodmas_tile_desc td = load_const(A.tiles, tile);
    if (td.check) {
        process_tile<K, DT, COMP, CF, M, true>(A, td, lds);
    } else {
        if constexpr (M == 1 && !CF && K >= 2) {
            if (A.shift == 4 && td.iz0 >= A.shift_iz0) {
                process_tile<K, DT, COMP, CF, M, false, 4>(A, td, lds);
                return;
            }
        }
        process_tile<K, DT, COMP, CF, M, false>(A, td, lds);
    }
}

// M == 1: workgroup b forms tile xcd_tile(b).  M == 2: workgroup b forms pair
// p = xcd_tile(b) of the n_tiles / 2 pairs -- the p-th tile of the grid's
// left half (row-major over its tile rows) and that tile's mirror image.
template <int K, int DT, bool COMP, bool CF, int M>
__global__ __launch_bounds__(kMaxBlock) void hodmas_frame_kernel(FrameArgs A)
{
    extern __shared__ float lds[];
    if constexpr (M == 1) {
        form_tile<K, DT, COMP, CF, 1>(A, xcd_tile(blockIdx.x, A.n_tiles), lds);
    } else {
        const int half = A.nx / A.tile_x / 2;     // tile columns left of the centre
        const int p = xcd_tile(blockIdx.x, A.n_tiles / 2);
        const int bz = p / half;
        form_tile<K, DT, COMP, CF, 2>(A, bz * 2 * half + (p - bz * half), lds);
    }
}

// Persistent form: one kernel per (order, storage type, pairing, coherence
// weighting).  Its fixed grid walks that kind's slice of the batch's work
// list -- (frame, tile) units of many frames with their own plans.  The slice
// is cut into one run per XCD (neighbouring tiles of one or a few frames, of
// about equal estimated cost, each sorted by cost); the g workgroups on XCD x
// (workgroups x, x+8, ...) walk run x, the l-th of them taking units l,
// 2g-1-l, 2g+l, ... (a snake, which evens out the per-workgroup cost).  With
// M == 2 a unit is a mirror pair, named by its left tile.  Each unit runs
// exactly the code of the per-frame kernel, so a frame's image does not depend
// on what else is in the batch.
// Mirror pairs keep two pixels' sums per lane.  At order 6 that takes a paired
// kernel a little above 80 VGPRs (five waves per SIMD), while a 64-element
// chunk's LDS leaves room for six workgroups per CU; asking for six waves
// costs a few dwords of spill per tile (values kept for the final store), none
// in the loops.  Lower orders fit six or seven waves without asking; with
// coherence weighting (two more sums per pixel) six waves would spill inside
// the loops, so those kernels are left at the four or five they fit.
constexpr int batch_min_waves(int K, int M, bool CF) { return M == 2 && K == 6 && !CF ? 6 : 1; }

template <int K, int DT, bool COMP, bool CF, int M>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(batch_min_waves(K, M, CF))))
void hodmas_batch_kernel(const BatchHeader* __restrict__ hdr, const BatchFrame* __restrict__ frames,
                         const BatchUnit* __restrict__ units)
{
    extern __shared__ float lds[];
    constexpr int kind = batch_kind(K, DT, M, CF ? 1 : 0);
    const int x = (int)blockIdx.x % kXcds, l = (int)blockIdx.x / kXcds;
    const int g = ((int)gridDim.x - x + kXcds - 1) / kXcds;   // workgroups on this XCD
    const int lo = load_const(&hdr->xcd[kind][0], x);
    const int first = load_const(&hdr->begin[0], kind) + lo;
    const int n = load_const(&hdr->xcd[kind][0], x + 1) - lo;
    for (int r = 0; r * g < n; ++r) {
        const int u = (r & 1) ? (r + 1) * g - 1 - l : r * g + l;
        if (u >= n)
            continue;
        const BatchUnit un = load_const(units, first + u);
        const BatchFrame fr = load_const(frames, un.frame);
        form_tile<K, DT, COMP, CF, M>(fr.args, un.tile, lds);
    }
}

// ---------------------------------------------------------------------------
// Every order 1..KMAX in one pass.  The delay, gather and interpolation are
// the same for all orders; the roots share their transcendentals
// (|v|^(1/4) = sqrt(|v|^(1/2)), |v|^(1/6) = sqrt(|v|^(1/3)), one log2 serves
// the cube and fifth roots); and many power sums coincide across orders,
// since y_k^j = sign(v)^j |v|^(j/k) depends only on j/k and the parity of j:
// orders 1..6 need 15 distinct sums instead of 21.
//
//   sum   exponent  signed   used as p_j of order k
//    0      1        yes     k1 p1, k3 p3, k5 p5
//    1      1        no      k2 p2, k4 p4, k6 p6
//    2      1/2      yes     k2 p1, k6 p3
//    3      1/2      no      k4 p2
//    4      1/3      yes     k3 p1
//    5      1/3      no      k6 p2
//    6      2/3      no      k3 p2, k6 p4
//    7      1/4      yes     k4 p1
//    8      3/4      yes     k4 p3
//    9..12  j/5      j odd   k5 p1..p4
//   13      1/6      yes     k6 p1
//   14      5/6      yes     k6 p5
constexpr int kSums = kOrderSums;
constexpr int kSumOf[HODMAS_MAX_ORDER + 1][HODMAS_MAX_ORDER] = {
    {0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0},
    {2, 1, 0, 0, 0, 0},
    {4, 6, 0, 0, 0, 0},
    {7, 3, 8, 1, 0, 0},
    {9, 10, 11, 12, 0, 0},
    {13, 5, 2, 6, 14, 1},
};

// Is sum i needed by some order <= KMAX?
constexpr bool sum_needed(int i, int kmax)
{
    for (int k = 1; k <= kmax; ++k)
        for (int j = 0; j < k; ++j)
            if (kSumOf[k][j] == i)
                return true;
    return false;
}

template <int KMAX>
__device__ __forceinline__ void terms_all(float v, float (&T)[kSums])
{
    const float a = __builtin_fabsf(v);
    T[0] = v;
    T[1] = a;
    if constexpr (KMAX >= 2) {
        const float r2 = __builtin_amdgcn_sqrtf(a);
        T[2] = __builtin_copysignf(r2, v);
        T[3] = r2;
        if constexpr (KMAX >= 3) {
            const float L = __builtin_amdgcn_logf(a);
            const float r3 = __builtin_amdgcn_exp2f(L * (1.0f / 3));
            T[4] = __builtin_copysignf(r3, v);
            T[5] = r3;
            T[6] = r3 * r3;
            if constexpr (KMAX >= 4) {
                const float y4 = __builtin_copysignf(__builtin_amdgcn_sqrtf(r2), v);
                T[7] = y4;
                T[8] = y4 * r2;
                if constexpr (KMAX >= 5) {
                    const float r5 = __builtin_amdgcn_exp2f(L * 0.2f);
                    const float y5 = __builtin_copysignf(r5, v);
                    const float q5 = r5 * r5;
                    T[9] = y5;
                    T[10] = q5;
                    T[11] = y5 * q5;
                    T[12] = q5 * q5;
                    if constexpr (KMAX >= 6) {
                        const float y6 = __builtin_copysignf(__builtin_amdgcn_sqrtf(r3), v);
                        T[13] = y6;
                        T[14] = y6 * T[6];
                    }
                }
            }
        }
    }
}

template <int KMAX, bool COMP, bool CHECK, bool HALF>
__device__ __forceinline__ void process_group_all(const hodmas_chan_entry (&e)[4], float u2, float q,
                                                  const float* __restrict__ lds, int zero, float (&s)[kSums],
                                                  float (&P)[kSums], bool more, ConstEntry En,
                                                  hodmas_chan_entry (&en)[4])
{
    Tap tp[4];
    float s0[4], s1[4], v[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
        tp[m] = locate(e[m], u2, q);
    if (CHECK) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
            redirect(tp[m], e[m], zero);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        s0[m] = lds_at(lds, tp[m].addr);
        s1[m] = lds_at(lds, tp[m].addr + 4);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
        v[m] = interp<HALF>(tp[m], s0[m], s1[m]);
    asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]) : "memory");
    if (more)
        load_group(En, en);
    // two elements at a time keep the live term count at 2 * kSums
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        float Ta[kSums], Tb[kSums];
        terms_all<KMAX>(v[2 * h], Ta);
        terms_all<KMAX>(v[2 * h + 1], Tb);
#pragma unroll
        for (int j = 0; j < kSums; ++j) {
            if (!sum_needed(j, KMAX))
                continue;
            if (COMP) {
                P[j] += Ta[j] + Tb[j];
            } else {
                s[j] += Ta[j];
                s[j] += Tb[j];
            }
        }
    }
}

template <int KMAX, bool COMP>
__device__ __forceinline__ void flush_all(float (&s)[kSums], float (&c)[kSums], float (&P)[kSums])
{
#pragma unroll
    for (int j = 0; j < kSums; ++j) {
        if (!sum_needed(j, KMAX))
            continue;
        kahan_add(s[j], c[j], P[j]);
        P[j] = 0.f;
    }
}

template <int KMAX, bool COMP, bool CHECK, bool HALF>
__device__ __forceinline__ void accumulate_chunk_all(ConstEntry E, int n, float u2, float q,
                                                     const float* __restrict__ lds, int zero, float (&s)[kSums],
                                                     float (&c)[kSums])
{
    float P[kSums];
#pragma unroll
    for (int j = 0; j < kSums; ++j)
        P[j] = 0.f;
    int sl = 0;
    if (n >= 4) {
        hodmas_chan_entry ea[4], eb[4];
        load_group(E, ea);
        int groups = 0;
        while (true) {
            const bool more_a = sl + 8 <= n;
            process_group_all<KMAX, COMP, CHECK, HALF>(ea, u2, q, lds, zero, s, P, more_a, E + sl + 4, eb);
            if (COMP && (++groups & 7) == 0)
                flush_all<KMAX, COMP>(s, c, P);
            sl += 4;
            if (!more_a)
                break;
            const bool more_b = sl + 8 <= n;
            process_group_all<KMAX, COMP, CHECK, HALF>(eb, u2, q, lds, zero, s, P, more_b, E + sl + 4, ea);
            if (COMP && (++groups & 7) == 0)
                flush_all<KMAX, COMP>(s, c, P);
            sl += 4;
            if (!more_b)
                break;
        }
    }
    for (; sl < n; ++sl) {
        const hodmas_chan_entry e = load_const(E, sl);
        Tap tp = locate(e, u2, q);
        if (CHECK)
            redirect(tp, e, zero);
        float T[kSums];
        terms_all<KMAX>(interp<HALF>(tp, lds_at(lds, tp.addr), lds_at(lds, tp.addr + 4)), T);
#pragma unroll
        for (int j = 0; j < kSums; ++j) {
            if (!sum_needed(j, KMAX))
                continue;
            if (COMP)
                P[j] += T[j];
            else
                s[j] += T[j];
        }
    }
    if (COMP)
        flush_all<KMAX, COMP>(s, c, P);
}

template <int K, bool COMP>
__device__ __forceinline__ void store_order(const float (&s)[kSums], const float (&c)[kSums], float out_scale,
                                            float* __restrict__ dst)
{
    using R = typename std::conditional<(K >= 5), double, float>::type;
    R p[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
        p[j] = COMP ? R(s[kSumOf[K][j]]) - R(c[kSumOf[K][j]]) : R(s[kSumOf[K][j]]);
    *dst = (float)(newton<K, R>(p) * R(out_scale));
}

template <int KMAX, int DT, bool COMP, bool CHECK>
__device__ __forceinline__ void orders_tile(const FrameArgs& A, const OrderImages& out, const hodmas_tile_desc& td,
                                            float* __restrict__ lds)
{
    constexpr int NT = kSums;
    constexpr bool kDirect = !CHECK && (DT == HODMAS_F32 || DT == HODMAS_F16);
    constexpr bool kHalf = kDirect && DT == HODMAS_F16;
    const int tid = threadIdx.x;
    const int npix = A.block / A.split;
    const int nwaves = A.block >> 6;
    const int g = __builtin_amdgcn_readfirstlane(tid / npix);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int pl = tid - g * npix;
    const int lx = pl % A.tile_x, lz = pl / A.tile_x;
    const bool valid = lx < td.nx && lz < td.nz;
    const int ix = td.ix0 + min(lx, td.nx - 1);
    const int iz = td.iz0 + min(lz, td.nz - 1);
    const int64_t pix = (int64_t)iz * A.nx + ix;

    const double u = A.x0s + ix * A.dxs - td.xa;
    const double w = A.z0s + iz * A.dzs - td.za;
    const float u2 = (float)(2.0 * u);
    const float q = (float)(u * u + w * (w + 2.0 * td.za));

    float s[NT], c[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        // unneeded sums stay zero and are never read
        s[j] = 0.f;
        c[j] = 0.f;
    }
    ConstEntry E = A.entries + td.first_entry;
    ConstStage St = A.stage + td.first_entry;
    for (int c0 = 0; c0 < td.n_active; c0 += A.chunk) {
        const int nch = min(A.chunk, td.n_active - c0);
        __syncthreads();
        if constexpr (kDirect)
            stage_direct<DT, 1>(A, St + c0, nch, td.window, lds, wave, nwaves, lane);
        else
            stage_chunk<DT, 1>(A, St + c0, nch, td.window, lds, wave, nwaves, lane);
        __syncthreads();
        int goff = 0;
        for (int h = 0; h < g; ++h)
            goff += (nch - h + A.split - 1) / A.split;
        const int ng = nch > g ? (nch - g + A.split - 1) / A.split : 0;
        accumulate_chunk_all<KMAX, COMP, CHECK, kHalf>(E + c0 + goff, ng, u2, q, lds, zero_offset(td.window), s, c);
    }
    if (A.split > 1) {
        __syncthreads();
        float* red = lds;
        if (g > 0) {
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                if (!sum_needed(j, KMAX))
                    continue;
                red[((g - 1) * npix + pl) * (2 * NT + 1) + 2 * j] = s[j];
                red[((g - 1) * npix + pl) * (2 * NT + 1) + 2 * j + 1] = c[j];
            }
        }
        __syncthreads();
        if (g == 0) {
            for (int gg = 1; gg < A.split; ++gg) {
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    if (!sum_needed(j, KMAX))
                        continue;
                    const float so = red[((gg - 1) * npix + pl) * (2 * NT + 1) + 2 * j];
                    const float co = red[((gg - 1) * npix + pl) * (2 * NT + 1) + 2 * j + 1];
                    if (COMP) {
                        kahan_add(s[j], c[j], so);
                        kahan_add(s[j], c[j], -co);
                    } else {
                        s[j] += so;
                    }
                }
            }
        }
    }
    if (g != 0 || !valid)
        return;
    // orders with fewer contributing elements than k are exactly 0
    const int na = td.n_active;
    if (na >= 1) store_order<1, COMP>(s, c, A.out_scale, out.img[0] + pix); else out.img[0][pix] = 0.f;
    if constexpr (KMAX >= 2) { if (na >= 2) store_order<2, COMP>(s, c, A.out_scale, out.img[1] + pix); else out.img[1][pix] = 0.f; }
    if constexpr (KMAX >= 3) { if (na >= 3) store_order<3, COMP>(s, c, A.out_scale, out.img[2] + pix); else out.img[2][pix] = 0.f; }
    if constexpr (KMAX >= 4) { if (na >= 4) store_order<4, COMP>(s, c, A.out_scale, out.img[3] + pix); else out.img[3][pix] = 0.f; }
    if constexpr (KMAX >= 5) { if (na >= 5) store_order<5, COMP>(s, c, A.out_scale, out.img[4] + pix); else out.img[4][pix] = 0.f; }
    if constexpr (KMAX >= 6) { if (na >= 6) store_order<6, COMP>(s, c, A.out_scale, out.img[5] + pix); else out.img[5][pix] = 0.f; }
}

template <int KMAX, int DT, bool COMP>
__global__ __launch_bounds__(kMaxBlock) void hodmas_orders_kernel(FrameArgs A, OrderImages out)
{
    extern __shared__ float lds[];
    const hodmas_tile_desc td = load_const(A.tiles, xcd_tile(blockIdx.x, A.n_tiles));
    if (td.check)
        orders_tile<KMAX, DT, COMP, true>(A, out, td, lds);
    else
        orders_tile<KMAX, DT, COMP, false>(A, out, td, lds);
}

template <int KMAX, int DT>
int launch_orders_k(const FrameArgs& a, const OrderImages& out, bool comp, int64_t lds_bytes, hipStream_t st)
{
    dim3 grid(a.n_tiles), block(a.block);
    if (comp)
        hipLaunchKernelGGL((hodmas_orders_kernel<KMAX, DT, true>), grid, block, (size_t)lds_bytes, st, a, out);
    else
        hipLaunchKernelGGL((hodmas_orders_kernel<KMAX, DT, false>), grid, block, (size_t)lds_bytes, st, a, out);
    return (int)hipGetLastError();
}

template <int DT>
int launch_orders_dt(const FrameArgs& a, const OrderImages& out, int kmax, bool comp, int64_t lds_bytes,
                     hipStream_t st)
{
    switch (kmax) {
    case 1: return launch_orders_k<1, DT>(a, out, comp, lds_bytes, st);
    case 2: return launch_orders_k<2, DT>(a, out, comp, lds_bytes, st);
    case 3: return launch_orders_k<3, DT>(a, out, comp, lds_bytes, st);
    case 4: return launch_orders_k<4, DT>(a, out, comp, lds_bytes, st);
    case 5: return launch_orders_k<5, DT>(a, out, comp, lds_bytes, st);
    case 6: return launch_orders_k<6, DT>(a, out, comp, lds_bytes, st);
    }
    return (int)hipErrorInvalidValue;
}

// A workgroup may hold more than 64 KB of LDS only once the kernel says so.
int launch_one(void (*fn)(FrameArgs), dim3 grid, dim3 block, int64_t lds_bytes, hipStream_t st,
               const FrameArgs& a)
{
    if (lds_bytes > 64 * 1024 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes) != hipSuccess)
        return (int)hipGetLastError();
    hipLaunchKernelGGL(fn, grid, block, (size_t)lds_bytes, st, a);
    return (int)hipGetLastError();
}

template <int K, int DT, int M>
int launch_km(const FrameArgs& a, bool comp, bool cf, int64_t lds_bytes, hipStream_t st)
{
    const dim3 grid(a.n_tiles / M), block(a.block);
    if (comp && cf)
        return launch_one(hodmas_frame_kernel<K, DT, true, true, M>, grid, block, lds_bytes, st, a);
    if (comp)
        return launch_one(hodmas_frame_kernel<K, DT, true, false, M>, grid, block, lds_bytes, st, a);
    if (cf)
        return launch_one(hodmas_frame_kernel<K, DT, false, true, M>, grid, block, lds_bytes, st, a);
    return launch_one(hodmas_frame_kernel<K, DT, false, false, M>, grid, block, lds_bytes, st, a);
}

template <int K, int DT>
int launch_k(const FrameArgs& a, bool comp, bool cf, bool mirror, int64_t lds_bytes, hipStream_t st)
{
    return mirror ? launch_km<K, DT, 2>(a, comp, cf, lds_bytes, st) : launch_km<K, DT, 1>(a, comp, cf, lds_bytes, st);
}

template <int DT>
int launch_dt(const FrameArgs& a, int order, bool comp, bool cf, bool mirror, int64_t lds_bytes,
              hipStream_t st)
{
    switch (order) {
    case 1: return launch_k<1, DT>(a, comp, cf, mirror, lds_bytes, st);
    case 2: return launch_k<2, DT>(a, comp, cf, mirror, lds_bytes, st);
    case 3: return launch_k<3, DT>(a, comp, cf, mirror, lds_bytes, st);
    case 4: return launch_k<4, DT>(a, comp, cf, mirror, lds_bytes, st);
    case 5: return launch_k<5, DT>(a, comp, cf, mirror, lds_bytes, st);
    case 6: return launch_k<6, DT>(a, comp, cf, mirror, lds_bytes, st);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace

int launch_frame(const FrameArgs& a, int order, int dtype, bool compensated, bool coherence,
                 bool mirror, int64_t lds_bytes, void* stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (dtype) {
    case HODMAS_F32: return launch_dt<HODMAS_F32>(a, order, compensated, coherence, mirror, lds_bytes, st);
    case HODMAS_F16: return launch_dt<HODMAS_F16>(a, order, compensated, coherence, mirror, lds_bytes, st);
    case HODMAS_I16: return launch_dt<HODMAS_I16>(a, order, compensated, coherence, mirror, lds_bytes, st);
    }
    return (int)hipErrorInvalidValue;
}

// coherence-weighted kinds exist for compensated accumulation only
template <int K, int DT, int M>
const void* batch_fn(bool comp, bool cf)
{
    if (cf)
        return comp ? reinterpret_cast<const void*>(&hodmas_batch_kernel<K, DT, true, true, M>) : nullptr;
    return comp ? reinterpret_cast<const void*>(&hodmas_batch_kernel<K, DT, true, false, M>)
                : reinterpret_cast<const void*>(&hodmas_batch_kernel<K, DT, false, false, M>);
}

template <int DT, int M>
const void* batch_fn_dt(int order, bool comp, bool cf)
{
    switch (order) {
    case 1: return batch_fn<1, DT, M>(comp, cf);
    case 2: return batch_fn<2, DT, M>(comp, cf);
    case 3: return batch_fn<3, DT, M>(comp, cf);
    case 4: return batch_fn<4, DT, M>(comp, cf);
    case 5: return batch_fn<5, DT, M>(comp, cf);
    case 6: return batch_fn<6, DT, M>(comp, cf);
    }
    return nullptr;
}

template <int M>
const void* batch_fn_m(int order, int dtype, bool comp, bool cf)
{
    switch (dtype) {
    case HODMAS_F32: return batch_fn_dt<HODMAS_F32, M>(order, comp, cf);
    case HODMAS_F16: return batch_fn_dt<HODMAS_F16, M>(order, comp, cf);
    case HODMAS_I16: return batch_fn_dt<HODMAS_I16, M>(order, comp, cf);
    }
    return nullptr;
}

int launch_orders(const FrameArgs& a, const OrderImages& out, int kmax, int dtype, bool compensated,
                  int64_t lds_bytes, void* stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (dtype) {
    case HODMAS_F32: return launch_orders_dt<HODMAS_F32>(a, out, kmax, compensated, lds_bytes, st);
    case HODMAS_F16: return launch_orders_dt<HODMAS_F16>(a, out, kmax, compensated, lds_bytes, st);
    case HODMAS_I16: return launch_orders_dt<HODMAS_I16>(a, out, kmax, compensated, lds_bytes, st);
    }
    return (int)hipErrorInvalidValue;
}

const void* batch_kernel(int kind, bool compensated)
{
    if (kind < 0 || kind >= kBatchKinds)
        return nullptr;
    const int order = kind_order(kind), dtype = kind_dtype(kind);
    const bool cf = kind_cf(kind) != 0;
    switch (kind_pairing(kind)) {
    case 1: return batch_fn_m<1>(order, dtype, compensated, cf);
    case 2: return batch_fn_m<2>(order, dtype, compensated, cf);
    }
    return nullptr;
}

int launch_batch(int kind, const BatchHeader* hdr, const BatchFrame* frames, const BatchUnit* units, int grid,
                 bool compensated, int64_t lds_bytes, void* stream)
{
    const void* fn = batch_kernel(kind, compensated);
    if (!fn)
        return (int)hipErrorInvalidValue;
    void* args[] = {(void*)&hdr, (void*)&frames, (void*)&units};
    return (int)hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, (size_t)lds_bytes,
                                static_cast<hipStream_t>(stream));
}

}  // namespace hodmas
