// MFMA GEMMs of the actor-critic MLPs for gfx950 (CDNA4).
//
// C[M, N] = A[M, K] * B[N, K]^T with float32 accumulation, for every layer of
// the forward pass (z = h W^T + b, then ELU), the input-gradient chain
// (dh = dz W, times ELU'), and the weight gradients (dW = dz^T h, split over
// the sample dimension).  Several independent problems (actor and critic, or
// all layers of both) share one launch: blockIdx.x is mapped to a
// (problem, split, tile) triple through the prefix sums in GemmArgs.
//
// Work decomposition: 256 threads = 4 wave64s per 128 x 128 tile, 2 x 2 waves
// of 64 x 64, each wave 2 x 2 MFMA blocks of 32 x 32.  bf16 operands use
// v_mfma_f32_32x32x16_bf16; float32 operands use four v_mfma_f32_32x32x2_f32
// per 8-wide k chunk.  Tiles are staged in LDS with K contiguous and a 16-byte
// row pad (conflict-free 16-byte reads for 16 consecutive rows); two k-slabs
// are in flight while the current one is multiplied (two register staging
// sets, two LDS buffers, one barrier per slab).  Operands stored transposed in memory
// (the sample-major activations used by dW) are transposed in registers, one
// 16-byte vector per row of an 8 x 8 (bf16) or 4 x 4 (float32) block.
#include "common.hpp"

#include <cstdlib>
#include <type_traits>

namespace ppo {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;

template <typename T> struct Mma;

template <> struct Mma<uint16_t> {
    // One 16-byte vector per lane = 8 consecutive k of one row: a full
    // 32x32x16 MFMA (lane l holds row l % 32, k = 8 (l / 32) .. + 7).
    __device__ static inline void mac(floatx16 &acc, const u32x4 &a, const u32x4 &b) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), acc, 0, 0, 0);
    }
};

template <> struct Mma<float> {
    // One 16-byte vector per lane = 4 consecutive k.  MFMA e (0..3) pairs
    // lane-half 0's element e with lane-half 1's element e, i.e. k = e and
    // k = 4 + e of the 8-wide chunk; A and B use the same pairing.
    __device__ static inline void mac(floatx16 &acc, const u32x4 &a, const u32x4 &b) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
    }
};

template <typename T> __device__ inline uint32_t raw_bits(T v);
template <> __device__ inline uint32_t raw_bits<float>(float v) { return __float_as_uint(v); }
template <> __device__ inline uint32_t raw_bits<uint16_t>(uint16_t v) { return v; }

// Output-side arithmetic: float32 outputs keep expm1 (the float32 path is
// held to float32 accuracy); bf16 outputs use the hardware exponential and
// the hardware round-to-nearest-even conversion, whose errors are far below
// one bf16 ulp.
template <typename T> struct Act;
template <> struct Act<float> {
    __device__ static inline float elu(float v) { return v > 0.0f ? v : expm1f(v); }
    __device__ static inline float store(float v) { return v; }
};
template <> struct Act<uint16_t> {
    __device__ static inline float elu(float v) { return v > 0.0f ? v : __expf(v) - 1.0f; }
    __device__ static inline uint16_t store(float v) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v)); }
};

// Pack VEC scalars (zero where invalid) into a 16-byte vector.
template <typename T, int VEC>
__device__ inline u32x4 pack_elems(const T (&e)[VEC]) {
    u32x4 r;
    if constexpr (sizeof(T) == 4) {
        r.x = raw_bits<T>(e[0]); r.y = raw_bits<T>(e[1]); r.z = raw_bits<T>(e[2]); r.w = raw_bits<T>(e[3]);
    } else {
        r.x = raw_bits<T>(e[0]) | (raw_bits<T>(e[1]) << 16);
        r.y = raw_bits<T>(e[2]) | (raw_bits<T>(e[3]) << 16);
        r.z = raw_bits<T>(e[4]) | (raw_bits<T>(e[5]) << 16);
        r.w = raw_bits<T>(e[6]) | (raw_bits<T>(e[7]) << 16);
    }
    return r;
}

// Row-major operand: element (r, k) at src[r * ld + k]; zero outside
// r < R, k < kend.
template <typename T>
__device__ inline u32x4 load_rowmajor(const T *src, int ld, int r, int k, int R, int kend, bool vec_ok) {
    constexpr int VEC = 16 / sizeof(T);
    if (r < R && k + VEC <= kend && vec_ok)
        return *reinterpret_cast<const u32x4 *>(src + static_cast<long long>(r) * ld + k);
    T e[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i)
        e[i] = (r < R && k + i < kend) ? src[static_cast<long long>(r) * ld + k + i] : T(0);
    return pack_elems<T, VEC>(e);
}

// Transposed operand: element (r, k) at src[k * ld + r]; loads VEC
// consecutive r for one k.
template <typename T>
__device__ inline u32x4 load_transposed(const T *src, int ld, int r, int k, int R, int kend, bool vec_ok) {
    constexpr int VEC = 16 / sizeof(T);
    if (k < kend && r + VEC <= R && vec_ok)
        return *reinterpret_cast<const u32x4 *>(src + static_cast<long long>(k) * ld + r);
    T e[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i)
        e[i] = (k < kend && r + i < R) ? src[static_cast<long long>(k) * ld + r + i] : T(0);
    return pack_elems<T, VEC>(e);
}

// in[e] holds VEC elements along r for k = e; returns the VEC elements along
// k for r = i.
template <typename T>
__device__ inline u32x4 transpose_col(const u32x4 *in, int i) {
    u32x4 o;
    if constexpr (sizeof(T) == 4) {
        o.x = in[0][i]; o.y = in[1][i]; o.z = in[2][i]; o.w = in[3][i];
    } else {
        const int w = i >> 1;
        if (i & 1) {
            o.x = (in[0][w] >> 16) | (in[1][w] & 0xFFFF0000u);
            o.y = (in[2][w] >> 16) | (in[3][w] & 0xFFFF0000u);
            o.z = (in[4][w] >> 16) | (in[5][w] & 0xFFFF0000u);
            o.w = (in[6][w] >> 16) | (in[7][w] & 0xFFFF0000u);
        } else {
            o.x = (in[0][w] & 0xFFFFu) | (in[1][w] << 16);
            o.y = (in[2][w] & 0xFFFFu) | (in[3][w] << 16);
            o.z = (in[4][w] & 0xFFFFu) | (in[5][w] << 16);
            o.w = (in[6][w] & 0xFFFFu) | (in[7][w] << 16);
        }
    }
    return o;
}

// Buffer resource over [base, base + bytes) (raw buffer, no swizzle): loads
// past the end return zeros instead of touching memory.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *base, long long bytes) {
    const int n = bytes > 0x7FFFFFFFLL ? 0x7FFFFFFF : static_cast<int>(bytes < 0 ? 0 : bytes);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), static_cast<short>(0), n, 0x00020000);
}

// bf16 operands stored transposed (MODE 1) are staged without any register
// transpose: each 16-byte global vector (8 consecutive rows at one k) goes to
// LDS as is, in a k-major tile [BK][ROWS] whose 16-byte columns are XOR-
// swizzled per k-row, and the MFMA fragments are read back with the LDS
// transpose load (see frag_tr).  The swizzle keeps both the stores and the
// transposed reads of a half-wave on distinct banks.
template <int ROWS>
__device__ inline int tr_swz(int k) {
    return ROWS == 128 ? ((k & 3) << 2) : (((k >> 1) & 1) << 2);
}
template <int ROWS>
__device__ inline int tr_index(int k, int r) {  // element (k, r) of a k-major tile
    return k * ROWS + ((((r >> 3) ^ tr_swz<ROWS>(k))) << 3) + (r & 7);
}

template <typename T, int MODE, int ROWS, int BK>
struct TileLoader {
    static constexpr int VEC = 16 / sizeof(T);
    static constexpr int PITCH = BK + VEC;
    // TR: bf16 transposed operand staged k-major (no register transpose).
    static constexpr bool TR = MODE == 1 && sizeof(T) == 2;
    static_assert(!TR || ROWS == 64 || ROWS == 128, "k-major tiles have 64 or 128 rows");
    // Elements of one LDS tile of this operand.
    static constexpr int ELEMS = TR ? BK * ROWS : ROWS * PITCH;
    // MODE 0 and TR: units are 16-byte vectors (along k, resp. along rows);
    // float32 MODE 1: VEC x VEC blocks transposed in registers.
    static constexpr int UNITS = (MODE == 0 || TR) ? ROWS * BK / VEC : (ROWS / VEC) * (BK / VEC);
    static constexpr int NT = UNITS < kThreads ? UNITS : kThreads;
    static constexpr int PER = UNITS / NT;
    static constexpr int REGS = (MODE == 0 || TR) ? PER : PER * VEC;
    static_assert(UNITS % NT == 0, "tile units must divide evenly");
    u32x4 r[REGS];
    int voff[PER];  // fast path: byte offset of each load at k = 0
    int kofs[PER];  // fast path, MODE 0: k of each load within the slab

    // Position of unit u: MODE 0 (row, k) of a k-vector; TR (k, row) of a
    // row-vector.
    __device__ static inline void unit0(int u, int &row, int &kv) {
        row = u / (BK / VEC);
        kv = (u % (BK / VEC)) * VEC;
    }
    __device__ static inline void unit_tr(int u, int &kk, int &rv) {
        kk = u / (ROWS / VEC);
        rv = (u % (ROWS / VEC)) * VEC;
    }

    // Fast path set-up for a tile starting at row r0.  The operand must be
    // 16-byte aligned with ld % VEC == 0 and kend % VEC == 0; its buffer
    // resource ends at the last valid byte (MODE 0: R rows of ld; MODE 1:
    // kend rows of ld), so rows past R (MODE 0) and k past kend (MODE 1)
    // read as zeros.  MODE 1 rows past R read neighbouring features, which
    // only reach outputs the epilogue discards.
    __device__ inline void setup(int ld, int r0, int t) {
        if (NT < kThreads && (t < 0 || t >= NT)) return;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int u = t + p * NT;
            if constexpr (MODE == 0) {
                int row, kv;
                unit0(u, row, kv);
                voff[p] = ((r0 + row) * ld + kv) * static_cast<int>(sizeof(T));
                kofs[p] = kv;
            } else if constexpr (TR) {
                int kk, rv;
                unit_tr(u, kk, rv);
                voff[p] = (kk * ld + r0 + rv) * static_cast<int>(sizeof(T));
                kofs[p] = 0;
            } else {
                const int kb = u % (BK / VEC);
                const int rb = u / (BK / VEC);
                voff[p] = (kb * VEC * ld + r0 + rb * VEC) * static_cast<int>(sizeof(T));
                kofs[p] = 0;
            }
        }
    }

    // Fast path: one buffer load per 16-byte vector, k0 folded into the
    // scalar offset, nothing done to the loaded registers (so the loads stay
    // in flight until the LDS store).  MODE 0 vectors at or past kend (a
    // partial last slab) get an offset past the resource's end and read as
    // zeros.
    static constexpr int kOutside = 0x7FFFFFF0;
    __device__ inline void load_fast(__amdgpu_buffer_rsrc_t rs, int ld, int k0, int kend, int t) {
        if (NT < kThreads && (t < 0 || t >= NT)) return;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            // k0 and ld are uniform; readfirstlane keeps the scalar offset in an
            // SGPR (the compiler cannot always prove uniformity by itself)
            if constexpr (MODE == 0) {
                const int so = __builtin_amdgcn_readfirstlane(k0 * static_cast<int>(sizeof(T)));
                const int vo = k0 + kofs[p] < kend ? voff[p] : kOutside;
                r[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0);
            } else if constexpr (TR) {
                const int so = __builtin_amdgcn_readfirstlane(k0 * ld * static_cast<int>(sizeof(T)));
                r[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff[p], so, 0);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int so = __builtin_amdgcn_readfirstlane((k0 + e) * ld * static_cast<int>(sizeof(T)));
                    r[p * VEC + e] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff[p], so, 0);
                }
            }
        }
    }

    __device__ inline void load(const T *src, int ld, int R, int r0, int k0, int kend, int t, bool vec_ok) {
        if (NT < kThreads && (t < 0 || t >= NT)) return;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int u = t + p * NT;
            if constexpr (MODE == 0) {
                int row, kv;
                unit0(u, row, kv);
                r[p] = load_rowmajor<T>(src, ld, r0 + row, k0 + kv, R, kend, vec_ok);
            } else if constexpr (TR) {
                int kk, rv;
                unit_tr(u, kk, rv);
                r[p] = load_transposed<T>(src, ld, r0 + rv, k0 + kk, R, kend, vec_ok);
            } else {
                // k-block fastest across lanes: the transposed LDS rows written by
                // neighbouring lanes then fall on disjoint banks (see store()).
                const int kb = u % (BK / VEC);
                const int rb = u / (BK / VEC);
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    r[p * VEC + e] = load_transposed<T>(src, ld, r0 + rb * VEC, k0 + kb * VEC + e, R, kend, vec_ok);
            }
        }
    }

    __device__ inline void store(T *lds, int t) const {
        if (NT < kThreads && (t < 0 || t >= NT)) return;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int u = t + p * NT;
            if constexpr (MODE == 0) {
                int row, kv;
                unit0(u, row, kv);
                *reinterpret_cast<u32x4 *>(lds + row * PITCH + kv) = r[p];
            } else if constexpr (TR) {
                int kk, rv;
                unit_tr(u, kk, rv);
                *reinterpret_cast<u32x4 *>(lds + tr_index<ROWS>(kk, rv)) = r[p];
            } else {
                const int kb = u % (BK / VEC);
                const int rb = u / (BK / VEC);
#pragma unroll
                for (int i = 0; i < VEC; ++i)
                    *reinterpret_cast<u32x4 *>(lds + (rb * VEC + i) * PITCH + kb * VEC) =
                        transpose_col<T>(&r[p * VEC], i);
            }
        }
    }

    // TR only: add this thread's staged vectors (8 rows each, the same 8
    // rows for every unit of the thread) to its per-row partial sums.
    __device__ inline void accumulate_rows(float (&acc)[VEC], int t) const {
        if (NT < kThreads && (t < 0 || t >= NT)) return;
#pragma unroll
        for (int p = 0; p < PER; ++p)
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                acc[2 * w] += __uint_as_float(r[p][w] << 16);
                acc[2 * w + 1] += __uint_as_float(r[p][w] & 0xFFFF0000u);
            }
    }
};

// MFMA fragment (32 rows x 16 k, bf16) from a k-major swizzled tile with the
// gfx950 LDS transpose load.  Within each 16-lane group, lane i receives
// element (i mod 4) of the 8-byte chunks addressed by lanes i/4, i/4+4,
// i/4+8 and i/4+12 of its group; so lane s of a group addresses the chunk
// (k = kb + s/4, rows 4 (s mod 4) .. +3) and receives row s at k = kb .. kb+3.
// Two loads (k and k + 4) give the 8 consecutive k of the MFMA operand.
typedef short v4i16 __attribute__((ext_vector_type(4)));
template <int ROWS>
__device__ inline u32x4 frag_tr(const uint16_t *tile, int frow0, int kc, int lane) {
    const int g = lane >> 4, sl = lane & 15;
    const int r = frow0 + 16 * (g & 1) + 4 * (sl & 3);
    const int k = kc * 16 + 8 * (g >> 1) + (sl >> 2);
    typedef __attribute__((address_space(3))) v4i16 lds_v4i16;
    const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
        (lds_v4i16 *)(const_cast<uint16_t *>(tile) + tr_index<ROWS>(k, r)));
    const v4i16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
        (lds_v4i16 *)(const_cast<uint16_t *>(tile) + tr_index<ROWS>(k + 4, r)));
    u32x4 o;
    o.x = static_cast<uint16_t>(lo.x) | (static_cast<uint32_t>(static_cast<uint16_t>(lo.y)) << 16);
    o.y = static_cast<uint16_t>(lo.z) | (static_cast<uint32_t>(static_cast<uint16_t>(lo.w)) << 16);
    o.z = static_cast<uint16_t>(hi.x) | (static_cast<uint32_t>(static_cast<uint16_t>(hi.y)) << 16);
    o.w = static_cast<uint16_t>(hi.z) | (static_cast<uint32_t>(static_cast<uint16_t>(hi.w)) << 16);
    return o;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Give XCD x a contiguous range of logical tiles, so neighbouring
// tiles -- which share an A row block (forward, input gradient) or a k-range
// of both operands (weight gradient) -- are served from the same L2.
constexpr int kXcds = 8;
__device__ inline int xcd_swizzle(int b, int n) {
    const int xcd = b % kXcds, slot = b / kXcds;
    const int q = n / kXcds, r = n % kXcds;
    return xcd * q + min(xcd, r) + slot;
}

// FAST: every problem of the launch has 16-byte aligned operands with
// ld % VEC == 0 and K % VEC == 0 (checked on the host); its slabs are loaded
// with buffer loads and nothing else, so the loads stay in flight across the
// multiply of the previous slabs.  Otherwise every element is bounds-checked.
// Decodes dispatch index d into the tile it computes: problem pi, tile
// origin (m0, n0), split and column-tile index, and the split's k-range.
template <int BM, int BN, int BK>
__device__ inline void decode_tile(const GemmArgs &args, int d, int &pi, int &m0, int &n0, int &split, int &tn,
                                   int &kbeg, int &kend) {
    const int bid = xcd_swizzle(d, args.total_tiles);
    pi = 0;
    while (pi + 1 < args.count && bid >= args.p[pi + 1].tile_begin) ++pi;
    const GemmProblem &P = args.p[pi];
    const int local = bid - P.tile_begin;
    const int per_split = P.tiles_m * P.tiles_n;
    split = local / per_split;
    const int rem = local - split * per_split;
    const int tm = rem / P.tiles_n;
    tn = rem - tm * P.tiles_n;
    m0 = tm * BM;
    n0 = tn * BN;
    kbeg = split * P.kps;
    kend = min(P.K, kbeg + P.kps);
}

// Persistent on the FAST path: workgroup b takes dispatch indices b, b + G,
// b + 2G, ... (G = gridDim.x, a multiple of 8, so every index of a workgroup
// maps to the same XCD range) and loads the first slab of its next tile while
// it runs the current tile's epilogue.
template <typename T, int BM, int BN, int AMODE, int BMODE, int EPI, bool FAST>
__global__ __launch_bounds__(kThreads, 2) void gemm_kernel(const GemmArgs args) {
    constexpr int BK = GemmTile<T>::BK;
    constexpr int WM = BM / 2, WN = BN / 2;   // per-wave tile (2 x 2 waves)
    constexpr int MI = WM / 32, NJ = WN / 32;  // 32 x 32 MFMA blocks per wave
    constexpr int VEC = 16 / sizeof(T);
    constexpr int PITCH = BK + VEC;
    constexpr int KC = 2 * VEC;  // k covered by one 16-byte read in each lane-half
    using LA = TileLoader<T, AMODE, BM, BK>;
    using LB = TileLoader<T, BMODE, BN, BK>;
    // Split the threads between the two operands when neither needs all of them.
    constexpr int B_OFF = (LA::NT + LB::NT <= kThreads) ? LA::NT : 0;

    // Two buffers of both operand tiles; the epilogue reuses the same memory
    // to stage the float32 accumulators (WM rows of WN + 8 floats per wave).
    constexpr int BUF = LA::ELEMS + LB::ELEMS;
    constexpr int EP = WN + 8;
    constexpr size_t TILE_BYTES = 2 * BUF * sizeof(T);
    constexpr size_t STAGE_BYTES = 4 * WM * EP * sizeof(float);
    constexpr size_t LDS_BYTES = TILE_BYTES > STAGE_BYTES ? TILE_BYTES : STAGE_BYTES;
    __shared__ __attribute__((aligned(16))) unsigned char lds_mem[LDS_BYTES];
    T *const lds0 = reinterpret_cast<T *>(lds_mem);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lrow = lane & 31;
    const int lk = (lane >> 5) * VEC;

    floatx16 acc[MI][NJ];
    constexpr int TPR = kThreads / BM;
    float rowsum = 0.0f;
    float rows8[VEC];  // k-major A tiles: per-thread partial sums of its 8 rows

    // Two k-slabs in flight: staging set 0 holds even slabs, set 1 odd ones.
    // While slab kt is multiplied out of one LDS buffer, slab kt + 1 sits in
    // registers on its way to the other buffer and slab kt + 2 is loading.
    LA la0, la1;
    LB lb0, lb1;
    auto setup_loaders = [&](int pi, int m0, int n0) {
        if constexpr (FAST) {
            la0.setup(args.p[pi].lda, m0, tid);
            lb0.setup(args.p[pi].ldb, n0, tid - B_OFF);
#pragma unroll
            for (int p = 0; p < LA::PER; ++p) {
                la1.voff[p] = la0.voff[p];
                la1.kofs[p] = la0.kofs[p];
            }
#pragma unroll
            for (int p = 0; p < LB::PER; ++p) {
                lb1.voff[p] = lb0.voff[p];
                lb1.kofs[p] = lb0.kofs[p];
            }
        }
    };
    // Loads slab kt of a tile into a staging set.  With a second B operand
    // the k-range runs twice: slabs nkb .. 2 nkb - 1 pair A's slabs 0 ..
    // nkb - 1 with B2 (slabs past the end read zeros either way).
    auto load_slab = [&](int pi, int m0, int n0, int kbeg, int kend, LA &la, LB &lb, int kt) {
        const GemmProblem &Q = args.p[pi];
        const int nkb = (kend - kbeg + BK - 1) / BK;
        const bool second = Q.B2 != nullptr && kt >= nkb;
        const int k0 = kbeg + (second ? kt - nkb : kt) * BK;
        const void *Bp = second ? Q.B2 : Q.B;
        if constexpr (FAST) {
            const __amdgpu_buffer_rsrc_t a_rs =
                make_rsrc(Q.A, static_cast<long long>(AMODE == 0 ? Q.M : kend) * Q.lda * static_cast<int>(sizeof(T)));
            const __amdgpu_buffer_rsrc_t b_rs =
                make_rsrc(Bp, static_cast<long long>(BMODE == 0 ? Q.N : kend) * Q.ldb * static_cast<int>(sizeof(T)));
            la.load_fast(a_rs, Q.lda, k0, kend, tid);
            lb.load_fast(b_rs, Q.ldb, k0, kend, tid - B_OFF);
        } else {
            // 16-byte vector loads need a 16-byte aligned base and row pitch.
            const bool a_vec = (Q.lda % VEC) == 0 && (reinterpret_cast<uintptr_t>(Q.A) & 15u) == 0;
            const bool b_vec = (Q.ldb % VEC) == 0 && (reinterpret_cast<uintptr_t>(Bp) & 15u) == 0;
            la.load(static_cast<const T *>(Q.A), Q.lda, Q.M, m0, k0, kend, tid, a_vec);
            lb.load(static_cast<const T *>(Bp), Q.ldb, Q.N, n0, k0, kend, tid - B_OFF, b_vec);
        }
    };
    // Stores a staging set into LDS buffer `buf`; k-major A tiles also feed
    // the row sums of the bias gradient from the staged registers.
    auto store_slab = [&](bool do_rowsum, LA &la, LB &lb, int buf) {
        la.store(lds0 + buf * BUF, tid);
        lb.store(lds0 + buf * BUF + LA::ELEMS, tid - B_OFF);
        if constexpr (LA::TR && EPI == kEpiPartial) {
            if (do_rowsum) la.accumulate_rows(rows8, tid);
        }
    };
    auto compute = [&](bool do_rowsum, int buf) {
        const T *As = lds0 + buf * BUF;
        const T *Bs = As + LA::ELEMS;
#pragma unroll
        for (int kc = 0; kc < BK / KC; ++kc) {
            u32x4 a[MI], b[NJ];
#pragma unroll
            for (int i = 0; i < MI; ++i) {
                if constexpr (LA::TR)
                    a[i] = frag_tr<BM>(reinterpret_cast<const uint16_t *>(As), wm * WM + i * 32, kc, lane);
                else
                    a[i] = *reinterpret_cast<const u32x4 *>(As + (wm * WM + i * 32 + lrow) * PITCH + kc * KC + lk);
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                if constexpr (LB::TR)
                    b[j] = frag_tr<BN>(reinterpret_cast<const uint16_t *>(Bs), wn * WN + j * 32, kc, lane);
                else
                    b[j] = *reinterpret_cast<const u32x4 *>(Bs + (wn * WN + j * 32 + lrow) * PITCH + kc * KC + lk);
            }
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j) Mma<T>::mac(acc[i][j], a[i], b[j]);
        }
        if (!LA::TR && do_rowsum) {
            // TPR adjacent threads per row of A, each summing a part of the slab.
            const int row = tid / TPR;
            const T *src = As + row * PITCH + (tid % TPR) * (BK / TPR);
#pragma unroll
            for (int e = 0; e < BK / TPR; ++e) rowsum += Elem<T>::to_f(src[e]);
        }
    };

    // Epilogue constants: WN / 4 lanes cover one staged row (4 floats each);
    // for WN = 64 every 16-lane group of a 16-byte LDS read touches all 64
    // banks once.
    constexpr int CW = 4;
    constexpr int LPR = WN / CW;         // lanes per staged row
    constexpr int RPI = 64 / LPR;        // rows per iteration
    constexpr int ITS = WM / RPI;        // epilogue iterations per lane
    const int sub_r = lane / LPR;
    const int sub_c = (lane % LPR) * CW;

    const int total = args.total_tiles;
    const int G = gridDim.x;
    int d = blockIdx.x;
    int pi, m0, n0, split, tn, kbeg, kend;
    decode_tile<BM, BN, BK>(args, d, pi, m0, n0, split, tn, kbeg, kend);
    setup_loaders(pi, m0, n0);
    // On the FAST path every load and LDS store of the loop is unconditional:
    // slabs past the end read as zeros (their offsets fall outside the buffer
    // resources) and land in a buffer nobody reads again.  Conditional loads
    // would make the compiler wait for them before the next LDS store.
    auto slabs = [&](const GemmProblem &Q, int kb, int ke) { return ((ke - kb + BK - 1) / BK) * (Q.B2 ? 2 : 1); };
    load_slab(pi, m0, n0, kbeg, kend, la0, lb0, 0);
    if (FAST || slabs(args.p[pi], kbeg, kend) > 1) load_slab(pi, m0, n0, kbeg, kend, la1, lb1, 1);

    while (true) {
        const GemmProblem &P = args.p[pi];
        const int nk = slabs(P, kbeg, kend);
        const bool do_rowsum = (EPI == kEpiPartial) && tn == 0;
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
        rowsum = 0.0f;
#pragma unroll
        for (int e = 0; e < VEC; ++e) rows8[e] = 0.0f;

        store_slab(do_rowsum, la0, lb0, 0);
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            // even slab kt in buffer 0
            if (FAST || kt + 2 < nk) load_slab(pi, m0, n0, kbeg, kend, la0, lb0, kt + 2);
            compute(do_rowsum, 0);
            if (FAST || kt + 1 < nk) store_slab(do_rowsum, la1, lb1, 1);
            __syncthreads();
            if (kt + 1 >= nk) break;
            // odd slab kt + 1 in buffer 1
            if (FAST || kt + 3 < nk) load_slab(pi, m0, n0, kbeg, kend, la1, lb1, kt + 3);
            compute(do_rowsum, 1);
            if (FAST || kt + 2 < nk) store_slab(do_rowsum, la0, lb0, 0);
            __syncthreads();
        }

        if constexpr (EPI == kEpiPartial && LA::TR) {
            // every thread summed the same 8 rows in every slab: combine the
            // threads of each row group through LDS, in thread order
            if (do_rowsum) {
                constexpr int GROUPS = BM / VEC;            // row groups of 8
                constexpr int PER_GROUP = kThreads / GROUPS;
                float *red = reinterpret_cast<float *>(lds_mem);
#pragma unroll
                for (int e = 0; e < VEC; ++e) red[tid * VEC + e] = rows8[e];
                __syncthreads();
                if (tid < BM) {
                    const int gq = tid / VEC, e = tid % VEC;
                    float v = 0.0f;
                    for (int q = 0; q < PER_GROUP; ++q) v += red[(gq + GROUPS * q) * VEC + e];
                    const int row = m0 + tid;
                    if (row < P.M) P.rowsum[static_cast<long long>(split) * P.M + row] = v;
                }
                __syncthreads();
            }
        } else if constexpr (EPI == kEpiPartial) {
            if (do_rowsum) {
#pragma unroll
                for (int o = 1; o < TPR; o <<= 1) rowsum += __shfl_xor(rowsum, o);
                const int row = m0 + tid / TPR;
                if (tid % TPR == 0 && row < P.M) P.rowsum[static_cast<long long>(split) * P.M + row] = rowsum;
            }
        }

        // Epilogue: accumulators -> LDS (float32, per-wave WM x WN tile) -> each
        // lane takes 4 consecutive columns of a row, applies the epilogue and
        // writes them with one 8-byte (bf16) or 16-byte (float32) store.  Rows are
        // padded to EP = WN + 8 floats (EP = 8 mod 16), so the two lane halves of
        // the scattered accumulator writes (rows 4 apart) hit disjoint banks.
        const int col = n0 + wn * WN + sub_c;
        const bool full_cols = col + CW <= P.N;

        // ELU' input: every activation this lane needs is loaded before the
        // accumulators go through LDS, all loads in flight at once (the output
        // stores that follow could alias them as far as the compiler knows, so
        // loads inside the store loop would each wait for the previous store).
        T hreg[ITS][CW];
        if constexpr (EPI == kEpiDElu && FAST) {
            // buffer loads: rows past M read as zeros, no branches, one scalar
            // offset per iteration
            const __amdgpu_buffer_rsrc_t h_rs =
                make_rsrc(P.H, static_cast<long long>(P.M) * P.ldh * static_cast<int>(sizeof(T)));
            const int vo = ((m0 + wm * WM + sub_r) * P.ldh + col) * static_cast<int>(sizeof(T));
#pragma unroll
            for (int it = 0; it < ITS; ++it) {
                const int so = __builtin_amdgcn_readfirstlane(it * RPI * P.ldh * static_cast<int>(sizeof(T)));
                if constexpr (sizeof(T) == 2) {
                    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
                    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(h_rs, vo, so, 0);
                    *reinterpret_cast<u32x2 *>(hreg[it]) = v;
                } else {
                    *reinterpret_cast<u32x4 *>(hreg[it]) = __builtin_amdgcn_raw_buffer_load_b128(h_rs, vo, so, 0);
                }
            }
        } else if constexpr (EPI == kEpiDElu) {
            const bool h_vec = full_cols && (P.ldh % CW) == 0 && (reinterpret_cast<uintptr_t>(P.H) & 15u) == 0;
#pragma unroll
            for (int it = 0; it < ITS; ++it) {
                const int row = m0 + wm * WM + it * RPI + sub_r;
#pragma unroll
                for (int e = 0; e < CW; ++e) hreg[it][e] = T(0);
                if (row >= P.M || col >= P.N) continue;
                const T *hsrc = static_cast<const T *>(P.H) + static_cast<long long>(row) * P.ldh + col;
                if (h_vec) {
                    if constexpr (sizeof(T) == 2) {
                        *reinterpret_cast<uint2 *>(hreg[it]) = *reinterpret_cast<const uint2 *>(hsrc);
                    } else {
                        *reinterpret_cast<u32x4 *>(hreg[it]) = *reinterpret_cast<const u32x4 *>(hsrc);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < CW; ++e) hreg[it][e] = (col + e < P.N) ? hsrc[e] : T(0);
                }
            }
        }

        float *stage = reinterpret_cast<float *>(lds_mem) + wave * WM * EP;
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    stage[(i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3)) * EP + j * 32 + lrow] = acc[i][j][r];
        __syncthreads();

        // the next tile's first slab loads while this tile's epilogue runs
        const int dn = d + G;
        const bool has_next = FAST && dn < total;
        int npi = pi, nm0 = m0, nn0 = n0, nsplit = split, ntn = tn, nkbeg = kbeg, nkend = kend;
        if (has_next) {
            decode_tile<BM, BN, BK>(args, dn, npi, nm0, nn0, nsplit, ntn, nkbeg, nkend);
            setup_loaders(npi, nm0, nn0);
            load_slab(npi, nm0, nn0, nkbeg, nkend, la0, lb0, 0);
        }

        if (col < P.N) {
            float bias[CW];
            if constexpr (EPI == kEpiBiasElu) {
#pragma unroll
                for (int e = 0; e < CW; ++e) bias[e] = (col + e < P.N) ? P.bias[col + e] : 0.0f;
            }
            const bool c_vec = full_cols && (P.ldc % CW) == 0 && (reinterpret_cast<uintptr_t>(P.C) & 15u) == 0;
            // Full 4-column segments go out as one buffer store each (rows past
            // M fall outside the resource and are dropped); ragged column edges
            // take element stores.  Keeping the two paths on different
            // instructions stops the compiler from merging them into split
            // partial-width stores.
            using OutT = typename std::conditional<EPI == kEpiPartial, float, T>::type;
            OutT *cbase = static_cast<OutT *>(P.C) + (EPI == kEpiPartial ? split * P.c_split_stride : 0);
            const __amdgpu_buffer_rsrc_t c_rs =
                make_rsrc(cbase, static_cast<long long>(P.M) * P.ldc * static_cast<int>(sizeof(OutT)));
            const int c_vo = ((m0 + wm * WM + sub_r) * P.ldc + col) * static_cast<int>(sizeof(OutT));
#pragma unroll
            for (int it = 0; it < ITS; ++it) {
                const int lr = it * RPI + sub_r;
                const int row = m0 + wm * WM + lr;
                const int c_so = __builtin_amdgcn_readfirstlane(it * RPI * P.ldc * static_cast<int>(sizeof(OutT)));
                float v[CW];
                *reinterpret_cast<float4 *>(&v[0]) = *reinterpret_cast<const float4 *>(stage + lr * EP + sub_c);
                OutT out[CW];
                if constexpr (EPI == kEpiPartial) {
#pragma unroll
                    for (int e = 0; e < CW; ++e) out[e] = v[e];
                } else {
                    if constexpr (EPI == kEpiBiasElu) {
#pragma unroll
                        for (int e = 0; e < CW; ++e) v[e] = Act<T>::elu(v[e] + bias[e]);
                    } else {
#pragma unroll
                        for (int e = 0; e < CW; ++e) {
                            const float hv = Elem<T>::to_f(hreg[it][e]);
                            v[e] *= hv > 0.0f ? 1.0f : hv + 1.0f;
                        }
                    }
#pragma unroll
                    for (int e = 0; e < CW; ++e) out[e] = Act<T>::store(v[e]);
                }
                if (c_vec) {
                    if constexpr (sizeof(OutT) == 2) {
                        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
                        __builtin_amdgcn_raw_buffer_store_b64(*reinterpret_cast<const u32x2 *>(out), c_rs, c_vo, c_so,
                                                              0);
                    } else {
                        __builtin_amdgcn_raw_buffer_store_b128(*reinterpret_cast<const u32x4 *>(out), c_rs, c_vo, c_so,
                                                               0);
                    }
                } else if (row < P.M) {
                    OutT *dst = cbase + static_cast<long long>(row) * P.ldc + col;
#pragma unroll
                    for (int e = 0; e < CW; ++e)
                        if (col + e < P.N) dst[e] = out[e];
                }
            }
        }

        if (!has_next) break;
        d = dn;
        pi = npi;
        m0 = nm0;
        n0 = nn0;
        split = nsplit;
        tn = ntn;
        kbeg = nkbeg;
        kend = nkend;
        load_slab(pi, m0, n0, kbeg, kend, la1, lb1, 1);
        // the staged accumulators are read before the next tile's slab 0 goes
        // into the same memory
        __syncthreads();
    }
}

// Whether every problem qualifies for the buffer-load path.
template <typename T>
bool all_fast(const GemmArgs &args) {
    constexpr int VEC = 16 / sizeof(T);
    auto ok = [](const void *p, int ld) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0 && ld % VEC == 0; };
    for (int i = 0; i < args.count; ++i) {
        const GemmProblem &q = args.p[i];
        if (!ok(q.A, q.lda) || !ok(q.B, q.ldb) || q.K % VEC != 0) return false;
        if (q.B2 && !ok(q.B2, q.ldb)) return false;
        if (q.splits > 1 && q.kps % VEC != 0) return false;
    }
    return true;
}

// Workgroups of a persistent FAST kernel: as many as can be resident at
// once (occupancy per CU times the CU count, rounded down to a multiple of
// 8), queried once per kernel.  PPO_GEMM_GRID_CAP=0 turns persistence off
// (one tile per workgroup).  Launched non-persistently, the same kernel runs
// exactly one tile per workgroup.
int persistence_enabled() {
    static const int on = [] {
        const char *e = std::getenv("PPO_GEMM_GRID_CAP");
        return e && std::atoi(e) <= 0 ? 0 : 1;
    }();
    return on;
}

template <typename K>
int resident_grid(K kernel) {
    static int grid = -1;
    if (grid < 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess) {
            grid = 0;
        } else {
            grid = (cus * per_cu) / 8 * 8;
        }
    }
    return grid;
}

template <typename T, int BM, int BN, int AMODE, int BMODE, int EPI, bool FAST>
hipError_t launch_one(const GemmArgs &args, hipStream_t s) {
    auto kernel = gemm_kernel<T, BM, BN, AMODE, BMODE, EPI, FAST>;
    int g = args.total_tiles;
    // measured: persistence pays off for the 128 x 128 tiles only (smaller
    // tiles already overlap through more resident workgroups per CU)
    if (FAST && BM == 128 && BN == 128 && persistence_enabled()) {
        const int cap = resident_grid(kernel);
        if (cap > 0 && g > cap) g = cap;
    }
    hipLaunchKernelGGL(kernel, dim3(g), dim3(kThreads), 0, s, args);
    return hipGetLastError();
}

template <typename T, int BM, int BN, bool FAST>
hipError_t launch_tiled(int a_mode, int b_mode, int epi, const GemmArgs &args, hipStream_t s) {
    if (a_mode == 0 && b_mode == 0 && epi == kEpiBiasElu)
        return launch_one<T, BM, BN, 0, 0, kEpiBiasElu, FAST>(args, s);
    if (a_mode == 0 && b_mode == 0 && epi == kEpiDElu)
        return launch_one<T, BM, BN, 0, 0, kEpiDElu, FAST>(args, s);
    if (a_mode == 0 && b_mode == 1 && epi == kEpiDElu)
        return launch_one<T, BM, BN, 0, 1, kEpiDElu, FAST>(args, s);
    if (a_mode == 1 && b_mode == 1 && epi == kEpiPartial)
        return launch_one<T, BM, BN, 1, 1, kEpiPartial, FAST>(args, s);
    return hipErrorInvalidValue;
}

template <typename T, int BM, int BN>
hipError_t launch_tiled(int a_mode, int b_mode, int epi, const GemmArgs &args, hipStream_t s) {
    return all_fast<T>(args) ? launch_tiled<T, BM, BN, true>(a_mode, b_mode, epi, args, s)
                             : launch_tiled<T, BM, BN, false>(a_mode, b_mode, epi, args, s);
}

template <typename T>
hipError_t launch_typed(int a_mode, int b_mode, int epi, const GemmArgs &args, hipStream_t s) {
    switch (args.tile) {
        case kTile128x128: return launch_tiled<T, 128, 128>(a_mode, b_mode, epi, args, s);
        case kTile64x128: return launch_tiled<T, 64, 128>(a_mode, b_mode, epi, args, s);
        case kTile128x64: return launch_tiled<T, 128, 64>(a_mode, b_mode, epi, args, s);
        case kTile64x64: return launch_tiled<T, 64, 64>(a_mode, b_mode, epi, args, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_gemm(Precision prec, int a_mode, int b_mode, int epi, const GemmArgs &args, hipStream_t s) {
    if (args.total_tiles <= 0) return hipSuccess;
    return prec == kBF16 ? launch_typed<uint16_t>(a_mode, b_mode, epi, args, s)
                         : launch_typed<float>(a_mode, b_mode, epi, args, s);
}

}  // namespace ppo
