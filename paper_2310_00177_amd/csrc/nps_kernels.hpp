// HIP kernels for gfx950 (CDNA4) of the neural-preconditioned Poisson solve.
//
// One NPSDO iteration (Alg. 1) is a fixed sequence of launches, none of them
// a control kernel; each scalar stage of Alg. 1 runs inside the first kernel
// that needs its result:
//   residual    Step stage (alpha = r.d / d.Ad of the previous direction, or
//               a breakdown), x += alpha d, the literal residual r = b - A x
//               (double), partial ||r||^2
//   down_l1     CConv_1^1(r) and its 2x average pool (Alg. 2, first level)
//   down        CConv_1^l + pool on the coarser levels
//   bottom      the smallest levels in one workgroup (down, coarsest CConv,
//               up) and the Residual stage: ||r||, the convergence test, 1/||r||
//   up          trilinear upsampling + CConv_2^l + c1 x1 + c2 x2
//   up_l1       dhat = P(r)/||r|| on fluid cells; partial dhat . A d_i
//   ortho       Dots stage (beta_i = dhat . A d_i / d_i . A d_i), d = dhat -
//               sum beta_i d_i, A d; partial d . A d, r . d
// The per-cell kernels K_t(p) of a level are either regenerated from the
// labels on chip every application (MFMA for the large levels, vector ALU in
// FP64) or, for levels of at most 32768 cells, formed once per solve.
//
// No kernel synchronises across workgroups: each reduction writes one
// partial per block, and the kernel that consumes the sum adds the partials
// in block order (deterministic).  Kernel boundaries provide the cross-XCD
// visibility.
#pragma once

#include "nps_internal.hpp"

#include <cmath>
#include <type_traits>

namespace nps {

// Occupancy floor of a kernel (waves per SIMD): caps its registers at
// 512 / n so that n waves of it fit per SIMD.
#define NPS_WAVES_PER_EU(n) __attribute__((amdgpu_waves_per_eu(n)))

// The three-piece bf16 weights of the FP32 MFMA path need more registers.
// (Higher floors make the CConv kernels spill and run slower.)
constexpr int waves_floor(int km) { return km == kMfmaBf16x3 ? 3 : 4; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block sum of kRedWidth values; value w of block b goes to partials[w * kMaxRedBlocks + b].
template <int NT>
__device__ __forceinline__ void block_partials(double (&v)[kRedWidth], double* partials) {
    __shared__ double sh[kRedWidth][NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int w = 0; w < kRedWidth; ++w) v[w] = wave_sum(v[w]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int w = 0; w < kRedWidth; ++w) sh[w][wid] = v[w];
    }
    __syncthreads();
    if (threadIdx.x < kRedWidth) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += sh[threadIdx.x][i];
        partials[(size_t)threadIdx.x * kMaxRedBlocks + blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// tile helpers
// ---------------------------------------------------------------------------
struct TileOrigin {
    int x0, y0, z0;
};

// The tiles a block processes: [t0, t1) with stride `step`.  When the grid
// is a multiple of kXcds, die x (blocks b with b % kXcds == x) owns the x-th
// contiguous eighth of the tiles in x-fastest order, so tiles that share
// halos are staged through the same L2.
struct TileSpan {
    int t0, t1, step;
};

__device__ __forceinline__ TileSpan tile_span(int ntiles) {
    const int G = gridDim.x, b = blockIdx.x;
    if (G % kXcds != 0) return TileSpan{b, ntiles, G};
    const int chunk = (ntiles + kXcds - 1) / kXcds;
    const int x = b % kXcds;
    return TileSpan{x * chunk + b / kXcds, min((x + 1) * chunk, ntiles), G / kXcds};
}

__device__ __forceinline__ TileOrigin tile_origin(int tile, Tiles tl) {
    TileOrigin o;
    o.x0 = (tile % tl.ntx) * TX;
    o.y0 = ((tile / tl.ntx) % tl.nty) * TY;
    o.z0 = (tile / (tl.ntx * tl.nty)) * TZ;
    return o;
}

// Grids hold at most 1e9 cells (the entry points check), so the index of an
// in-grid cell is formed in 32 bits.
__device__ __forceinline__ size_t cell_index(Grid g, int z, int y, int x) {
    return (size_t)(uint32_t)((z * g.ny + y) * g.nx + x);
}

__device__ __forceinline__ bool in_grid(Grid g, int z, int y, int x) {
    return x >= 0 && y >= 0 && z >= 0 && x < g.nx && y < g.ny && z < g.nz;
}

// Offset of window position o = 9(oz+1) + 3(oy+1) + (ox+1) inside the haloed LDS tile.
__host__ __device__ constexpr int halo_off(int o) {
    return (o / 9 - 1) * HY * HX + ((o / 3) % 3 - 1) * HX + (o % 3 - 1);
}

__device__ __forceinline__ int halo_base(int lx, int ly, int lz) { return ((lz + 1) * HY + (ly + 1)) * HX + (lx + 1); }

// Stage NH elements of a tile into LDS in two phases: get(i) only issues
// the global loads of element i (always valid addresses: elements outside
// the grid read the pad constants below; no use of the loaded values, so
// the phase is straight-line code), then put(i, v) forms and stores the
// elements.  Every load of the thread is in flight before the first put, so
// the tile waits for one memory latency rather than one per element.  The
// last, partial round reloads element NH - 1 where it runs past the end and
// stores it past the end: the destination arrays hold whole rounds
// (pad_block), and nothing reads the padding.  load_batch / put_batch are
// the two phases on their own, for kernels that keep the next tile's loads
// in flight while they compute the current one.
template <int NH, class V>
struct Batch {
    static constexpr int K = (NH + kBlock - 1) / kBlock;
    V v[K];
};

template <int NH, class V, class Get>
__device__ __forceinline__ Batch<NH, V> load_batch(Get get) {
    Batch<NH, V> bt;
#pragma unroll
    for (int k = 0; k < Batch<NH, V>::K; ++k) bt.v[k] = get(min((int)threadIdx.x + k * kBlock, NH - 1));
    return bt;
}

template <int NH, class V, class Put>
__device__ __forceinline__ void put_batch(const Batch<NH, V>& bt, Put put) {
#pragma unroll
    for (int k = 0; k < Batch<NH, V>::K; ++k) put(threadIdx.x + k * kBlock, bt.v[k]);
}

template <int NH, class V, class Get, class Put>
__device__ __forceinline__ void stage_batched(Get get, Put put) {
    put_batch<NH, V>(load_batch<NH, V>(get), put);
}

// What an element outside the grid reads: zero (vectors, counts) or the
// solid label.  Never written; not const, so that they sit in the global
// address space like the arrays they stand in for and a select between the
// two stays a global (not a flat) load: flat loads share the LDS counter and
// would make every LDS wait also wait for the loads in flight.
__device__ uint64_t g_pad_zero[2] = {0, 0};
__device__ uint8_t g_pad_solid[8] = {kSolid, kSolid, kSolid, kSolid, kSolid, kSolid, kSolid, kSolid};

template <class V>
__device__ __forceinline__ const V* pad_zero() {
    return reinterpret_cast<const V*>(g_pad_zero);
}

// &p[q] inside the grid, else the pad.
template <class V>
__device__ __forceinline__ const V* at_or(const V* p, size_t q, bool in, const V* pad) {
    return in ? p + q : pad;
}

// Grid coordinates of element i of the one-cell haloed tile.
__device__ __forceinline__ void halo_coords(int i, TileOrigin o, int& x, int& y, int& z) {
    x = o.x0 + i % HX - 1;
    y = o.y0 + (i / HX) % HY - 1;
    z = o.z0 + i / (HX * HY) - 1;
}

// Global address (cell index, 0 when outside) of element i of the one-cell
// haloed tile, and whether it lies inside the grid.
struct HaloCell {
    size_t q;
    bool in;
};

__device__ __forceinline__ HaloCell halo_cell(Grid g, TileOrigin o, int i) {
    int x, y, z;
    halo_coords(i, o, x, y, z);
    const bool in = in_grid(g, z, y, x);
    return HaloCell{in ? cell_index(g, z, y, x) : 0, in};
}

// The image of a level at element i of the haloed tile.  Level 1: labels
// (outside the grid: solid).  Coarser levels: packed counts n_fluid |
// n_air << 16 (outside: 0, i.e. solid).
template <bool L1>
__device__ __forceinline__ uint32_t image_load(const void* img, Grid g, TileOrigin o, int i) {
    const HaloCell c = halo_cell(g, o, i);
    if constexpr (L1) return *at_or(static_cast<const uint8_t*>(img), c.q, c.in, g_pad_solid);
    else return *at_or(static_cast<const uint32_t*>(img), c.q, c.in, pad_zero<uint32_t>());
}

template <bool L1>
__device__ __forceinline__ void stage_image(uint32_t* img_s, const void* img, Grid g, TileOrigin o) {
    stage_batched<kHalo, uint32_t>([&](int i) { return image_load<L1>(img, g, o, i); },
                                   [&](int i, uint32_t v) { img_s[i] = v; });
}

// Runs body(tile, pre, prefetch) over the block's tiles, where pre holds the
// loads of the tile (load(tile), issued earlier) and prefetch() issues the
// loads of the block's next tile into pre: the body calls it once it has
// consumed pre and issued its own loads, so the next tile's memory latency
// overlaps the current tile's compute.  Everything the body reads from
// memory for the current tile must be issued before prefetch(): vector
// loads retire in order, so waiting for a later one waits for the prefetch.
// The solve's stop flag (stop->done) is read alongside the first tile's
// loads and tested once they are out (a test at the top of the kernel would
// put its memory latency in front of them); returns false when it stopped.
template <class Load, class Body>
__device__ __forceinline__ bool tile_pipeline(int ntiles, Load load, Body body, const State* stop) {
    const int done = stop->done;
    const TileSpan sp = tile_span(ntiles);
    if (sp.t0 >= sp.t1) return !done;
    auto pre = load(sp.t0);
    __asm__ volatile("" ::: "memory");   // the loads stay above the test
    if (done) return false;
    for (int tile = sp.t0; tile < sp.t1; tile += sp.step) {
        const int next = tile + sp.step;
        body(tile, pre, [&] {
            if (next < sp.t1) pre = load(next);
        });
    }
    return true;
}

template <bool L1>
__device__ __forceinline__ void counts_of(uint32_t v, uint32_t& n0, uint32_t& n1) {
    if (L1) {
        n0 = v == kFluid;
        n1 = v == kAir;
    } else {
        n0 = v & 0xffffu;
        n1 = v >> 16;
    }
}

// Window class of the cell at `base`: pure label c (0..2) when all 27 window
// cells are pure cells of label c, else -1.  any_fluid: a window cell holds fluid.
template <bool L1>
__device__ __forceinline__ int window_class(const uint32_t* img_s, int base, uint32_t full, bool& any_fluid) {
    int cls = -2;
    bool mixed = false;
    any_fluid = false;
#pragma unroll
    for (int o = 0; o < kTaps; ++o) {
        const uint32_t v = img_s[base + halo_off(o)];
        int c;
        if (L1) {
            c = (int)v;
            any_fluid |= (v == kFluid);
        } else {
            const uint32_t n0 = v & 0xffffu, n1 = v >> 16;
            any_fluid |= (n0 != 0u);
            c = n0 == full ? 0 : (n1 == full ? 1 : ((n0 | n1) == 0u ? 2 : -1));
        }
        mixed |= (c < 0) || (cls >= 0 && c != cls);
        cls = c;
    }
    return mixed ? -1 : cls;
}

// Wave-uniform choice of the CConv path: -3 every output of the wave is
// zero, 0..2 every window of the wave is pure label c (constant kernel),
// -1 general.
template <bool L1>
__device__ __forceinline__ int choose_mode(bool active, const uint32_t* img_s, int base, uint32_t full,
                                  bool zero_if_no_fluid, bool out_only_on_fluid) {
    bool any_fluid = false;
    int cls = -1;
    bool own_fluid = false;
    if (active) {
        cls = window_class<L1>(img_s, base, full, any_fluid);
        own_fluid = img_s[base] == (uint32_t)kFluid;
    }
    if (zero_if_no_fluid && __all(!active || !any_fluid)) return -3;
    if (out_only_on_fluid && __all(!active || !own_fluid)) return -3;
    const int c0 = __shfl(cls, 0, 64);
    if (__all(active && cls == c0 && cls >= 0)) return c0;
    return -1;
}

// The mode of the calling wave for tile `tile`: from the table formed at
// setup (k_wave_modes; the labels do not change during a solve) when given,
// else computed here.  Wave-uniform.
template <bool L1>
__device__ __forceinline__ int wave_mode(const int8_t* __restrict__ tab, int entry, bool active,
                                         const uint32_t* img_s, int base, uint32_t full, bool zero_if_no_fluid,
                                         bool out_only_on_fluid) {
    // in a scalar register, so that what the mode selects is read by scalar loads
    return __builtin_amdgcn_readfirstlane(
        tab ? entry : choose_mode<L1>(active, img_s, base, full, zero_if_no_fluid, out_only_on_fluid));
}

// The table entry of the wave's mode for a tile (0 without a table).  Read
// at the top of the tile, before the next tile's loads are issued: vector
// loads retire in order, so a load issued after them would wait for them.
// The tile's TZ = 4 entries are one aligned word, read with a scalar load
// (the tile index is uniform), so the mode lands in a scalar register and
// the pure-window weights it selects are scalar loads too.
__device__ __forceinline__ int wave_mode_entry(const int8_t* __restrict__ tab, int tile, int lz) {
    static_assert(TZ == 4, "one word of the mode table per tile");
    if (!tab) return 0;
    const uint32_t word = reinterpret_cast<const uint32_t*>(tab)[tile];
    return __builtin_amdgcn_readfirstlane((int)(int8_t)(word >> (8 * lz)));
}

// ---------------------------------------------------------------------------
// CConv evaluation of one output cell, per kernel-generation mode
// ---------------------------------------------------------------------------
// Vector ALU: K from the count form, then the 27-tap apply.
template <class T, bool L1>
__device__ __forceinline__ T cconv_vector(const uint32_t* img_s, const T* r_s, int base, const CConvW<T>* __restrict__ w) {
    T K[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) K[t] = w->C[t];
#pragma unroll
    for (int o = 0; o < kTaps; ++o) {
        uint32_t c0, c1;
        counts_of<L1>(img_s[base + halo_off(o)], c0, c1);
        const T n0 = (T)c0, n1 = (T)c1;
#pragma unroll
        for (int t = 0; t < kTaps; ++t) K[t] = fma(w->D[o][t][0], n0, fma(w->D[o][t][1], n1, K[t]));
    }
    T acc = T(0);
#pragma unroll
    for (int t = 0; t < kTaps; ++t) acc = fma(K[t], r_s[base + halo_off(t)], acc);
    return acc;
}

template <class T>
__device__ __forceinline__ T cconv_pure(const T* r_s, int base, const CConvW<T>* __restrict__ w, int c) {
    T acc = T(0);
#pragma unroll
    for (int t = 0; t < kTaps; ++t) acc = fma(w->Kpure[c][t], r_s[base + halo_off(t)], acc);
    return acc;
}

// Stored kernels: K[t][cell] formed at setup.  The 27 loads are issued
// together before the multiply-adds (one memory latency, not 27).
template <class T>
__device__ __forceinline__ T cconv_stored(const T* r_s, int base, const T (&kv)[kTaps]) {
    T acc = T(0);
#pragma unroll
    for (int t = 0; t < kTaps; ++t) acc = fma(kv[t], r_s[base + halo_off(t)], acc);
    return acc;
}

// The stored kernel of the thread's cell, loaded at the start of a tile so
// that its latency overlaps the staging instead of following it.  Done by
// the float kernels of levels >= 2 only: 27 doubles do not stay in
// registers beside the staging, nor 27 floats beside the level-1 staging
// (the others load it where the CConv needs it).
template <class T, int KM, bool COARSE>
constexpr bool kpre_on = KM == kStored && COARSE && sizeof(T) == 4;

template <class T, bool ON>
struct KPre {};
template <class T>
struct KPre<T, true> {
    T kv[kTaps];
};

template <class T, bool ON>
__device__ __forceinline__ KPre<T, ON> k_preload(const T* __restrict__ kst, size_t n, size_t idx) {
    KPre<T, ON> k;
    if constexpr (ON) {
#pragma unroll
        for (int t = 0; t < kTaps; ++t) k.kv[t] = kst[(size_t)t * n + idx];
    }
    return k;
}

__device__ __forceinline__ int halo_off_rt(int o) {   // runtime version of halo_off
    const int oz = o / 9, oy = (o / 3) - 3 * oz, ox = o - 3 * (o / 3);
    return (oz - 1) * HY * HX + (oy - 1) * HX + (ox - 1);
}

__host__ __device__ constexpr bool is_mfma(int km) { return km == kMfmaBf16x3 || km == kMfmaBf16 || km == kMfmaF16; }

// The two MFMA features of one window cell as one word, in the B-operand
// element order: the fluid count in the low half, the air count in the high
// half, each as bf16 (small integers: the top half of the fp32 pattern,
// exactly) or fp16.  Staged once per haloed tile cell.
template <int KM, bool L1>
__device__ __forceinline__ uint32_t feat_word(uint32_t v) {
    uint32_t c0, c1;
    counts_of<L1>(v, c0, c1);
    if constexpr (KM == kMfmaF16)
        return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)(float)c0) |
               ((uint32_t)__builtin_bit_cast(unsigned short, (_Float16)(float)c1) << 16);
    else
        return (__float_as_uint((float)c0) >> 16) | (__float_as_uint((float)c1) & 0xffff0000u);
}

// Feature pair 54/55 of the second feature step: the constant 1 (carrying
// C) and a zero.
template <int KM>
__device__ __forceinline__ uint32_t feat_one() {
    return KM == kMfmaF16 ? 0x3c00u : 0x3f80u;
}

// What a wave keeps for all its MFMA CConvs: the weight fragments (A
// operand), the haloed-tile index of its lane's cell in row 0, and the
// offsets of the lane's window positions 16 s + 4 g + j (s = feature step or
// tap block, g = lane / 16, j < 4; positions past 26 clamped, their A rows
// and columns are zero).  The same offsets address the features (window
// offset o) and the taps (tap t) because both run over the 27 positions in
// the same order.
template <int KM>
struct MfmaCtx {
    static constexpr int P = KM == kMfmaBf16x3 ? kPieces : 1;
    u16x8 a[P][2][2];
    int base0;
    int off[2][4];
    bool one;   // lane group 2: word 3 of step 1 is feature pair 54/55
};

template <int KM>
__device__ __forceinline__ MfmaCtx<KM> mfma_ctx(const MfmaW* __restrict__ wm, int lz) {
    MfmaCtx<KM> c;
    if constexpr (is_mfma(KM)) {
        const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
#pragma unroll
        for (int p = 0; p < MfmaCtx<KM>::P; ++p)
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const uint16_t* src = KM == kMfmaF16 ? &wm->f16[mb][ks][lane][0] : &wm->bf16[p][mb][ks][lane][0];
                    c.a[p][mb][ks] = *reinterpret_cast<const u16x8*>(src);
                }
        c.base0 = halo_base(n, 0, lz);
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int j = 0; j < 4; ++j) c.off[s2][j] = halo_off_rt(min(16 * s2 + 4 * g + j, kTaps - 1));
        c.one = g == 2;
    }
    return c;
}

// MFMA: one wave evaluates the CConv of its 64 cells (one z-plane of the
// tile, x = lane % 16, y = lane / 16) as four 16-cell groups.  For group q
// (y = q) the kernels of the 16 cells are K^T[tap][cell] = A[tap][feature] x
// B[feature][cell] on v_mfma_f32_16x16x32 (2 tap blocks x 2 feature steps,
// times the bf16 pieces); each lane then applies its 8 taps of one cell and
// the four lane groups are summed with two butterflies.  Returns the output
// of the lane's own cell.  All 64 lanes must call it.
template <int KM>
__device__ __forceinline__ float cconv_mfma(const uint32_t* feat_s, const float* r_s, const MfmaCtx<KM>& c) {
    constexpr int P = MfmaCtx<KM>::P;
    const int g = (threadIdx.x & 63) >> 4;
    float mine = 0.0f;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        const int bq = c.base0 + q * HX;
        uint32_t wv[2][4];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int j = 0; j < 4; ++j) wv[ks][j] = feat_s[bq + c.off[ks][j]];
        wv[1][3] = c.one ? feat_one<KM>() : wv[1][3];
        u16x8 B[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            B[ks] = __builtin_bit_cast(u16x8, (u32x4){wv[ks][0], wv[ks][1], wv[ks][2], wv[ks][3]});
        }
        f32x4 acc[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            acc[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    if (KM == kMfmaF16)
                        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, c.a[p][mb][ks]),
                                                                         __builtin_bit_cast(f16x8, B[ks]), acc[mb], 0, 0, 0);
                    else
                        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, c.a[p][mb][ks]),
                                                                          __builtin_bit_cast(bf16x8, B[ks]), acc[mb], 0, 0, 0);
                }
        }
        float part = 0.0f;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) part = fmaf(acc[mb][i], r_s[bq + c.off[mb][i]], part);
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        if (q == g) mine = part;
    }
    return mine;
}

// One CConv output of the thread's cell (lx, ly, lz) for a wave-uniform mode.
// kp: the preloaded stored kernel (PRE), else loaded here from kst.
template <class T, int KM, bool L1, bool PRE>
__device__ __forceinline__ T cconv_any(int mode, bool active, const uint32_t* img_s, const uint32_t* feat_s,
                                       const T* r_s, int base, const CConvW<T>* __restrict__ w,
                                       const MfmaCtx<KM>& mc, const T* __restrict__ kst, size_t n, size_t idx,
                                       const KPre<T, PRE>& kp) {
    if (mode == -3) return T(0);
    if (mode >= 0) return active ? cconv_pure<T>(r_s, base, w, mode) : T(0);
    if constexpr (KM == kStored) {
        if (!active) return T(0);
        if constexpr (PRE) {
            return cconv_stored<T>(r_s, base, kp.kv);
        } else {
            T kv[kTaps];
#pragma unroll
            for (int t = 0; t < kTaps; ++t) kv[t] = kst[(size_t)t * n + idx];
            return cconv_stored<T>(r_s, base, kv);
        }
    } else if constexpr (KM == kVector) {
        return active ? cconv_vector<T, L1>(img_s, r_s, base, w) : T(0);
    } else {
        static_assert(sizeof(T) == 4, "MFMA paths are float");
        return cconv_mfma<KM>(feat_s, reinterpret_cast<const float*>(r_s), mc);
    }
}

// The mixed-BC 7-point matrix applied at `base` of a staged tile with row
// stride (sx, sy): diagonal = fluid or air face neighbours (out of grid is
// solid), -1 per fluid face neighbour, zero on non-fluid rows (Sec.
// "Spatial Discretization").
// sx: stride of y, sz: stride of z; Acc: accumulation type.
template <class Acc, class V, class L>
__device__ __forceinline__ Acc apply_A(const L* lab_s, const V* v_s, int base, int sx, int sz) {
    if (lab_s[base] != kFluid) return Acc(0);
    const int nb[6] = {-sz, sz, -sx, sx, -1, 1};
    int cnt = 0;
    Acc s = Acc(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const uint32_t l = lab_s[base + nb[k]];
        cnt += (l != (uint32_t)kSolid);
        if (l == (uint32_t)kFluid) s += (Acc)v_s[base + nb[k]];
    }
    return (Acc)cnt * (Acc)v_s[base] - s;
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
__global__ void k_state_init(State* st, int max_iter, int fixed, int n_ortho, int method, int sym) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        State s = {};
        s.max_iter = max_iter;
        s.fixed = fixed;
        s.n_ortho = n_ortho;
        s.method = method;
        s.sym = sym;
        s.scale = 1.0;
        *st = s;
    }
}

// Validate labels and b, count fluid cells, ||b||^2, x0 = 0.
template <class X>
__global__ __launch_bounds__(kBlock) void k_scan(const uint8_t* __restrict__ lab, const double* __restrict__ b,
                                                 size_t n, X* x, double* partials) {
    double v[kRedWidth] = {0.0, 0.0, 0.0, 0.0};   // bb, n_fluid, bad labels, non-finite
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        const uint8_t l = lab[i];
        const double bv = b[i];   // read with the label (used on fluid cells only)
        if (l > kSolid) v[2] += 1.0;
        if (l == kFluid) {
            v[1] += 1.0;
            if (!isfinite(bv)) v[3] += 1.0;
            else v[0] += bv * bv;
        }
        x[i] = X(0);
    }
    block_partials<kBlock>(v, partials);
}

// Counts of level l+1 from level l: sums of the 2x2x2 children.
template <bool FROM_LABELS>
__global__ __launch_bounds__(kBlock) void k_pool_counts(const void* __restrict__ in, Grid gin,
                                                        uint32_t* __restrict__ out, Grid gout) {
    const size_t n = ncells(gout);
    for (size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (size_t)gridDim.x * kBlock) {
        const int x = (int)(q % gout.nx), y = (int)((q / gout.nx) % gout.ny), z = (int)(q / ((size_t)gout.nx * gout.ny));
        uint32_t n0 = 0, n1 = 0;
        for (int k = 0; k < 8; ++k) {
            const size_t c = cell_index(gin, 2 * z + (k >> 2), 2 * y + ((k >> 1) & 1), 2 * x + (k & 1));
            if (FROM_LABELS) {
                const uint8_t l = static_cast<const uint8_t*>(in)[c];
                n0 += l == kFluid;
                n1 += l == kAir;
            } else {
                const uint32_t v = static_cast<const uint32_t*>(in)[c];
                n0 += v & 0xffffu;
                n1 += v >> 16;
            }
        }
        out[q] = n0 | (n1 << 16);
    }
}

// The image-window sums of Aff_1^l and Aff_2^l (global means), in double:
// S = sum_p sum_o sum_c w[c][o] i_c(p + o), the image solid outside the grid.
// With q = p + o the in-grid part is sum_q sum_c i_c(q) W_c(q), where
// W_c(q) = sum of w[c][o] over the o with q - o in the grid (all 27 for an
// interior cell), so each cell is read once; the out-of-grid part is
// sum_o w[solid][o] (n - #{p : p + o in the grid}), with that count the
// product over the axes of (N_a - |o_a|), added by one thread.
template <bool L1>
__global__ __launch_bounds__(kBlock) void k_aff(const void* __restrict__ img, Grid g, double inv_full,
                                                const AffW* __restrict__ a1, const AffW* __restrict__ a2,
                                                double* partials) {
    const size_t n = ncells(g);
    double v[kRedWidth] = {0.0, 0.0, 0.0, 0.0};
    __shared__ double full_s[6];   // W_c of an interior cell, for Aff_1 and Aff_2
    if (threadIdx.x < 6) {
        const AffW* a = threadIdx.x < 3 ? a1 : a2;
        double t = 0.0;
        for (int o = 0; o < kTaps; ++o) t += a->w[threadIdx.x % 3][o];
        full_s[threadIdx.x] = t;
    }
    __syncthreads();
    const double full1[3] = {full_s[0], full_s[1], full_s[2]}, full2[3] = {full_s[3], full_s[4], full_s[5]};
    for (size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (size_t)gridDim.x * kBlock) {
        const int x = (int)(p % g.nx), y = (int)((p / g.nx) % g.ny), z = (int)(p / ((size_t)g.nx * g.ny));
        double i0, i1;
        if (L1) {
            const uint8_t l = static_cast<const uint8_t*>(img)[p];
            i0 = l == kFluid;
            i1 = l == kAir;
        } else {
            const uint32_t c = static_cast<const uint32_t*>(img)[p];
            i0 = (double)(c & 0xffffu) * inv_full;
            i1 = (double)(c >> 16) * inv_full;
        }
        const double i2 = 1.0 - i0 - i1;
        double W1[3] = {full1[0], full1[1], full1[2]}, W2[3] = {full2[0], full2[1], full2[2]};
        const bool interior = x >= 1 && y >= 1 && z >= 1 && x + 1 < g.nx && y + 1 < g.ny && z + 1 < g.nz;
        if (!interior) {
            for (int c = 0; c < 3; ++c) W1[c] = W2[c] = 0.0;
            for (int o = 0; o < kTaps; ++o) {
                if (!in_grid(g, z - (o / 9 - 1), y - ((o / 3) % 3 - 1), x - (o % 3 - 1))) continue;
                for (int c = 0; c < 3; ++c) {
                    W1[c] += a1->w[c][o];
                    W2[c] += a2->w[c][o];
                }
            }
        }
        v[0] += i0 * W1[0] + i1 * W1[1] + i2 * W1[2];
        v[1] += i0 * W2[0] + i1 * W2[1] + i2 * W2[2];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {   // the solid padding
        for (int o = 0; o < kTaps; ++o) {
            const double in = (double)max(g.nz - abs(o / 9 - 1), 0) * (double)max(g.ny - abs((o / 3) % 3 - 1), 0) *
                              (double)max(g.nx - abs(o % 3 - 1), 0);
            v[0] += a1->w[2][o] * ((double)n - in);
            v[1] += a2->w[2][o] * ((double)n - in);
        }
    }
    block_partials<kBlock>(v, partials);
}

// K[t][cell] of one CConv block on one level, formed in double (setup).
template <class T, bool L1, int TG>
__global__ __launch_bounds__(kBlock) void k_kgen_store(const void* __restrict__ img, Grid g,
                                                       const CConvW<double>* __restrict__ w, T* __restrict__ kst) {
    // one thread per (group j of TG taps, cell p), i = j n + p: the taps of a
    // block share their weights (uniform loads), the stores are contiguous;
    // each tap sums its 27 window terms in window order.  TG = 1 spreads a
    // small level over many threads; TG = 27 reads each window once on a
    // large one (27 taps per thread would re-read it 27 times)
    static_assert(kTaps % TG == 0, "whole tap groups");
    const size_t n = ncells(g);
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < (size_t)(kTaps / TG) * n;
         i += (size_t)gridDim.x * kBlock) {
        const int t0 = (int)(i / n) * TG;
        const size_t p = i - (size_t)(t0 / TG) * n;
        const int x = (int)(p % g.nx), y = (int)((p / g.nx) % g.ny), z = (int)(p / ((size_t)g.nx * g.ny));
        double K[TG];
#pragma unroll
        for (int u = 0; u < TG; ++u) K[u] = w->C[t0 + u];
        // the window loop is unrolled for one tap; with all 27 it stays a loop
        // (27 x 27 unrolled terms would not fit the instruction cache)
        constexpr int UO = TG == 1 ? kTaps : 1;
#pragma unroll UO
        for (int o = 0; o < kTaps; ++o) {
            // solid padding (no fluid, no air) outside the grid: the cell itself is
            // read there and its weights zeroed, so the 27 reads are unconditional
            const int qz = z + o / 9 - 1, qy = y + (o / 3) % 3 - 1, qx = x + o % 3 - 1;
            const bool in = in_grid(g, qz, qy, qx);
            const size_t q = in ? cell_index(g, qz, qy, qx) : p;
            const uint32_t v = L1 ? (uint32_t)static_cast<const uint8_t*>(img)[q] : static_cast<const uint32_t*>(img)[q];
            uint32_t c0, c1;
            counts_of<L1>(v, c0, c1);
            const double m = in ? 1.0 : 0.0;
#pragma unroll
            for (int u = 0; u < TG; ++u)
                K[u] += (w->D[o][t0 + u][0] * m) * (double)c0 + (w->D[o][t0 + u][1] * m) * (double)c1;
        }
#pragma unroll
        for (int u = 0; u < TG; ++u) kst[(size_t)(t0 + u) * n + p] = (T)K[u];
    }
}

// K[t][cell] of one CConv block on a large level (training and the symmetric
// variant store every level), formed on matrix cores: per 16-cell group along
// x, K^T[tap][cell] = A[tap][feature] B[feature][cell] as in the solve's
// kernels (KM = kMfmaBf16x3: three bf16 pieces, the FP32 bar; kMfmaBf16: one
// piece, the bf16 training leg), B from the 27 window cells' counts (exact in
// bf16 up to level 3; solid outside the grid).  Lane (g, n) holds taps
// 16 mb + 4 g + j of cell n and stores them, 16 consecutive cells per tap.
template <int KM, bool L1>
__global__ __launch_bounds__(kBlock) void k_kgen_store_mfma(const void* __restrict__ img, Grid g,
                                                            const MfmaW* __restrict__ wm, float* __restrict__ kst) {
    constexpr int P = KM == kMfmaBf16x3 ? kPieces : 1;
    const int lane = threadIdx.x & 63, gl = lane >> 4, n = lane & 15;
    u16x8 a[P][2][2];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) a[p][mb][ks] = *reinterpret_cast<const u16x8*>(&wm->bf16[p][mb][ks][lane][0]);
    const size_t ncell = ncells(g);
    const int nxg = (g.nx + 15) / 16;
    const size_t ngroups = (size_t)g.nz * g.ny * nxg;
    const int waves = (int)(gridDim.x * (kBlock / 64));
    for (size_t grp = (size_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); grp < ngroups; grp += waves) {
        const int xb = (int)(grp % nxg), y = (int)((grp / nxg) % g.ny), z = (int)(grp / ((size_t)nxg * g.ny));
        const int x = 16 * xb + n;
        const bool valid = x < g.nx;
        uint32_t fw[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {   // window position 16 (j / 4) + 4 g + j % 4 (past 26: zero A rows and columns)
            const int o = min(16 * (j >> 2) + 4 * gl + (j & 3), kTaps - 1);
            const int qz = z + o / 9 - 1, qy = y + (o / 3) % 3 - 1, qx = x + o % 3 - 1;
            const bool in = valid && in_grid(g, qz, qy, qx);
            const size_t q = in ? cell_index(g, qz, qy, qx) : 0;
            const uint32_t v = L1 ? (uint32_t)*at_or(static_cast<const uint8_t*>(img), q, in, g_pad_solid)
                                  : (in ? static_cast<const uint32_t*>(img)[q] : 0u);
            fw[j] = feat_word<KM, L1>(v);
        }
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u16x8 B0 = __builtin_bit_cast(u16x8, (u32x4){fw[0], fw[1], fw[2], fw[3]});
        const u16x8 B1 = __builtin_bit_cast(u16x8, (u32x4){fw[4], fw[5], fw[6], gl == 2 ? feat_one<KM>() : fw[7]});
        f32x4 acc[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            acc[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int p = 0; p < P; ++p) {
                acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[p][mb][0]),
                                                                  __builtin_bit_cast(bf16x8, B0), acc[mb], 0, 0, 0);
                acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[p][mb][1]),
                                                                  __builtin_bit_cast(bf16x8, B1), acc[mb], 0, 0, 0);
            }
        }
        if (valid) {
            const size_t cell = ((size_t)z * g.ny + y) * g.nx + x;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int t = 16 * mb + 4 * gl + j;
                    if (t < kTaps) kst[(size_t)t * ncell + cell] = acc[mb][j];
                }
        }
    }
}

// ---------------------------------------------------------------------------
// the one-block control kernel
// ---------------------------------------------------------------------------
// Sums nparts per-block partials (structure of arrays, block order: a fixed
// summation order) and updates the state for one stage of the iteration.
// The stopping decision is mirrored to host memory (hf) for the host loop.
// Per-wave CConv modes of one level (see choose_mode), one byte per (tile,
// z-plane of the tile).  Level 1: m_down for the down kernel (zero where no
// window of the wave holds fluid), m_up for the up kernel (zero where the
// wave has no fluid cell).  Coarser levels: pure-window classes in m_down.
template <bool L1>
__global__ __launch_bounds__(kBlock) void k_wave_modes(const void* __restrict__ img, Grid g, uint32_t full,
                                                       int8_t* __restrict__ m_down, int8_t* __restrict__ m_up) {
    __shared__ uint32_t img_s[kHaloP];
    const Tiles tl = tiles_of(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    for (TileSpan sp = tile_span(tl.count()); sp.t0 < sp.t1; sp.t0 += sp.step) {
        const int tile = sp.t0;
        const TileOrigin o = tile_origin(tile, tl);
        __syncthreads();
        stage_image<L1>(img_s, img, g, o);
        __syncthreads();
        const bool active = in_grid(g, o.z0 + lz, o.y0 + ly, o.x0 + lx);
        const int md = choose_mode<L1>(active, img_s, base, full, L1, false);
        const int mu = L1 ? choose_mode<L1>(active, img_s, base, full, false, true) : md;
        if ((threadIdx.x & 63) == 0) {
            m_down[tile * TZ + lz] = (int8_t)md;
            if (L1) m_up[tile * TZ + lz] = (int8_t)mu;
        }
    }
}

// Rows of partials each stage sums.
template <int STAGE>
constexpr int ctl_width() {
    return STAGE == kStageScan ? 4 : STAGE == kStageAff ? 2 : STAGE == kStageResidual ? 1
         : STAGE == kStageDots ? kMaxOrtho : STAGE == kStageLoss ? 1 : 2;
}

// Partial sums (sum_partials below) in two parts: head_partials issues the
// first round of loads (partials b < kSumU NT, every row w < W, which must lie
// inside the buffer) ahead of other work, finish_partials adds them and the
// rest.  Every thread of the block calls both.
constexpr int kSumU = 4;

template <int W, int NT>
__device__ __forceinline__ void head_partials(const double* __restrict__ partials, int nparts,
                                              double (&t)[W][kSumU]) {
#pragma unroll
    for (int u = 0; u < kSumU; ++u) {
        const int b = u * NT + (int)threadIdx.x;
#pragma unroll
        for (int w = 0; w < W; ++w) t[w][u] = b < nparts ? partials[(size_t)w * kMaxRedBlocks + b] : 0.0;
    }
}

template <int W, int NT>
__device__ __forceinline__ void finish_partials(const double (&t0)[W][kSumU], const double* __restrict__ partials,
                                                int nparts, int rows, double (&v)[W]) {
    constexpr int U = kSumU;
    __shared__ double sh[W][NT / 64];
#pragma unroll
    for (int w = 0; w < W; ++w) v[w] = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int w = 0; w < W; ++w) v[w] += w < rows ? t0[w][u] : 0.0;
    for (int b0 = U * NT; b0 < nparts; b0 += U * NT) {
        double t[W][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * NT + (int)threadIdx.x;
#pragma unroll
            for (int w = 0; w < W; ++w) t[w][u] = w < rows && b < nparts ? partials[(size_t)w * kMaxRedBlocks + b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] += t[w][u];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int w = 0; w < W; ++w) v[w] = wave_sum(v[w]);
    if (lane == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) sh[w][wid] = v[w];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < NT / 64; ++i) t += sh[w][i];
            v[w] = t;
        }
    }
}

// Sum of rows w < rows (of W) of nparts per-block partials (structure of
// arrays, block order, a fixed reduction tree for a given NT), left in v of
// thread 0 of a block of NT threads.  Every thread must call it.
// Each thread issues kSumU partials per row before adding any: one memory
// latency per kSumU NT partials (a load-add loop would wait for every load in
// turn).
template <int W, int NT>
__device__ __forceinline__ void sum_partials(const double* __restrict__ partials, int nparts, int rows, double (&v)[W]) {
    double t[W][kSumU];
    head_partials<W, NT>(partials, nparts, t);
    finish_partials<W, NT>(t, partials, nparts, rows, v);
}

// The state the Dots stage reads (sl: ring slots of d_(k-1), d_(k-2), ...),
// gathered in one go so that its loads can go out early.
struct DotsIn {
    int method, nprev;
    double dAd[kMaxOrtho];
    double rho_prev;
};

__device__ __forceinline__ DotsIn dots_in(const State* st, const int (&sl)[kMaxOrtho]) {
    DotsIn d;
    d.method = st->method;
    d.nprev = st->nprev;
#pragma unroll
    for (int j = 0; j < kMaxOrtho; ++j) d.dAd[j] = st->dAd[sl[j]];
    d.rho_prev = st->rho_prev;
    return d;
}

// The Dots stage: the coefficients beta_j of the direction update from the
// summed dots v (and, for the PCG forms, rho = r . d^), formed without
// writing the state.
__device__ __forceinline__ void dots_betas(const DotsIn& in, const double* v, double (&beta)[kMaxOrtho], double& rho) {
    rho = 0.0;
    if (in.method == 0) {
#pragma unroll
        for (int j = 0; j < kMaxOrtho; ++j) beta[j] = j < in.nprev ? v[j] / in.dAd[j] : 0.0;
    } else {
        // With s = P(r) = ||r|| d^ and directions kept scaled by 1/||r||,
        // d^_k + c d^_(k-1) is parallel to s_k + beta d_(k-1) for
        // c = beta ||r_(k-1)|| / ||r_k||: PCG c = rho_k / rho_(k-1),
        // flexible PCG c = (rho_k - d^_k . r_(k-1)) / rho_(k-1), rho = r . d^.
        rho = v[0];
        const double num = in.method == 1 ? rho : rho - v[1];
        beta[0] = in.nprev > 0 ? -num / in.rho_prev : 0.0;
        for (int j = 1; j < kMaxOrtho; ++j) beta[j] = 0.0;
    }
}

// The iteration count and stop flag, mirrored to pinned (fine-grained, not
// L2-cached) host memory for the host loop, which only paces its enqueueing
// by them: plain stores, no fence (a system-scope fence would write back the
// whole L2).  The stream order, not these flags, orders the final state.
__device__ __forceinline__ void host_flags(HostFlags* hf, int iter, int done) {
    volatile HostFlags* h = hf;
    h->iter = iter;
    h->done = done;
}

// The Step stage from d . A d and r . d: the step length (NPSDO: exact line
// search; PCG forms: alpha = r . s / d . A d), or a breakdown when d . A d is
// not positive or a dot is not finite.  step_alpha forms it without writing
// the state; step_update also records it (i0: ring slot of the direction).
struct StepIn {
    int method;
    double rho;
};

__device__ __forceinline__ StepIn step_in(const State* st) { return StepIn{st->method, st->rho}; }

__device__ __forceinline__ bool step_alpha(const StepIn& in, double dAd, double rd, double& alpha) {
    if (!(dAd > 0.0) || !isfinite(dAd) || !isfinite(rd)) return false;
    alpha = (in.method == 0 ? rd : in.rho) / dAd;
    return true;
}

__device__ __forceinline__ void step_update(State* st, const StepIn& in, int i0, double dAd, double rd,
                                            HostFlags* hf) {
    double alpha;
    st->dAd[i0] = dAd;
    st->rd = rd;
    if (!step_alpha(in, dAd, rd, alpha)) {
        st->done = 1;
        st->status = -6;   // NPS_EBREAKDOWN
        if (hf) host_flags(hf, st->iter, 1);
    } else {
        st->alpha = alpha;
        st->rho_prev = in.rho;
        st->pending = 1;
    }
}

// The state the Residual stage reads, gathered in one go so that its loads
// can go out early.
struct ResidualIn {
    int iter, pending, xcur, n_ortho, method, fixed, max_iter;
    double tol2bb;
};

__device__ __forceinline__ ResidualIn residual_in(const State* st) {
    return ResidualIn{st->iter, st->pending, st->xcur, st->n_ortho, st->method, st->fixed, st->max_iter, st->tol2bb};
}

// The Residual stage from rr = ||b - A x_k||^2 of the iterate down_l1 just
// formed: the iteration count, 1/||r||, the dot count and the convergence
// test; returns the stop flag.
__device__ __forceinline__ int residual_stage(State* st, const ResidualIn& in, double rr, HostFlags* hf) {
    const int iter = in.iter + (in.pending ? 1 : 0);
    st->iter = iter;
    st->xcur = in.xcur ^ 1;   // the residual kernel wrote the other solution buffer
    st->pending = 0;
    st->rr = rr;
    st->scale = rr > 0.0 ? 1.0 / sqrt(rr) : 0.0;
    const int nprev = min(iter, in.n_ortho);
    st->nprev = nprev;
    // NPSDO: d^ . A d_i per previous direction; PCG: r . d^; flexible PCG
    // also d^ . r_(k-1)
    st->ndots = in.method == 0 ? nprev : in.method == 1 ? 1 : 2;
    int done = 0, status = 0;
    if (!isfinite(rr)) {
        done = 1;
        status = -6;   // NPS_EBREAKDOWN
    } else if (!in.fixed && rr < in.tol2bb) {
        done = 1;
        status = 0;
    } else if (iter >= in.max_iter) {
        done = 1;
        status = in.fixed ? 0 : 1;   // NPS_OK / NPS_NOT_CONVERGED
    }
    if (done) {
        st->done = 1;
        st->status = status;
    }
    if (hf) host_flags(hf, iter, done);
    return done;
}

// The state update of one stage from its summed partials v (one thread).
// The stopping decision is mirrored to host memory (hf) for the host loop.
// The Dots stage may run in every block of a kernel at once (each with the
// same sums): it reads no field it writes.
template <int STAGE>
__device__ __forceinline__ void control_update(State* st, const double* v, int i0, int i1, int i2, int i3, double d0,
                                               double d1, double d2, HostFlags* hf) {
    if constexpr (STAGE == kStageScan) {            // d0 = tol
        st->bb = v[0];
        st->n_fluid = (int)v[1];
        st->bad_label = (int)v[2];
        st->nonfinite = (int)v[3];
        st->tol2bb = d0 * d0 * v[0];
    } else if constexpr (STAGE == kStageAff) {      // i0 = level index, d0/d1 = Aff biases, d2 = 27 n_l
        st->c1[i0] = d0 + v[0] / d2;
        st->c2[i0] = d1 + v[1] / d2;
    } else if constexpr (STAGE == kStageResidual) { // ||b - A x_k||^2 of the iterate down_l1 just formed
        residual_stage(st, residual_in(st), v[0], hf);
    } else if constexpr (STAGE == kStageDots) {     // i0..i3: ring slots of d_(k-1), d_(k-2), ...
        const int sl[kMaxOrtho] = {i0, i1, i2, i3};
        double beta[kMaxOrtho], rho;
        dots_betas(dots_in(st, sl), v, beta, rho);
        for (int j = 0; j < kMaxOrtho; ++j) st->beta[j] = beta[j];
        if (st->method != 0) st->rho = rho;
    } else if constexpr (STAGE == kStageLoss) {     // training loss: ||b - A y||^2
        st->rr = v[0];
    } else if constexpr (STAGE == kStageStep) {     // i0: ring slot of the new direction
        step_update(st, step_in(st), i0, v[0], v[1], hf);
    }
}

// The one-block control kernel: sums nparts per-block partials and updates
// the state for one stage of the iteration.
template <int STAGE>
__global__ __launch_bounds__(kCtlBlock) void k_control(State* st, const double* __restrict__ partials, int nparts,
                                                       int i0, int i1, int i2, int i3, double d0, double d1,
                                                       double d2, HostFlags* hf) {
    // the stop flag is read alongside the partials and tested after them
    const int done = STAGE == kStageResidual || STAGE == kStageDots || STAGE == kStageStep ? st->done : 0;
    constexpr int W = ctl_width<STAGE>();
    double v[W];
    sum_partials<W, kCtlBlock>(partials, nparts, W, v);
    if (done) return;
    if (threadIdx.x == 0) control_update<STAGE>(st, v, i0, i1, i2, i3, d0, d1, d2, hf);
}

// ---------------------------------------------------------------------------
// network kernels (Alg. 2)
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void pool_tile_to(const T* out_s, TileOrigin o, Grid g, T* rnext) {
    if (threadIdx.x < kBlock / 8) {
        const int cx = threadIdx.x % (TX / 2), cy = (threadIdx.x / (TX / 2)) % (TY / 2),
                  cz = threadIdx.x / ((TX / 2) * (TY / 2));
        const Grid gc = coarser(g);
        const int gx = o.x0 / 2 + cx, gy = o.y0 / 2 + cy, gz = o.z0 / 2 + cz;
        if (gx < gc.nx && gy < gc.ny && gz < gc.nz) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int fx = 2 * cx + (k & 1), fy = 2 * cy + ((k >> 1) & 1), fz = 2 * cz + (k >> 2);
                s += out_s[(fz * TY + fy) * TX + fx];
            }
            rnext[cell_index(gc, gz, gy, gx)] = s * T(0.125);
        }
    }
}

// Level 1 of the down sweep: x1 = CConv_1^1(r) and r^2 = Pool(x1), with r
// the network input (masked to fluid: the solve's residual is zero off
// fluid already, nps_apply_precond's input need not be).
template <class X, class T>
struct XDL {   // x, the pending direction and the label of one staged cell
    X x;
    T d;
    uint8_t l;
};

template <class T>
struct RL {    // network input and label of one haloed cell
    T r;
    uint8_t l;
};

template <class T, int KM>
__global__ __launch_bounds__(kBlock) NPS_WAVES_PER_EU(3) void k_down_l1(
    const uint8_t* __restrict__ lab, Grid g, const T* __restrict__ r, T* __restrict__ x1, T* __restrict__ rnext,
    const CConvW<T>* __restrict__ w, const MfmaW* __restrict__ wm, const T* __restrict__ kst, const State* st,
    const int8_t* __restrict__ wmode) {
    __shared__ uint32_t img_s[kHaloP];
    __shared__ uint32_t feat_s[is_mfma(KM) ? kHaloP : 1];
    __shared__ T r_s[kHaloP];
    __shared__ T out_s[kBlock];
    const Tiles tl = tiles_of(g);
    const size_t n = ncells(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    const MfmaCtx<KM> mc = mfma_ctx<KM>(wm, lz);
    auto load = [&](int tile) {
        const TileOrigin o = tile_origin(tile, tl);
        return load_batch<kHalo, RL<T>>([&](int i) {
            const HaloCell c = halo_cell(g, o, i);
            return RL<T>{*at_or(r, c.q, c.in, pad_zero<T>()), *at_or(lab, c.q, c.in, g_pad_solid)};
        });
    };
    tile_pipeline(tl.count(), load, [&](int tile, const auto& pre, auto prefetch) {
        const TileOrigin o = tile_origin(tile, tl);
        const int wm_e = wave_mode_entry(wmode, tile, lz);
        const int xx = o.x0 + lx, yy = o.y0 + ly, zz = o.z0 + lz;
        const bool active = in_grid(g, zz, yy, xx);
        const size_t idx = active ? cell_index(g, zz, yy, xx) : 0;
        __syncthreads();
        put_batch(pre, [&](int i, RL<T> e) {
            r_s[i] = e.l == kFluid ? e.r : T(0);
            img_s[i] = e.l;
            if constexpr (is_mfma(KM)) feat_s[i] = feat_word<KM, true>(e.l);
        });
        prefetch();
        __syncthreads();
        const int mode = wave_mode<true>(wmode, wm_e, active, img_s, base, 1u, true, false);
        const T out = cconv_any<T, KM, true>(mode, active, img_s, feat_s, r_s, base, w, mc, kst, n, idx,
                                             KPre<T, false>{});
        if (active) x1[idx] = out;
        out_s[threadIdx.x] = active ? out : T(0);
        __syncthreads();
        pool_tile_to<T>(out_s, o, g, rnext);
    }, st);
}

// x1 = CConv_1(r, I) on one level l >= 2, and (POOL) r_next = Pool(x1).
template <class T>
struct CR {    // packed counts and network input of one haloed cell
    uint32_t c;
    T r;
};

template <class T, int KM, bool POOL>
__global__ __launch_bounds__(kBlock) NPS_WAVES_PER_EU(waves_floor(KM)) void k_down(
    const uint32_t* __restrict__ cnt, Grid g, uint32_t full, const T* __restrict__ rin, T* __restrict__ x1,
    T* __restrict__ rnext, const CConvW<T>* __restrict__ w, const MfmaW* __restrict__ wm, const T* __restrict__ kst,
    const State* st, const int8_t* __restrict__ wmode) {
    __shared__ uint32_t img_s[kHaloP];
    __shared__ uint32_t feat_s[is_mfma(KM) ? kHaloP : 1];
    __shared__ T r_s[kHaloP];
    __shared__ T out_s[kBlock];
    const Tiles tl = tiles_of(g);
    const size_t n = ncells(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    const MfmaCtx<KM> mc = mfma_ctx<KM>(wm, lz);
    auto load = [&](int tile) {
        const TileOrigin o = tile_origin(tile, tl);
        return load_batch<kHalo, CR<T>>([&](int i) {
            const HaloCell c = halo_cell(g, o, i);
            return CR<T>{*at_or(cnt, c.q, c.in, pad_zero<uint32_t>()), *at_or(rin, c.q, c.in, pad_zero<T>())};
        });
    };
    tile_pipeline(tl.count(), load, [&](int tile, const auto& pre, auto prefetch) {
        const TileOrigin o = tile_origin(tile, tl);
        const int wm_e = wave_mode_entry(wmode, tile, lz);
        const int xx = o.x0 + lx, yy = o.y0 + ly, zz = o.z0 + lz;
        const bool active = in_grid(g, zz, yy, xx);
        const size_t idx = active ? cell_index(g, zz, yy, xx) : 0;
        const auto kp = k_preload<T, kpre_on<T, KM, true>>(kst, n, idx);
        __syncthreads();
        put_batch(pre, [&](int i, CR<T> e) {
            img_s[i] = e.c;
            if constexpr (is_mfma(KM)) feat_s[i] = feat_word<KM, false>(e.c);
            r_s[i] = e.r;
        });
        prefetch();
        __syncthreads();
        const int mode = KM == kStored ? -1 : wave_mode<false>(wmode, wm_e, active, img_s, base, full, false, false);
        const T out = cconv_any<T, KM, false>(mode, active, img_s, feat_s, r_s, base, w, mc, kst, n, idx, kp);
        if (active) x1[idx] = out;
        if (POOL) {
            out_s[threadIdx.x] = active ? out : T(0);
            __syncthreads();
            pool_tile_to<T>(out_s, o, g, rnext);
        }
    }, st);
}

// Linear 2x upsampling weights along one axis (cell-centred, edges clamped):
// fine f -> coarse j = f/2 (weight 3/4) and its neighbour on f's side (1/4).
__device__ __forceinline__ void up_axis(int f, int nc, int& j, int& jn) {
    j = f >> 1;
    jn = (f & 1) ? min(j + 1, nc - 1) : max(j - 1, 0);
}

template <class T>
__device__ __forceinline__ T interp_at(const T* __restrict__ xc, Grid gc, int z, int y, int x) {
    int jx, jxn, jy, jyn, jz, jzn;
    up_axis(x, gc.nx, jx, jxn);
    up_axis(y, gc.ny, jy, jyn);
    up_axis(z, gc.nz, jz, jzn);
    const T a = T(0.75), b = T(0.25);
    const T p00 = a * xc[cell_index(gc, jz, jy, jx)] + b * xc[cell_index(gc, jz, jy, jxn)];
    const T p01 = a * xc[cell_index(gc, jz, jyn, jx)] + b * xc[cell_index(gc, jz, jyn, jxn)];
    const T p10 = a * xc[cell_index(gc, jzn, jy, jx)] + b * xc[cell_index(gc, jzn, jy, jxn)];
    const T p11 = a * xc[cell_index(gc, jzn, jyn, jx)] + b * xc[cell_index(gc, jzn, jyn, jxn)];
    return a * (a * p00 + b * p01) + b * (a * p10 + b * p11);
}

// Stage Interp(xc) over the haloed tile (zero outside the level's grid: the
// zero padding of the CConv input).  The coarse cells the tile needs, a
// CX x CY x CZ block starting two coarse cells before the tile, are first
// staged in LDS with their coordinates clamped into the coarse grid, which is
// exactly the interpolation's edge rule, so the fine values are formed from
// LDS without further clamping.
constexpr int CXS = TX / 2 + 4, CYS = TY / 2 + 4, CZS = TZ / 2 + 4;
constexpr int kCoarseTile = CXS * CYS * CZS;
constexpr int kCoarseTileP = pad_block(kCoarseTile);

template <class T>
struct UpLoads {
    Batch<kHalo, uint32_t> img;       // image over the haloed tile
    Batch<kCoarseTile, T> c;          // the coarse cells the tile interpolates from
};

template <bool L1, class T>
__device__ __forceinline__ UpLoads<T> load_image_interp(const void* img, const T* __restrict__ xc, Grid g,
                                                        TileOrigin o) {
    const Grid gc = coarser(g);
    const int bx = o.x0 / 2 - 2, by = o.y0 / 2 - 2, bz = o.z0 / 2 - 2;
    UpLoads<T> u;
    u.img = load_batch<kHalo, uint32_t>([&](int i) { return image_load<L1>(img, g, o, i); });
    u.c = load_batch<kCoarseTile, T>([&](int i) {
        const int cx = i % CXS, cy = (i / CXS) % CYS, cz = i / (CXS * CYS);
        const int jx = min(max(bx + cx, 0), gc.nx - 1), jy = min(max(by + cy, 0), gc.ny - 1),
                  jz = min(max(bz + cz, 0), gc.nz - 1);
        return xc[cell_index(gc, jz, jy, jx)];
    });
    return u;
}

template <bool L1, int KM, class T>
__device__ __forceinline__ void put_image_interp(const UpLoads<T>& u, uint32_t* img_s, uint32_t* feat_s, T* c_s) {
    put_batch(u.img, [&](int i, uint32_t v) {
        img_s[i] = v;
        if constexpr (is_mfma(KM)) feat_s[i] = feat_word<KM, L1>(v);
    });
    put_batch(u.c, [&](int i, T v) { c_s[i] = v; });
}

// Interp(xc) over the haloed tile from the staged coarse cells (zero
// outside the level's grid: the zero padding of the CConv input).  The
// coarse block starts two coarse cells before the tile and its coordinates
// were clamped into the coarse grid, which is exactly the interpolation's
// edge rule, so no further clamping is needed here.
//
// Fine cell f (along one axis) lies between coarse cells f >> 1 (weight
// 3/4) and its neighbour on f's side (weight 1/4): the pair (f >> 1, +1)
// for odd f, (f >> 1 - 1, f >> 1) for even f.  Tile origins are even, so
// for each staged element the lower corner of its 2x2x2 coarse stencil in
// the coarse block and the parities are the same on every tile: they are
// formed once per thread (InterpSlots, one packed word per element the
// thread stages) and the eight corners are read at fixed offsets from the
// lower one.
struct InterpSlots {
    static constexpr int K = (kHalo + kBlock - 1) / kBlock;
    uint32_t w[K];   // corner offset | odd x, y, z << 10..12 | hx << 13 | hy << 18 | hz << 21
};

__device__ __forceinline__ InterpSlots interp_slots() {
    static_assert(kCoarseTile <= 1024 && HX <= 32 && HY <= 8 && HZ <= 8, "slot fields");
    InterpSlots sl;
#pragma unroll
    for (int k = 0; k < InterpSlots::K; ++k) {
        const int i = min((int)threadIdx.x + k * kBlock, kHalo - 1);
        const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
        // fine offset from the tile origin h - 1; its coarse cell sits at
        // ((h - 1) >> 1) + 2 in the coarse block
        const int ox = (hx - 1) & 1, oy = (hy - 1) & 1, oz = (hz - 1) & 1;
        const int jx = ((hx - 1) >> 1) + 2 - (1 - ox), jy = ((hy - 1) >> 1) + 2 - (1 - oy),
                  jz = ((hz - 1) >> 1) + 2 - (1 - oz);
        sl.w[k] = (uint32_t)((jz * CYS + jy) * CXS + jx) | (uint32_t)ox << 10 | (uint32_t)oy << 11 |
                  (uint32_t)oz << 12 | (uint32_t)hx << 13 | (uint32_t)hy << 18 | (uint32_t)hz << 21;
    }
    return sl;
}

// (1 - w) lo + w hi, as lo + w (hi - lo); w = 1/4 when lo is the own cell
// (odd fine coordinate), 3/4 when hi is.
template <class T>
__device__ __forceinline__ T interp_lerp(T lo, T hi, T w) {
    return fma(w, hi - lo, lo);
}

template <class T>
__device__ __forceinline__ void interp_tile(T* r_s, const T* c_s, Grid g, TileOrigin o, const InterpSlots& sl) {
    // the whole haloed tile inside the grid: no per-element test
    const bool inner = o.x0 >= 1 && o.y0 >= 1 && o.z0 >= 1 && o.x0 + TX < g.nx && o.y0 + TY < g.ny &&
                       o.z0 + TZ < g.nz;
    constexpr int DY = CXS, DZ = CXS * CYS;
#pragma unroll
    for (int k = 0; k < InterpSlots::K; ++k) {
        const int i = threadIdx.x + k * kBlock;
        if (k == InterpSlots::K - 1 && i >= kHalo) break;
        const uint32_t w = sl.w[k];
        bool in = true;
        if (!inner) {
            const int hx = (w >> 13) & 31, hy = (w >> 18) & 7, hz = (w >> 21) & 7;
            in = in_grid(g, o.z0 + hz - 1, o.y0 + hy - 1, o.x0 + hx - 1);
        }
        T v = T(0);
        if (in) {
            const T* c = c_s + (w & 1023u);
            const T wx = (w >> 10) & 1 ? T(0.25) : T(0.75), wy = (w >> 11) & 1 ? T(0.25) : T(0.75),
                    wz = (w >> 12) & 1 ? T(0.25) : T(0.75);
            const T p00 = interp_lerp(c[0], c[1], wx), p01 = interp_lerp(c[DY], c[DY + 1], wx);
            const T p10 = interp_lerp(c[DZ], c[DZ + 1], wx), p11 = interp_lerp(c[DZ + DY], c[DZ + DY + 1], wx);
            v = interp_lerp(interp_lerp(p00, p01, wy), interp_lerp(p10, p11, wy), wz);
        }
        r_s[i] = v;
    }
}

// Image and Interp(xc) of one tile in one go (for kernels that do not
// pipeline their tiles).
template <bool L1, int KM, class T>
__device__ __forceinline__ void stage_image_interp(uint32_t* img_s, uint32_t* feat_s, const void* img, T* r_s, T* c_s,
                                                   const T* __restrict__ xc, Grid g, TileOrigin o) {
    put_image_interp<L1, KM, T>(load_image_interp<L1, T>(img, xc, g, o), img_s, feat_s, c_s);
    __syncthreads();
    interp_tile<T>(r_s, c_s, g, o, interp_slots());
}

// x = c1 x1 + c2 CConv_2(Interp(xc), I) on one level l >= 2.
template <class T, int KM>
__global__ __launch_bounds__(kBlock) NPS_WAVES_PER_EU(waves_floor(KM)) void k_up(const uint32_t* __restrict__ cnt, Grid g, uint32_t full,
                                               const T* __restrict__ xc, const T* __restrict__ x1,
                                               T* __restrict__ xout, const CConvW<T>* __restrict__ w,
                                               const MfmaW* __restrict__ wm, const T* __restrict__ kst, int lvl,
                                               const State* st, T* __restrict__ x2out,
                                               const int8_t* __restrict__ wmode) {
    __shared__ uint32_t img_s[kHaloP];
    __shared__ uint32_t feat_s[is_mfma(KM) ? kHaloP : 1];
    __shared__ T r_s[kHaloP];
    __shared__ T c_s[kCoarseTileP];
    const T c1 = (T)st->c1[lvl], c2 = (T)st->c2[lvl];
    const Tiles tl = tiles_of(g);
    const size_t n = ncells(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    const MfmaCtx<KM> mc = mfma_ctx<KM>(wm, lz);
    const InterpSlots isl = interp_slots();
    auto load = [&](int tile) { return load_image_interp<false, T>(cnt, xc, g, tile_origin(tile, tl)); };
    tile_pipeline(tl.count(), load, [&](int tile, const auto& pre, auto prefetch) {
        const TileOrigin o = tile_origin(tile, tl);
        const int wm_e = wave_mode_entry(wmode, tile, lz);
        const int xx = o.x0 + lx, yy = o.y0 + ly, zz = o.z0 + lz;
        const bool active = in_grid(g, zz, yy, xx);
        const size_t idx = active ? cell_index(g, zz, yy, xx) : 0;
        const auto kp = k_preload<T, kpre_on<T, KM, true>>(kst, n, idx);
        __syncthreads();
        put_image_interp<false, KM, T>(pre, img_s, feat_s, c_s);
        const T x1v = x1[idx];
        prefetch();
        __syncthreads();
        interp_tile<T>(r_s, c_s, g, o, isl);
        __syncthreads();
        const int mode = KM == kStored ? -1 : wave_mode<false>(wmode, wm_e, active, img_s, base, full, false, false);
        const T x2 = cconv_any<T, KM, false>(mode, active, img_s, feat_s, r_s, base, w, mc, kst, n, idx, kp);
        if (active) xout[idx] = c1 * x1v + c2 * x2;
        if (active && x2out) x2out[idx] = x2;
    }, st);
}

// Level 1 of the up sweep: dhat = (c1 x1 + c2 CConv_2(Interp(x^2))) / ||r|| on
// fluid cells (0 elsewhere), and the state's ndots partial dots of dhat with
// ad0.. (NPSDO: the stored A d_i of the previous directions; PCG: r; flexible
// PCG: r and the previous residual).
template <class T, int KM, bool HOOK>
__global__ __launch_bounds__(kBlock) NPS_WAVES_PER_EU(waves_floor(KM)) void k_up_l1(
    const uint8_t* __restrict__ lab, Grid g, const T* __restrict__ xc, const T* __restrict__ x1,
    T* __restrict__ dhat, const CConvW<T>* __restrict__ w, const MfmaW* __restrict__ wm,
    const T* __restrict__ kst, const State* st, double* partials, const T* __restrict__ ad0,
    const T* __restrict__ ad1, const T* __restrict__ ad2, const T* __restrict__ ad3, T* __restrict__ x2out,
    const int8_t* __restrict__ wmode) {
    __shared__ uint32_t img_s[kHaloP];
    __shared__ uint32_t feat_s[is_mfma(KM) ? kHaloP : 1];
    __shared__ T r_s[kHaloP];
    __shared__ T c_s[kCoarseTileP];
    const T c1 = (T)st->c1[0], c2 = (T)st->c2[0];
    const T scale = HOOK ? T(1) : (T)st->scale;
    const int ndots = HOOK || st->sym ? 0 : st->ndots;   // the symmetric variant dots after P^T
    const Tiles tl = tiles_of(g);
    const size_t n = ncells(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    const MfmaCtx<KM> mc = mfma_ctx<KM>(wm, lz);
    double v[kRedWidth] = {0.0, 0.0, 0.0, 0.0};
    const T* adp[kMaxOrtho] = {ad0, ad1, ad2, ad3};
    const InterpSlots isl = interp_slots();
    auto load = [&](int tile) { return load_image_interp<true, T>(lab, xc, g, tile_origin(tile, tl)); };
    const bool ran = tile_pipeline(tl.count(), load, [&](int tile, const auto& pre, auto prefetch) {
        const TileOrigin o = tile_origin(tile, tl);
        const int wm_e = wave_mode_entry(wmode, tile, lz);
        const int xx = o.x0 + lx, yy = o.y0 + ly, zz = o.z0 + lz;
        const bool active = in_grid(g, zz, yy, xx);
        const size_t idx = active ? cell_index(g, zz, yy, xx) : 0;
        __syncthreads();
        put_image_interp<true, KM, T>(pre, img_s, feat_s, c_s);
        // per-cell operands, issued before the next tile's loads (an unused
        // A d_i slot reads x1 instead: always a valid address)
        const T x1v = x1[idx];
        T adv[kMaxOrtho];
#pragma unroll
        for (int j = 0; j < kMaxOrtho; ++j) adv[j] = (!HOOK && j < ndots ? adp[j] : x1)[idx];
        prefetch();
        __syncthreads();
        interp_tile<T>(r_s, c_s, g, o, isl);
        __syncthreads();
        const int mode = wave_mode<true>(wmode, wm_e, active, img_s, base, 1u, false, true);
        const T x2 = cconv_any<T, KM, true>(mode, active, img_s, feat_s, r_s, base, w, mc, kst, n, idx,
                                            KPre<T, false>{});
        if (active) {
            T out = T(0);
            if (img_s[base] == (uint32_t)kFluid) out = (c1 * x1v + c2 * x2) * scale;
            dhat[idx] = out;
            if (x2out) x2out[idx] = x2;
            if (!HOOK) {   // only the state's ndots slots (a uniform count)
                const double od = (double)out;
#pragma unroll
                for (int j = 0; j < kMaxOrtho; ++j)
                    if (j < ndots) v[j] = fma(od, (double)adv[j], v[j]);
            }
        }
    }, st);
    if (!HOOK && ran) block_partials<kBlock>(v, partials);
}

// The smallest levels lb..L in one workgroup, in LDS, with stored kernels:
// down sweep (CConv_1 + pool), coarsest CConv_1, up sweep (Interp + CConv_2 +
// combine).  Reads r^lb, writes x^lb.

// The bottom levels live in LDS with a one-cell zero border, so that every
// CConv tap is a fixed offset with no bounds test.
__host__ __device__ inline int padded_cells(Grid g) { return (g.nx + 2) * (g.ny + 2) * (g.nz + 2); }

// Cell p of a bottom level (p < kBottomThreads <= 512) splits into (z, y, x)
// by multiplies: with m = ceil(2^20 / d) = (2^20 + e) / d, 0 <= e < d,
// (p m) >> 20 = floor(p / d + p e / (d 2^20)), and the added term is below
// p / 2^20 < 1 / d for every d < 2048, too small to pass the next multiple
// of 1 / d.  So (p m) >> 20 == p / d exactly.
constexpr int kDivShift = 20;
__host__ __device__ inline uint32_t div_magic(int d) { return (uint32_t)(((1u << kDivShift) + d - 1) / d); }

// One bottom level as the kernel addresses it, set up on the host: one scalar
// load per level per phase, no divisions and no running sums in the kernel.
struct BottomLevel {
    Grid g;
    int n;              // cells
    int sy, sz;         // padded strides of y and z
    int r, x1;          // LDS offsets (elements) of the level's two padded slots
    uint32_t mx, mxy;   // div_magic(nx), div_magic(nx * ny)
};

template <class T>
struct BottomArgs {
    int lb, L;
    int used;   // LDS elements the levels occupy
    BottomLevel lv[kMaxLevels + 1];
    const T* k1[kMaxLevels + 1];
    const T* k2[kMaxLevels + 1];
    const T* rin;
    T* xout;
    // when set, the iteration's Residual stage runs here (sum of res_nparts
    // partials of ||r||^2), before the network reads the state it decides
    const double* res_partials;
    int res_nparts;
    HostFlags* hf;
};

constexpr int kBottomThreads = 512;
constexpr int kBottomLds = 3072;   // elements: >= 2 * sum of the bottom levels' padded cells
static_assert(kBottomMaxCells <= kBottomThreads, "one cell of each bottom level per thread");
static_assert(kBottomThreads <= 512 && kBottomMaxCells <= 512, "cell splitting by div_magic");

// A load through a pointer that is known to address device memory: pointers
// read from a kernel-argument array are generic, and a generic (flat) load
// would share the LDS counter.
template <class T>
__device__ __forceinline__ T ld_global(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;   // address-space cast (C-style only)
}

// One output of a stored-kernel CConv at padded index c of a level with
// padded strides (sy, sz) (input v in the padded layout: its border is zero,
// the CConv's zero padding).
template <class T>
__device__ __forceinline__ T bottom_cconv(const T (&kv)[kTaps], const T* v, int sy, int sz, int c) {
    T acc = T(0);
#pragma unroll
    for (int t = 0; t < kTaps; ++t) acc = fma(kv[t], v[c + (t / 9 - 1) * sz + ((t / 3) % 3 - 1) * sy + (t % 3 - 1)], acc);
    return acc;
}

// Interp(xc) at fine cell (z, y, x) from the coarse level vc in the padded
// layout (coarse coordinates clamped: the interpolation's edge rule).
template <class T>
__device__ __forceinline__ T bottom_interp(const T* xc, const BottomLevel& vc, int z, int y, int x) {
    int jx, jxn, jy, jyn, jz, jzn;
    up_axis(x, vc.g.nx, jx, jxn);
    up_axis(y, vc.g.ny, jy, jyn);
    up_axis(z, vc.g.nz, jz, jzn);
    auto at = [&](int zz, int yy, int xx) { return xc[(zz + 1) * vc.sz + (yy + 1) * vc.sy + xx + 1]; };
    const T a = T(0.75), b = T(0.25);
    const T p00 = a * at(jz, jy, jx) + b * at(jz, jy, jxn);
    const T p01 = a * at(jz, jyn, jx) + b * at(jz, jyn, jxn);
    const T p10 = a * at(jzn, jy, jx) + b * at(jzn, jy, jxn);
    const T p11 = a * at(jzn, jyn, jx) + b * at(jzn, jyn, jxn);
    return a * (a * p00 + b * p01) + b * (a * p10 + b * p11);
}

// Levels lb and lb + 1 hold at most one cell per thread (lb has at most
// kBottomThreads cells): every global load they need (r^lb and their stored
// kernels) is issued at the start, so the sweep waits for one memory
// latency instead of one per level.  Levels past lb + 1 (a handful of
// cells) load their kernels where they are used.  The result of level l
// (x1^l, then x^l once the up sweep has combined it in place) stays in the
// level's x1 slot; the r slot holds r^l on the way down and Interp(x^(l+1))
// on the way up.
template <class T>
__global__ __launch_bounds__(kBottomThreads) void k_bottom(BottomArgs<T> a, State* st) {
    const int done = st->done;   // tested once the network is formed
    const ResidualIn rin = residual_in(st);   // read by the Residual stage below
    __shared__ T buf[kBottomLds];
    const int lb = a.lb, L = a.L, p = threadIdx.x;
    const BottomLevel v0 = a.lv[lb];
    const int n0 = v0.n, n1 = lb < L ? a.lv[lb + 1].n : 1;
    const int q0 = min(p, n0 - 1), q1 = min(p, n1 - 1);   // clamped: every load is in bounds
    // All loads go out at once: the Residual stage's partials (its sums are
    // only needed at the end), the input and the stored kernels.
    double rpart[1][kSumU];
    head_partials<1, kBottomThreads>(a.res_partials, a.res_partials ? a.res_nparts : 0, rpart);
    T r0 = ld_global(a.rin + q0);
    // the combination weights of level lb (set up before the solve)
    const T c1_0 = (T)st->c1[lb - 1], c2_0 = (T)st->c2[lb - 1];
    T k1_0[kTaps], k2_0[kTaps], k1_1[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) k1_0[t] = ld_global(a.k1[lb] + (size_t)t * n0 + q0);
    if (lb < L) {   // in the order of use; level lb + 1's kernel only for its cells (whole waves skip it)
        if (p < n1) {
#pragma unroll
            for (int t = 0; t < kTaps; ++t) k1_1[t] = ld_global(a.k1[lb + 1] + (size_t)t * n1 + q1);
        } else {
#pragma unroll
            for (int t = 0; t < kTaps; ++t) k1_1[t] = T(0);
        }
#pragma unroll
        for (int t = 0; t < kTaps; ++t) k2_0[t] = ld_global(a.k2[lb] + (size_t)t * n0 + q0);
    }
    // zero borders: clear the whole buffer, then fill the interiors
    for (int i = p; i < a.used; i += kBottomThreads) buf[i] = T(0);
    // cell p of a level (at most one per thread) and its padded index
    auto cell = [&](const BottomLevel& v, int& z, int& y, int& x) {
        const int t = (int)(__umul24((uint32_t)p, v.mx) >> kDivShift);   // p / nx
        z = (int)(__umul24((uint32_t)p, v.mxy) >> kDivShift);            // p / (nx ny)
        x = p - t * v.g.nx;
        y = t - z * v.g.ny;
        return (z + 1) * v.sz + (y + 1) * v.sy + x + 1;
    };
    int z0, y0, x0;
    const int c0 = cell(v0, z0, y0, x0);
    __syncthreads();
    if (p < n0) buf[v0.r + c0] = r0;
    __syncthreads();
    // down sweep and coarsest level
    if (p < n0) buf[v0.x1 + c0] = bottom_cconv(k1_0, buf + v0.r, v0.sy, v0.sz, c0);
    __syncthreads();
    for (int l = lb; l < L; ++l) {
        const BottomLevel f = a.lv[l], v = a.lv[l + 1];
        int z, y, x;
        const int c = cell(v, z, y, x);
        if (p < v.n) {   // Pool(x1^l)
            const T* s = buf + f.x1 + (2 * z + 1) * f.sz + (2 * y + 1) * f.sy + 2 * x + 1;
            T sum = T(0);
#pragma unroll
            for (int k = 0; k < 8; ++k) sum += s[(k >> 2) * f.sz + ((k >> 1) & 1) * f.sy + (k & 1)];
            buf[v.r + c] = sum * T(0.125);
        }
        __syncthreads();
        if (p < v.n) {
            T acc;
            if (l == lb) {
                acc = bottom_cconv(k1_1, buf + v.r, v.sy, v.sz, c);
            } else {
                T kv[kTaps];
#pragma unroll
                for (int t = 0; t < kTaps; ++t) kv[t] = ld_global(a.k1[l + 1] + (size_t)t * v.n + p);
                acc = bottom_cconv(kv, buf + v.r, v.sy, v.sz, c);
            }
            buf[v.x1 + c] = acc;
        }
        __syncthreads();
    }
    // up sweep: x^L = x1^L.  Interp(x^(l+1)) is formed once per level into the
    // level's r slot (its down input is no longer needed; the border stays
    // zero), then CConv_2 gathers from it and the combination overwrites
    // x1^l, which only this thread reads, with x^l.
    for (int l = L - 1; l >= lb; --l) {
        const BottomLevel v = a.lv[l], vc = a.lv[l + 1];
        const T c1 = l == lb ? c1_0 : (T)st->c1[l - 1], c2 = l == lb ? c2_0 : (T)st->c2[l - 1];
        int z, y, x;
        const int c = cell(v, z, y, x);
        if (p < v.n) buf[v.r + c] = bottom_interp<T>(buf + vc.x1, vc, z, y, x);
        __syncthreads();
        if (p < v.n) {
            T acc;
            if (l == lb) {
                acc = bottom_cconv(k2_0, buf + v.r, v.sy, v.sz, c);
            } else {
                T kv[kTaps];
#pragma unroll
                for (int t = 0; t < kTaps; ++t) kv[t] = ld_global(a.k2[l] + (size_t)t * v.n + p);
                acc = bottom_cconv(kv, buf + v.r, v.sy, v.sz, c);
            }
            T* xo = buf + v.x1 + c;
            *xo = c1 * *xo + c2 * acc;
        }
        if (l > lb) __syncthreads();   // level lb's cells are read back only by the thread that wrote them
    }
    // The network is linear in r, so the stop test and the Residual stage
    // (convergence, 1/||r||, read from the next kernel on) come last: a block
    // of a stopped solve writes nothing.
    if (done) return;
    if (a.res_partials) {
        __shared__ int done_s;
        double v[1];
        finish_partials<1, kBottomThreads>(rpart, a.res_partials, a.res_nparts, 1, v);
        if (p == 0) done_s = residual_stage(st, rin, v[0], a.hf);
        __syncthreads();
        if (done_s) return;
    }
    if (p < n0) a.xout[p] = buf[v0.x1 + c0];   // x^lb (x1^L itself when the bottom holds only the coarsest level)
}

// ---------------------------------------------------------------------------
// Krylov kernels (Alg. 1)
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// plane-marching geometry of the 7-point kernels
// ---------------------------------------------------------------------------
// A block owns a footprint of PX x PY columns (one thread per column) and
// marches it through a chunk of z-planes.  Each plane is staged once, with
// its x/y border, in rows of PX + 2 contiguous cells; the z neighbours of a
// cell come from the planes staged before and after its own.  Against a
// tile with a full 3-D halo this stages about 0.6x the elements, in rows
// 3.7x longer.
constexpr int PX = 64, PY = kBlock / PX;
constexpr int PHX = PX + 2, PHY = PY + 2;
constexpr int kPlane = PHX * PHY;
constexpr int kPlaneP = pad_block(kPlane);
struct Columns {   // column footprints x z-chunks of a grid
    int ncx, ncy, ncz, chunk;
    __host__ __device__ int count() const { return ncx * ncy * ncz; }
};

// Chunks of 8 planes (the plane below a chunk is read once more per chunk);
// 4 or 2 on grids that would otherwise give fewer than 512 chunks, so that
// small grids still spread over the compute units.  A function of the grid
// alone: launches and kernels agree on it.
__host__ __device__ inline Columns columns_of(Grid g) {
    const int ncx = (g.nx + PX - 1) / PX, ncy = (g.ny + PY - 1) / PY;
    int chunk = 8;
    while (chunk > 2 && ncx * ncy * ((g.nz + chunk - 1) / chunk) < 512) chunk /= 2;
    return Columns{ncx, ncy, (g.nz + chunk - 1) / chunk, chunk};
}

// Work items of the 7-point kernels that hold no fluid cell.  On such an
// item r = 0 and A d = 0, and it adds nothing to any dot (every term has a
// factor r or A d), so once its cells hold zeros in the solver's vectors the
// kernels need not visit it: they walk a list of the other ("live") items.
// Buffers zeroed on the items without fluid at set-up (2, 4 or 8 B elements).
struct ZeroBufs {
    void* p[2 * kRing + 3];
    int bytes[2 * kRing + 3];
    int n;
};

// One block per item (a thread per column, columns_of order): live[w] = 1
// when item w holds a fluid cell; otherwise the item's cells are zeroed in
// every buffer of zb.
__global__ __launch_bounds__(kBlock) void k_item_live(const uint8_t* __restrict__ lab, Grid g,
                                                      uint8_t* __restrict__ live, ZeroBufs zb) {
    const Columns cl = columns_of(g);
    const int w = blockIdx.x;
    const int x0 = (w % cl.ncx) * PX, y0 = ((w / cl.ncx) % cl.ncy) * PY, z0 = (w / (cl.ncx * cl.ncy)) * cl.chunk;
    const int z1 = min(z0 + cl.chunk, g.nz);
    const int xx = x0 + threadIdx.x % PX, yy = y0 + threadIdx.x / PX;
    const bool col = xx < g.nx && yy < g.ny;
    int f = 0;
    if (col)
        for (int z = z0; z < z1; ++z) f |= lab[cell_index(g, z, yy, xx)] == kFluid;
    const int any = __syncthreads_or(f);
    if (threadIdx.x == 0) live[w] = any ? 1 : 0;
    if (any || !col) return;
    for (int i = 0; i < zb.n; ++i)
        for (int z = z0; z < z1; ++z) {
            const size_t q = cell_index(g, z, yy, xx);
            if (zb.bytes[i] == 8) static_cast<double*>(zb.p[i])[q] = 0.0;
            else if (zb.bytes[i] == 4) static_cast<float*>(zb.p[i])[q] = 0.0f;
            else static_cast<uint16_t*>(zb.p[i])[q] = 0;
        }
}

// One block: items[0 .. nlive) = the live items in increasing order (z-major,
// so each XCD's contiguous share of the list is a z-range), st->nlive = nlive.
__global__ __launch_bounds__(kBlock) void k_item_list(const uint8_t* __restrict__ live, int count,
                                                      uint32_t* __restrict__ items, State* st) {
    constexpr int W = kBlock / 64;
    __shared__ uint32_t wsum[W];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t base = 0;
    for (int i0 = 0; i0 < count; i0 += kBlock) {
        const int i = i0 + threadIdx.x;
        const bool f = i < count && live[i] != 0;
        const uint64_t m = __ballot(f);
        if (lane == 0) wsum[wv] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t off = base, tot = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            off += k < wv ? wsum[k] : 0u;
            tot += wsum[k];
        }
        if (f) items[off + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)i;
        base += tot;
        __syncthreads();   // wsum is rewritten by the next round
    }
    if (threadIdx.x == 0) st->nlive = (int)base;
}

// d = dhat - sum_j beta_j d_(k-1-j) (classical Gram-Schmidt in the A inner
// product; equal to the paper's sequential update because the directions in
// the window are already mutually A-orthogonal), A d, and the partial dots
// d . A d and r . d.
// NO: the number of previous-direction buffers passed (n_ortho); the first
// nprev of them enter (state), the rest are loaded and not used.
// The coefficients come from the Dots stage, which every block runs on its
// own from the dnparts partials of the dots (the same sums in every block:
// a fixed order); block 0 records them in the state.  dots and partials
// must be different buffers (blocks write their partials while others may
// still read the dots).  Only the live items are visited (items[0 .. nlive));
// the others hold d = 0 and A d = 0 from set-up.
template <class T, int NO>
__global__ __launch_bounds__(kBlock) void k_ortho(const uint8_t* __restrict__ lab, Grid g, const T* __restrict__ dhat,
                                                  const T* __restrict__ p0, const T* __restrict__ p1,
                                                  const T* __restrict__ p2, const T* __restrict__ p3,
                                                  const T* __restrict__ r, T* __restrict__ dout, T* __restrict__ adout,
                                                  State* st, const double* __restrict__ dots, int dnparts, int sl0,
                                                  int sl1, int sl2, int sl3, double* __restrict__ partials,
                                                  const uint32_t* __restrict__ items, int nlive) {
    __shared__ uint32_t lab_s[2][kPlaneP];
    __shared__ T d_s[2][kPlaneP];
    __shared__ double beta_s[kMaxOrtho];
    const int done = st->done;   // tested once the first loads are out
    const int nprev = st->nprev;
    const int sl[kMaxOrtho] = {sl0, sl1, sl2, sl3};
    const DotsIn din = dots_in(st, sl);
    const int ndots = st->ndots;
    T bj[kMaxOrtho] = {T(0), T(0), T(0), T(0)};
    const T* pp[kMaxOrtho] = {p0, p1, p2, p3};
    const Columns cl = columns_of(g);
    const int lx = threadIdx.x % PX, ly = threadIdx.x / PX;
    const int own = (ly + 1) * PHX + (lx + 1);
    double v[kRedWidth] = {0.0, 0.0, 0.0, 0.0};
    struct LD {
        T dh;
        T p[NO > 0 ? NO : 1];
        uint8_t l;
    };
    auto element = [&](int zz, int yy, int xx) {
        const bool in = in_grid(g, zz, yy, xx);
        const size_t q = in ? cell_index(g, zz, yy, xx) : 0;
        LD e;
        e.dh = *at_or(dhat, q, in, pad_zero<T>());
#pragma unroll
        for (int j = 0; j < NO; ++j) e.p[j] = *at_or(pp[j], q, in, pad_zero<T>());
        e.l = *at_or(lab, q, in, g_pad_solid);
        return e;
    };
    auto plane = [&](int x0, int y0, int zz) {
        return load_batch<kPlane, LD>([&](int i) { return element(zz, y0 + i / PHX - 1, x0 + i % PHX - 1); });
    };
    auto direction = [&](const LD& e) {   // d = dhat - sum_j beta_j d_(k-1-j)
        T dv = e.dh;
#pragma unroll
        for (int j = 0; j < NO; ++j) dv = j < nprev ? dv - bj[j] * e.p[j] : dv;
        return dv;
    };
    // The Dots stage, once per block (its partials loaded first, the first
    // item's loads issued behind them); false: the solve has stopped and the
    // block writes nothing.  The up kernel forms ndots <= max(NO, 2) dots
    // (NPSDO: nprev <= n_ortho; the PCG forms: 1 or 2).
    constexpr int DW = NO > 2 ? NO : 2;
    double dpart[DW][kSumU];
    head_partials<DW, kBlock>(dots, dnparts, dpart);
    auto start = [&]() -> bool {
        if (done) return false;
        if (dnparts > 0) {
            double dw[DW], dv[kMaxOrtho] = {0.0, 0.0, 0.0, 0.0};
            finish_partials<DW, kBlock>(dpart, dots, dnparts, ndots, dw);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int j = 0; j < DW; ++j) dv[j] = dw[j];
                double beta[kMaxOrtho], rho;
                dots_betas(din, dv, beta, rho);
#pragma unroll
                for (int j = 0; j < kMaxOrtho; ++j) beta_s[j] = beta[j];
                if (blockIdx.x == 0) {
#pragma unroll
                    for (int j = 0; j < kMaxOrtho; ++j) st->beta[j] = beta[j];
                    if (din.method != 0) st->rho = rho;
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kMaxOrtho; ++j) bj[j] = (T)beta_s[j];
        }
        return true;
    };
    // One work item; the block's first (FIRST) runs the Dots stage once its
    // loads are out (false: the block stops).  The first item is peeled off the
    // loop, so the stage's registers are free during the others.
    auto item = [&](int w, auto first_tag) -> bool {
        const int x0 = (w % cl.ncx) * PX, y0 = ((w / cl.ncx) % cl.ncy) * PY, z0 = (w / (cl.ncx * cl.ncy)) * cl.chunk;
        const int z1 = min(z0 + cl.chunk, g.nz);
        const int xx = x0 + lx, yy = y0 + ly;
        const bool col = xx < g.nx && yy < g.ny;
        const LD below = element(z0 - 1, yy, xx);   // the z - 1 neighbour of plane z0
        auto pre = plane(x0, y0, z0);
        auto pre2 = plane(x0, y0, z0 + 1);
        if constexpr (decltype(first_tag)::value) {
            __asm__ volatile("" ::: "memory");   // the loads stay above the test
            if (!start()) return false;
        }
        T dm = direction(below);   // own column, plane s - 2
        uint32_t lm = below.l;
        T rv = T(0);               // r of plane s - 1
        auto step = [&](int s, auto& pre) {
            const int cur = s & 1, prev = cur ^ 1;
            __syncthreads();   // the reads of this buffer (plane s - 2) are done
            put_batch(pre, [&](int i, LD e) {
                d_s[cur][i] = direction(e);
                lab_s[cur][i] = e.l;
            });
            const T rnext = r[col && s < z1 ? cell_index(g, s, yy, xx) : 0];
            if (s + 2 <= z1) pre = plane(x0, y0, s + 2);
            __syncthreads();   // plane s is staged
            if (s > z0) {      // the own cell of plane s - 1
                const T dv = d_s[prev][own];
                const uint32_t lc = lab_s[prev][own];
                if (col) {
                    T ad = T(0);
                    if (lc == kFluid) {   // the mixed-BC 7-point row, neighbours z-, z+, y-, y+, x-, x+
                        const uint32_t nl[6] = {lm, lab_s[cur][own], lab_s[prev][own - PHX], lab_s[prev][own + PHX],
                                                lab_s[prev][own - 1], lab_s[prev][own + 1]};
                        const T nv[6] = {dm, d_s[cur][own], d_s[prev][own - PHX], d_s[prev][own + PHX],
                                         d_s[prev][own - 1], d_s[prev][own + 1]};
                        int cnt = 0;
                        T sum = T(0);
#pragma unroll
                        for (int k = 0; k < 6; ++k) {
                            cnt += (nl[k] != (uint32_t)kSolid);
                            if (nl[k] == (uint32_t)kFluid) sum += nv[k];
                        }
                        ad = (T)cnt * dv - sum;
                    }
                    const size_t q = cell_index(g, s - 1, yy, xx);
                    dout[q] = dv;
                    adout[q] = ad;
                    v[0] += (double)dv * (double)ad;
                    v[1] += (double)rv * (double)dv;
                }
                dm = dv;
                lm = lc;
            }
            rv = rnext;
        };
        // planes are loaded two steps ahead of their staging
        for (int s = z0; s <= z1; s += 2) {
            step(s, pre);
            if (s + 1 <= z1) step(s + 1, pre2);
        }
        return true;
    };
    TileSpan sp = tile_span(nlive);
    if (sp.t0 >= sp.t1) {   // a block without items
        if (!start()) return;
    } else {
        if (!item((int)items[sp.t0], std::true_type{})) return;
        for (sp.t0 += sp.step; sp.t0 < sp.t1; sp.t0 += sp.step) item((int)items[sp.t0], std::false_type{});
    }
    block_partials<kBlock>(v, partials);
}

// The start of an iteration (Alg. 1): applies the pending update
// x += alpha d and forms the literal residual r = b - A x (the stencil in
// double), writes x to the other solution buffer xnew (so no block reads a
// value another block already updated; the buffers alternate with the
// iteration, and the Residual stage flips state.xcur to match) and r as the
// network input, and the partial ||r||^2.  Plane-marching: step s stages
// plane s (x + alpha d and the labels, outside the grid x = 0 and solid)
// and forms plane s - 1.  Only the live items are visited (items[0 .. nlive),
// k_item_list); the others hold r = 0 and x = 0 from set-up.
// With snp > 0 the kernel first runs the previous iteration's Step stage:
// every block sums the snp partials of d . A d and r . d (the same sums in
// each, a fixed order), forms alpha and applies the update; block 0 records
// the stage (slot: ring slot of d); on a breakdown no block writes anything.
// With snp == 0 (the first iteration) there is no pending update.
template <class T, class X>
__global__ __launch_bounds__(kBlock) void k_residual(const uint8_t* __restrict__ lab, Grid g,
                                                     const double* __restrict__ b, const X* __restrict__ x,
                                                     X* __restrict__ xnew, const T* __restrict__ dpend,
                                                     T* __restrict__ r, State* st, const double* __restrict__ steps,
                                                     int snp, int slot, HostFlags* hf, double* partials,
                                                     const uint32_t* __restrict__ items, int nlive) {
    __shared__ uint32_t lab_s[2][kPlaneP];
    __shared__ X x_s[2][kPlaneP];
    __shared__ double alpha_s;
    __shared__ int ok_s;
    const int done = st->done;   // tested once the first loads are out
    const StepIn sin = step_in(st);   // read by the Step stage below
    const bool pend = snp > 0;
    X alpha = X(0);
    const Columns cl = columns_of(g);
    const int lx = threadIdx.x % PX, ly = threadIdx.x / PX;
    const int own = (ly + 1) * PHX + (lx + 1);
    double v[kRedWidth] = {0.0, 0.0, 0.0, 0.0};
    auto element = [&](int zz, int yy, int xx) {
        const bool in = in_grid(g, zz, yy, xx);
        const size_t q = in ? cell_index(g, zz, yy, xx) : 0;
        return XDL<X, T>{*at_or<X>(x, q, in, pad_zero<X>()), *at_or(dpend, q, in, pad_zero<T>()),
                         *at_or(lab, q, in, g_pad_solid)};
    };
    auto plane = [&](int x0, int y0, int zz) {
        return load_batch<kPlane, XDL<X, T>>([&](int i) { return element(zz, y0 + i / PHX - 1, x0 + i % PHX - 1); });
    };
    auto updated = [&](const XDL<X, T>& e) { return pend ? e.x + alpha * (X)e.d : e.x; };
    // The Step stage, once per block (its partials loaded first, the first
    // item's loads issued behind them); false: the solve has stopped or broken
    // down, and the block writes nothing.
    double spart[2][kSumU];
    head_partials<2, kBlock>(steps, pend ? snp : 0, spart);
    auto start = [&]() -> bool {
        if (done) return false;
        if (pend) {
            double sv[2];
            finish_partials<2, kBlock>(spart, steps, snp, 2, sv);
            if (threadIdx.x == 0) {
                double a = 0.0;
                ok_s = step_alpha(sin, sv[0], sv[1], a);
                alpha_s = a;
                if (blockIdx.x == 0) step_update(st, sin, slot, sv[0], sv[1], hf);
            }
            __syncthreads();
            if (!ok_s) return false;
            alpha = (X)alpha_s;
        }
        return true;
    };
    // One work item; the block's first (FIRST) runs the Step stage once its
    // loads are out (false: the block stops).  The first item is peeled off the
    // loop, so the stage's registers are free during the others.
    auto item = [&](int w, auto first_tag) -> bool {
        const int x0 = (w % cl.ncx) * PX, y0 = ((w / cl.ncx) % cl.ncy) * PY, z0 = (w / (cl.ncx * cl.ncy)) * cl.chunk;
        const int z1 = min(z0 + cl.chunk, g.nz);
        const int xx = x0 + lx, yy = y0 + ly;
        const bool col = xx < g.nx && yy < g.ny;
        const XDL<X, T> below = element(z0 - 1, yy, xx);   // the z - 1 neighbour of plane z0
        auto pre = plane(x0, y0, z0);
        auto pre2 = plane(x0, y0, z0 + 1);
        if constexpr (decltype(first_tag)::value) {
            __asm__ volatile("" ::: "memory");   // the loads stay above the test
            if (!start()) return false;
        }
        X xm = updated(below);   // own column, plane s - 2
        uint32_t lm = below.l;
        double bv = 0.0;         // b of plane s - 1
        auto step = [&](int s, auto& pre) {
            const int cur = s & 1, prev = cur ^ 1;
            __syncthreads();   // the reads of this buffer (plane s - 2) are done
            put_batch(pre, [&](int i, XDL<X, T> e) {
                lab_s[cur][i] = e.l;
                x_s[cur][i] = updated(e);
            });
            const double bnext = b[col && s < z1 ? cell_index(g, s, yy, xx) : 0];
            if (s + 2 <= z1) pre = plane(x0, y0, s + 2);
            __syncthreads();   // plane s is staged
            if (s > z0) {      // the own cell of plane c = s - 1
                const uint32_t lc = lab_s[prev][own];
                const X xc = x_s[prev][own];
                if (col) {
                    double rv = 0.0;
                    if (lc == kFluid) {   // the mixed-BC 7-point row, neighbours z-, z+, y-, y+, x-, x+
                        const uint32_t nl[6] = {lm, lab_s[cur][own], lab_s[prev][own - PHX], lab_s[prev][own + PHX],
                                                lab_s[prev][own - 1], lab_s[prev][own + 1]};
                        const X nv[6] = {xm, x_s[cur][own], x_s[prev][own - PHX], x_s[prev][own + PHX],
                                         x_s[prev][own - 1], x_s[prev][own + 1]};
                        int cnt = 0;
                        double sum = 0.0;
#pragma unroll
                        for (int k = 0; k < 6; ++k) {
                            cnt += (nl[k] != (uint32_t)kSolid);
                            if (nl[k] == (uint32_t)kFluid) sum += (double)nv[k];
                        }
                        rv = bv - ((double)cnt * (double)xc - sum);
                    }
                    const size_t q = cell_index(g, s - 1, yy, xx);
                    xnew[q] = xc;
                    r[q] = (T)rv;
                    const double rt = (double)(T)rv;
                    v[0] += rt * rt;
                }
                xm = xc;
                lm = lc;
            }
            bv = bnext;
        };
        // planes are loaded two steps ahead of their staging
        for (int s = z0; s <= z1; s += 2) {
            step(s, pre);
            if (s + 1 <= z1) step(s + 1, pre2);
        }
        return true;
    };
    TileSpan sp = tile_span(nlive);
    if (sp.t0 >= sp.t1) {   // a block without items
        if (!start()) return;
    } else {
        if (!item((int)items[sp.t0], std::true_type{})) return;
        for (sp.t0 += sp.step; sp.t0 < sp.t1; sp.t0 += sp.step) item((int)items[sp.t0], std::false_type{});
    }
    block_partials<kBlock>(v, partials);
}

// Partial dots v . a_j, j < the state's ndots (the up kernel's dots, for the
// symmetric variant whose direction is formed after P^T); an unused slot
// reads v itself.
template <class T>
__global__ __launch_bounds__(kBlock) void k_dots(size_t n, const T* __restrict__ v, const T* __restrict__ a0,
                                                 const T* __restrict__ a1, const T* __restrict__ a2,
                                                 const T* __restrict__ a3, const State* st, double* partials) {
    if (st->done) return;
    const int nd = st->ndots;
    const T* ap[kMaxOrtho] = {nd > 0 ? a0 : v, nd > 1 ? a1 : v, nd > 2 ? a2 : v, nd > 3 ? a3 : v};
    double acc[kRedWidth] = {0.0, 0.0, 0.0, 0.0};
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        const double vi = (double)v[i];
#pragma unroll
        for (int j = 0; j < kMaxOrtho; ++j) acc[j] += j < nd ? vi * (double)ap[j][i] : 0.0;
    }
    block_partials<kBlock>(acc, partials);
}

// Partial dots x.py, y.px, x.px, y.py (the asymmetry measure of the appendix
// on symmetry), summed by k_sum_partials.
template <class T>
__global__ __launch_bounds__(kBlock) void k_dot4(size_t n, const T* __restrict__ x, const T* __restrict__ y,
                                                 const T* __restrict__ px, const T* __restrict__ py, double* partials) {
    double acc[kRedWidth] = {0.0, 0.0, 0.0, 0.0};
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        const double xi = (double)x[i], yi = (double)y[i], pxi = (double)px[i], pyi = (double)py[i];
        acc[0] += xi * pyi;
        acc[1] += yi * pxi;
        acc[2] += xi * pxi;
        acc[3] += yi * pyi;
    }
    block_partials<kBlock>(acc, partials);
}

// out[w] = sum of the nparts partials of value w (block order), w < kRedWidth.
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ partials, int nparts,
                                                         double* __restrict__ out) {
    double v[kRedWidth];
    sum_partials<kRedWidth, kBlock>(partials, nparts, kRedWidth, v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int w = 0; w < kRedWidth; ++w) out[w] = v[w];
}

// x_out = x (the current solution buffer) on fluid cells, 0 elsewhere, in double.
template <class X>
__global__ __launch_bounds__(kBlock) void k_finalize(size_t n, const uint8_t* __restrict__ lab, const X* xb0,
                                                     const X* xb1, const State* st, double* __restrict__ xout) {
    const X* __restrict__ x = st->xcur ? xb1 : xb0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        xout[i] = lab[i] == kFluid ? (double)x[i] : 0.0;
}

// y = A x (parity hook; same stencil code as the solve).
template <class T>
__global__ __launch_bounds__(kBlock) void k_laplacian(const uint8_t* __restrict__ lab, Grid g,
                                                      const T* __restrict__ x, T* __restrict__ y) {
    __shared__ uint32_t lab_s[kHaloP];
    __shared__ T x_s[kHaloP];
    const Tiles tl = tiles_of(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    for (TileSpan sp = tile_span(tl.count()); sp.t0 < sp.t1; sp.t0 += sp.step) {
        const int tile = sp.t0;
        const TileOrigin o = tile_origin(tile, tl);
        __syncthreads();
        stage_image<true>(lab_s, lab, g, o);
        for (int i = threadIdx.x; i < kHalo; i += kBlock) {
            const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
            const int xx = o.x0 + hx - 1, yy = o.y0 + hy - 1, z = o.z0 + hz - 1;
            x_s[i] = in_grid(g, z, yy, xx) ? x[cell_index(g, z, yy, xx)] : T(0);
        }
        __syncthreads();
        const int xx = o.x0 + lx, yy = o.y0 + ly, z = o.z0 + lz;
        if (in_grid(g, z, yy, xx)) y[cell_index(g, z, yy, xx)] = apply_A<T, T, uint32_t>(lab_s, x_s, base, HX, HX * HY);
    }
}

}  // namespace nps
