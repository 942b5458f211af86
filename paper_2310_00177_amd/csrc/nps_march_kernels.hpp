// Level-1 network kernels on matrix cores, marching column footprints
// through z (Alg. 2, first level: CConv_1^1 + pool down, interpolation +
// CConv_2^1 + combine up).
//
// A block owns a footprint of PX x PY = 64 x 4 columns and walks it through a
// chunk of z-planes.  Every plane is staged once in LDS, with its x/y border,
// as one 8-byte record per cell: the CConv input (float) and the cell's two
// MFMA features (fluid and air counts as a bf16 / fp16 pair).  Four plane
// buffers form a ring, so the output plane c reads planes c-1, c, c+1 while
// plane c+2 is being written: one barrier per plane.
//
// Wave w covers x = 16 w .. 16 w + 15 of the footprint and its four rows;
// row q is one 16-cell group, the N dimension of v_mfma_f32_16x16x32.  For a
// group the per-cell kernels K^T[tap][cell] = A[tap][feature] B[feature][cell]
// come out of the matrix cores with lane (g, n) (g = lane / 16, n = lane % 16)
// holding the taps of window positions {4g + i, 16 + 4g + i : i < 4} of cell
// n; the lane reads the CConv input at exactly those positions (the feature
// and tap enumerations coincide), so the eight records it reads give both its
// B fragment and its eight input values.  The four partial sums of a cell (one
// per lane group) are combined for the four groups together with a
// reduce-scatter over the lane groups (two gfx950 permlane swaps): afterwards
// lane (g, n) holds the output of cell (x = 16 w + n, y = g).
//
// Groups are classified once per solve (k_group_modes; the labels do not
// change during a solve): zero (every output is zero), pure (every cell that
// matters has an all-fluid window: the constant fluid kernel) or general
// (matrix cores).  A wave reads its four group modes with one scalar load.
#pragma once

#include "nps_kernels.hpp"

namespace nps {

enum GroupMode : uint32_t { kGZero = 0, kGPure = 1, kGGeneral = 2 };

// Work items of the marching network kernels: a 64 x 4 column footprint
// over a chunk of 4 z-planes (2 on grids with fewer than 1024 such items).
// Shorter items than the 7-point kernels' keep the per-block work even: an
// item's cost depends on its group modes (interface footprints cost up to
// 1.7x empty ones) and the cost field is smooth in space.  When the grid of
// blocks is a multiple of the XCD count, XCD x (blocks b with b % 8 == x)
// takes the z-chunks zc with zc % 8 == x, every footprint of each, so its
// blocks share the y halos of a slab in their L2 while every XCD gets slabs
// from the whole height; its blocks take the XCD's items round-robin.  A
// function of the grid alone: launches and kernels agree on it.
__host__ __device__ inline Columns march_columns(Grid g) {
    const int ncx = (g.nx + PX - 1) / PX, ncy = (g.ny + PY - 1) / PY;
    const int chunk = ncx * ncy * ((g.nz + 3) / 4) >= 1024 ? 4 : 2;
    return Columns{ncx, ncy, (g.nz + chunk - 1) / chunk, chunk};
}

// One mode byte per (footprint, z, wave, row): index ((z ncy + cy) ncx + cx)
// * 16 + 4 w + q, so a wave's four modes are one aligned word.
__host__ __device__ inline size_t group_mode_bytes(Grid g) {
    const Columns cl = columns_of(g);
    return (size_t)cl.ncx * cl.ncy * g.nz * 16;
}

// Labels of a level-1 window (solid outside the grid): all fluid, any fluid.
__device__ __forceinline__ void window_flags(const uint8_t* __restrict__ lab, Grid g, int z, int y, int x,
                                             bool& all_fluid, bool& any_fluid) {
    all_fluid = true;
    any_fluid = false;
#pragma unroll
    for (int o = 0; o < kTaps; ++o) {
        const int zz = z + o / 9 - 1, yy = y + (o / 3) % 3 - 1, xx = x + o % 3 - 1;
        const uint8_t l = in_grid(g, zz, yy, xx) ? lab[cell_index(g, zz, yy, xx)] : (uint8_t)kSolid;
        all_fluid &= l == kFluid;
        any_fluid |= l == kFluid;
    }
}

// Group modes of the level-1 down (CConv_1, input zero off fluid) and up
// (CConv_2, output restricted to fluid) kernels.  One thread per cell, 16
// consecutive threads per group.
//   down: zero when no window of the group holds fluid; pure when every
//         window that holds fluid is all fluid (a window without fluid
//         outputs zero under any kernel);
//   up:   zero when no cell of the group is fluid; pure when every fluid
//         cell's window is all fluid (other outputs are masked).
__global__ __launch_bounds__(kBlock) void k_group_modes(const uint8_t* __restrict__ lab, Grid g,
                                                        uint8_t* __restrict__ mdown, uint8_t* __restrict__ mup) {
    const Columns cl = columns_of(g);
    const size_t total = (size_t)cl.ncx * cl.ncy * g.nz * 256;   // 16 groups x 16 cells per (footprint, z)
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t grp = i >> 4;
    const int k = (int)(i & 15), q = (int)(grp & 3), w = (int)((grp >> 2) & 3);
    const size_t rest = grp >> 4;
    const int cx = (int)(rest % cl.ncx), cy = (int)((rest / cl.ncx) % cl.ncy), z = (int)(rest / ((size_t)cl.ncx * cl.ncy));
    const int x = cx * PX + 16 * w + k, y = cy * PY + q;
    bool valid = i < total && in_grid(g, z, y, x), all_f = true, any_f = false, own_f = false;
    if (valid) {
        window_flags(lab, g, z, y, x, all_f, any_f);
        own_f = lab[cell_index(g, z, y, x)] == kFluid;
    }
    // per lane: 1 = the cell needs work, 2 = its window is not all fluid
    const uint64_t dn_any = __ballot(valid && any_f), dn_mixed = __ballot(valid && any_f && !all_f);
    const uint64_t up_any = __ballot(valid && own_f), up_mixed = __ballot(valid && own_f && !all_f);
    if (k == 0 && i < total) {
        const int sh = threadIdx.x & 48;   // the group's 16 lanes
        auto mode = [&](uint64_t any, uint64_t mixed) -> uint8_t {
            if (((any >> sh) & 0xffffu) == 0) return kGZero;
            return ((mixed >> sh) & 0xffffu) ? kGGeneral : kGPure;
        };
        mdown[grp] = mode(dn_any, dn_mixed);
        mup[grp] = mode(up_any, up_mixed);
    }
}

// One byte per work item (march_columns order), per kernel: 1 when every
// group of the item's planes is zero for that kernel (down: no window holds
// fluid; up: no fluid cell).  Such an item only writes its zero outputs.
__global__ __launch_bounds__(kBlock) void k_item_zero(Grid g, const uint32_t* __restrict__ mdown,
                                                      const uint32_t* __restrict__ mup, uint8_t* __restrict__ zdown,
                                                      uint8_t* __restrict__ zup) {
    const Columns cl = march_columns(g);
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (i >= cl.count()) return;
    const int cx = i % cl.ncx, cy = (i / cl.ncx) % cl.ncy, z0 = (i / (cl.ncx * cl.ncy)) * cl.chunk;
    const int z1 = min(z0 + cl.chunk, g.nz);
    uint32_t od = 0u, ou = 0u;
    for (int z = z0; z < z1; ++z) {
        const size_t row = (((size_t)z * cl.ncy + cy) * cl.ncx + cx) * 4;   // a plane's 16 mode bytes
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            od |= mdown[row + w];
            ou |= mup[row + w];
        }
    }
    zdown[i] = od == 0u;
    zup[i] = ou == 0u;
}

// A wave's MFMA and pure-kernel operands for all its groups.
template <int KM>
struct MarchCtx {
    static constexpr int P = KM == kMfmaBf16x3 ? kPieces : 1;
    u16x8 a[P][2][2];
    int lofs[8];    // record index of window position j for row 0, relative to a plane buffer
    int oz[8];      // its z offset (-1, 0, 1)
    float kp[8];    // the all-fluid kernel at tap j (0 past tap 26)
    bool one;       // lane group 2: position 27 carries the constant feature
};

template <int KM>
__device__ __forceinline__ MarchCtx<KM> march_ctx(const MfmaW* __restrict__ wm, const CConvW<float>* __restrict__ w) {
    MarchCtx<KM> c;
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15, wv = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < MarchCtx<KM>::P; ++p)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const uint16_t* src = KM == kMfmaF16 ? &wm->f16[mb][ks][lane][0] : &wm->bf16[p][mb][ks][lane][0];
                c.a[p][mb][ks] = *reinterpret_cast<const u16x8*>(src);
            }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int o = 16 * (j >> 2) + 4 * g + (j & 3);
        const int oc = min(o, kTaps - 1);
        const int oy = (oc / 3) % 3 - 1, ox = oc % 3 - 1;
        c.oz[j] = oc / 9 - 1;
        c.lofs[j] = (1 + oy) * PHX + 16 * wv + n + 1 + ox;
        c.kp[j] = o < kTaps ? w->Kpure[kFluid][o] : 0.0f;
    }
    c.one = g == 2;
    return c;
}

__device__ __forceinline__ uint32_t bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ float fbits(uint32_t v) { return __uint_as_float(v); }

// The partial CConv sum of the lane for group q (row q) of output plane c:
// sum over its eight window positions of K_t(cell) r(cell + t).
template <int KM>
__device__ __forceinline__ float march_group(const uint2* ring, const int (&pb)[8], int q, uint32_t mode,
                                             const MarchCtx<KM>& c) {
    if (mode == kGZero) return 0.0f;
    uint2 rv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) rv[j] = ring[pb[j] + c.lofs[j] + q * PHX];
    float pa = 0.0f, pb2 = 0.0f;   // two chains of four
    if (mode == kGPure) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            pa = fmaf(c.kp[j], fbits(rv[j].x), pa);
            pb2 = fmaf(c.kp[j + 4], fbits(rv[j + 4].x), pb2);
        }
        return pa + pb2;
    }
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u16x8 B[2];
    B[0] = __builtin_bit_cast(u16x8, (u32x4){rv[0].y, rv[1].y, rv[2].y, rv[3].y});
    B[1] = __builtin_bit_cast(u16x8, (u32x4){rv[4].y, rv[5].y, rv[6].y, c.one ? feat_one<KM>() : rv[7].y});
    f32x4 acc[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        acc[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int p = 0; p < MarchCtx<KM>::P; ++p)
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
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        pa = fmaf(acc[0][j], fbits(rv[j].x), pa);
        pb2 = fmaf(acc[1][j], fbits(rv[j + 4].x), pb2);
    }
    return pa + pb2;
}

// Sum of a value over the lane pairs (l, l ^ 32) and (l, l ^ 16), given per
// lane for four groups: returns for lane (g, n) the total over the four lane
// groups of group g's value at n.  v_permlane32_swap exchanges the upper half
// of its first operand with the lower half of its second, v_permlane16_swap
// the odd 16-lane rows of the first with the even rows of the second.
__device__ __forceinline__ float reduce_scatter4(const float (&p)[4]) {
    const auto s0 = __builtin_amdgcn_permlane32_swap(bits(p[0]), bits(p[2]), false, false);
    const auto s1 = __builtin_amdgcn_permlane32_swap(bits(p[1]), bits(p[3]), false, false);
    const float a0 = fbits(s0[0]) + fbits(s0[1]);   // lanes < 32: group 0, else group 2
    const float a1 = fbits(s1[0]) + fbits(s1[1]);   // lanes < 32: group 1, else group 3
    const auto t = __builtin_amdgcn_permlane16_swap(bits(a0), bits(a1), false, false);
    return fbits(t[0]) + fbits(t[1]);
}

// One output plane's CConv for the lane's cell: the four groups of the wave,
// then the reduce-scatter.  modes: the wave's four group modes (one byte each).
template <int KM>
__device__ __forceinline__ float march_cconv(const uint2* ring, int c, uint32_t modes, const MarchCtx<KM>& mc) {
    int pb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) pb[j] = ((c + mc.oz[j]) & 3) * kPlaneP;
    if (modes == 0) return 0.0f;   // every group zero (wave-uniform)
    float part[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) part[q] = march_group<KM>(ring, pb, q, (modes >> (8 * q)) & 0xffu, mc);
    return reduce_scatter4(part);
}

// The record of one staged cell: input value and features (outside the grid:
// zero input, solid features).
template <int KM>
__device__ __forceinline__ uint2 march_record(float r, uint8_t l) {
    return uint2{bits(l == kFluid ? r : 0.0f), feat_word<KM, true>(l)};
}

// The staged elements of a thread in a footprint's plane (element i = thread
// + k kBlock, clamped to the last one): offset y nx + x inside a plane and
// whether the column lies in the grid.  Formed once per footprint; a plane's
// loads then only add its z offset.
struct StageElems {
    static constexpr int K = (kPlane + kBlock - 1) / kBlock;
    uint32_t off[K];
    bool in[K];
};

__device__ __forceinline__ StageElems stage_elems(Grid g, int x0, int y0) {
    StageElems e;
#pragma unroll
    for (int k = 0; k < StageElems::K; ++k) {
        const int i = min((int)threadIdx.x + k * kBlock, kPlane - 1);
        const int yy = y0 + i / PHX - 1, xx = x0 + i % PHX - 1;
        e.in[k] = yy >= 0 && yy < g.ny && xx >= 0 && xx < g.nx;
        e.off[k] = e.in[k] ? (uint32_t)yy * g.nx + xx : 0u;
    }
    return e;
}

struct RLab {   // CConv input and label of one staged cell
    float r;
    uint8_t l;
};

// x1 = CConv_1^1(r) and r^2 = Pool(x1) (the input masked to fluid).  Plane-
// marching: step s writes plane s into the ring, issues the loads of plane
// s + 2, then forms output plane s - 1.  The 2x2x2 pool sums x pairs with a
// DPP quad permutation, y pairs with a permlane swap and z pairs in a
// register (chunks start on even planes and have even length).
template <int KM>
__global__ __launch_bounds__(kBlock) NPS_WAVES_PER_EU(KM == kMfmaBf16x3 ? 3 : 4) void k_down_l1m(const uint8_t* __restrict__ lab, Grid g,
                                                     const float* __restrict__ r, float* __restrict__ x1,
                                                     float* __restrict__ rnext, const CConvW<float>* __restrict__ w,
                                                     const MfmaW* __restrict__ wm, const State* st,
                                                     const uint32_t* __restrict__ gmode,
                                                     const uint8_t* __restrict__ izero) {
    __shared__ uint2 ring[4 * kPlaneP];
    const int done = st->done;   // tested once the first loads are out
    const MarchCtx<KM> mc = march_ctx<KM>(wm, w);
    const Columns cl = march_columns(g);
    const Grid gc = coarser(g);
    const int lane = threadIdx.x & 63, gq = lane >> 4, n = lane & 15;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t pstride = (uint32_t)g.ny * (uint32_t)g.nx;
    StageElems se;
    auto plane = [&](int zz) {
        Batch<kPlane, RLab> bt;
        const bool zin = zz >= 0 && zz < g.nz;
        const uint32_t base = zin ? (uint32_t)zz * pstride : 0u;
#pragma unroll
        for (int k = 0; k < StageElems::K; ++k) {
            const bool in = zin && se.in[k];
            const size_t q = base + se.off[k];
            bt.v[k] = RLab{*at_or(r, q, in, pad_zero<float>()), *at_or(lab, q, in, g_pad_solid)};
        }
        return bt;
    };
    bool first = true;
    const bool xs = gridDim.x % kXcds == 0;
    const int xcd = xs ? (int)(blockIdx.x % kXcds) : 0, lstep = xs ? (int)gridDim.x / kXcds : (int)gridDim.x;
    const int per = cl.ncx * cl.ncy, nzl = xs ? (cl.ncz - xcd + kXcds - 1) / kXcds : cl.ncz, zmul = xs ? kXcds : 1;
    for (int li = xs ? (int)blockIdx.x / kXcds : (int)blockIdx.x; li < per * nzl; li += lstep) {
        const int zc = xcd + zmul * (li / per), rest = li % per;
        const int cx = rest % cl.ncx, cy = rest / cl.ncx, z0 = zc * cl.chunk;
        const int x0 = cx * PX, y0 = cy * PY, z1 = min(z0 + cl.chunk, g.nz);
        const int xx = x0 + 16 * wv + n, yy = y0 + gq;
        const bool col = xx < g.nx && yy < g.ny;
        if (izero[zc * per + rest]) {   // no window holds fluid: x1 is zero (read nowhere), and so is the pool
            if (done) return;
            for (int c = z0 + 1; c < z1; c += 2)
                if (((n | gq) & 1) == 0 && col) rnext[cell_index(gc, c >> 1, yy >> 1, xx >> 1)] = 0.0f;
            continue;
        }
        const uint32_t* mrow = gmode + ((size_t)cy * cl.ncx + cx) * 4 + wv;   // + z * ncy * ncx * 4 words
        const size_t mstride = (size_t)cl.ncy * cl.ncx * 4;
        const uint32_t own_off = col ? (uint32_t)yy * g.nx + xx : 0u;
        se = stage_elems(g, x0, y0);
        // planes are loaded two steps ahead of their staging
        auto preA = plane(z0 - 1);
        auto preB = plane(z0);
        if (first) {
            __asm__ volatile("" ::: "memory");   // the loads stay above the test
            if (done) return;
            first = false;
        }
        __syncthreads();   // the previous footprint's reads of the ring are done
        float pool = 0.0f;
        auto step = [&](int s, auto& pre) {
            uint2* buf = ring + (s & 3) * kPlaneP;
            put_batch(pre, [&](int i, RLab e) { buf[i] = march_record<KM>(e.r, e.l); });
            if (s + 2 <= z1) pre = plane(s + 2);
            const int c = s - 1;
            const uint32_t modes = c >= z0 ? __builtin_amdgcn_readfirstlane(mrow[(size_t)c * mstride]) : 0u;
            __syncthreads();   // plane s is staged
            if (c < z0) return;
            const float out = march_cconv<KM>(ring, c, modes, mc);
            if (col) x1[(size_t)c * pstride + own_off] = out;
            // 2x2x2 pool: x pair (DPP quad_perm [1,0,3,2]), y pair (rows 2k, 2k+1)
            const float px = out + fbits(__builtin_amdgcn_update_dpp(0u, bits(out), 0xB1, 0xF, 0xF, false));
            const auto t = __builtin_amdgcn_permlane16_swap(bits(px), bits(px), false, false);
            pool += fbits(t[0]) + fbits(t[1]);
            if (c & 1) {
                if (((n | gq) & 1) == 0 && col)
                    rnext[cell_index(gc, c >> 1, yy >> 1, xx >> 1)] = pool * 0.125f;
                pool = 0.0f;
            }
        };
        // z1 - z0 is even, so the steps z0 - 1 .. z1 come in pairs
        for (int s = z0 - 1; s <= z1; s += 2) {
            step(s, preA);
            step(s + 1, preB);
        }
    }
}

// Level-1 up: dhat = (c1 x1 + c2 CConv_2^1(Interp(x^2))) / ||r|| on fluid
// cells (0 elsewhere) and the state's ndots partial dots of dhat with ad0..
// The interpolation (trilinear, cell-centred, edges clamped) is formed while
// staging each fine plane, from the two coarse planes it lies between, kept
// in a ring of three LDS planes of 34 x 4 coarse cells (the footprint's
// coarse cells with a one-cell border, coordinates clamped into the coarse
// grid, which is the interpolation's edge rule).
constexpr int kCX = PX / 2 + 2, kCY = PY / 2 + 2, kCPlane = kCX * kCY;
static_assert(kCPlane <= kBlock, "one coarse cell per thread");

template <int ND>
struct UpCell {   // operands of the lane's own cell for one output plane
    float x1;
    float ad[ND > 0 ? ND : 1];
};

// ND: the most dots the state can ask for (NPSDO: n_ortho; PCG 1; flexible
// PCG 2; 0 for the hook and the symmetric variant); HOOK: the parity hook
// (no scaling, no dots).
template <int KM, bool HOOK, int ND>
__global__ __launch_bounds__(kBlock) NPS_WAVES_PER_EU(KM == kMfmaBf16x3 ? 3 : 4) void k_up_l1m(const uint8_t* __restrict__ lab, Grid g,
                                                   const float* __restrict__ xc, const float* __restrict__ x1,
                                                   float* __restrict__ dhat, const CConvW<float>* __restrict__ w,
                                                   const MfmaW* __restrict__ wm, const State* st,
                                                   double* __restrict__ partials, const float* __restrict__ ad0,
                                                   const float* __restrict__ ad1, const float* __restrict__ ad2,
                                                   const float* __restrict__ ad3, const uint32_t* __restrict__ gmode,
                                                   const uint8_t* __restrict__ izero) {
    static_assert(!HOOK || ND == 0, "the hook forms no dots");
    __shared__ uint2 ring[4 * kPlaneP];
    __shared__ float csh[3][kCPlane];
    const int done = st->done;
    const float c1 = (float)st->c1[0], c2 = (float)st->c2[0];
    const float scale = HOOK ? 1.0f : (float)st->scale;
    const int ndots = HOOK || st->sym ? 0 : min(st->ndots, ND);   // the symmetric variant dots after P^T
    const MarchCtx<KM> mc = march_ctx<KM>(wm, w);
    const Columns cl = march_columns(g);
    const Grid gc = coarser(g);
    const int lane = threadIdx.x & 63, gq = lane >> 4, n = lane & 15;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float* adp[kMaxOrtho] = {ad0, ad1, ad2, ad3};
    const uint32_t fluid_word = feat_word<KM, true>(kFluid);
    double v[kRedWidth] = {0.0, 0.0, 0.0, 0.0};
    const uint32_t pstride = (uint32_t)g.ny * (uint32_t)g.nx, cstride = (uint32_t)gc.ny * (uint32_t)gc.nx;
    StageElems se;
    // per staged element: its four coarse cells (rows ly, lyn x columns lx, lxn of
    // the staged coarse block, one byte each), formed once per footprint
    uint32_t ipos[StageElems::K];
    uint32_t coff = 0;   // the thread's coarse cell (jy, jx) of the staged block, clamped
    // staged element i of a plane: fine (y0 - 1 + i / PHX, x0 - 1 + i % PHX)
    auto labels = [&](int zz) {
        Batch<kPlane, uint8_t> bt;
        const bool zin = zz >= 0 && zz < g.nz;
        const uint32_t base = zin ? (uint32_t)zz * pstride : 0u;
#pragma unroll
        for (int k = 0; k < StageElems::K; ++k) {
            const bool in = zin && se.in[k];
            bt.v[k] = *at_or(lab, (size_t)base + se.off[k], in, g_pad_solid);
        }
        return bt;
    };
    // coarse plane m (clamped) of the footprint
    auto coarse = [&](int m) {
        const int jz = min(max(m, 0), gc.nz - 1);
        return xc[(size_t)jz * cstride + coff];
    };
    auto put_coarse = [&](int m, float val) {
        if (threadIdx.x < kCPlane) csh[(m + 3) % 3][threadIdx.x] = val;
    };
    // the lane cell's operands of output plane zz (an unused dot slot reads x1)
    auto cell_ops = [&](int zz, uint32_t own_off) {
        const size_t q = (size_t)zz * pstride + own_off;
        UpCell<ND> u;
        u.x1 = x1[q];
#pragma unroll
        for (int j = 0; j < ND; ++j) u.ad[j] = (j < ndots ? adp[j] : x1)[q];
        return u;
    };
    bool first = true;
    const bool xs = gridDim.x % kXcds == 0;
    const int xcd = xs ? (int)(blockIdx.x % kXcds) : 0, lstep = xs ? (int)gridDim.x / kXcds : (int)gridDim.x;
    const int per = cl.ncx * cl.ncy, nzl = xs ? (cl.ncz - xcd + kXcds - 1) / kXcds : cl.ncz, zmul = xs ? kXcds : 1;
    for (int li = xs ? (int)blockIdx.x / kXcds : (int)blockIdx.x; li < per * nzl; li += lstep) {
        const int zc = xcd + zmul * (li / per), rest = li % per;
        const int cx = rest % cl.ncx, cy = rest / cl.ncx, z0 = zc * cl.chunk;
        const int x0 = cx * PX, y0 = cy * PY, z1 = min(z0 + cl.chunk, g.nz);
        const int xx = x0 + 16 * wv + n, yy = y0 + gq;
        const bool col = xx < g.nx && yy < g.ny;
        if (izero[zc * per + rest]) {   // no fluid cell: the output is zero, the dots get nothing
            if (done) return;
            if (col)
                for (int c = z0; c < z1; ++c) dhat[(size_t)c * pstride + (uint32_t)yy * g.nx + xx] = 0.0f;
            continue;
        }
        const int own = (gq + 1) * PHX + 16 * wv + n + 1;
        const uint32_t own_off = col ? (uint32_t)yy * g.nx + xx : 0u;
        const uint32_t* mrow = gmode + ((size_t)cy * cl.ncx + cx) * 4 + wv;
        const size_t mstride = (size_t)cl.ncy * cl.ncx * 4;
        const int m0 = z0 / 2;
        se = stage_elems(g, x0, y0);
        {
            const int i = min((int)threadIdx.x, kCPlane - 1);
            const int jy = min(max(y0 / 2 - 1 + i / kCX, 0), gc.ny - 1), jx = min(max(x0 / 2 - 1 + i % kCX, 0), gc.nx - 1);
            coff = (uint32_t)jy * gc.nx + jx;
        }
#pragma unroll
        for (int k = 0; k < StageElems::K; ++k) {
            // along each axis the own coarse cell f >> 1 (weight 3/4) and its
            // neighbour on f's side (1/4), as indices into the staged block
            const int i = min((int)threadIdx.x + k * kBlock, kPlane - 1);
            const int fy = y0 + i / PHX - 1, fx = x0 + i % PHX - 1;
            const int ly = (fy >> 1) - (y0 / 2 - 1), lyn = (fy & 1) ? ly + 1 : ly - 1;
            const int lx = (fx >> 1) - (x0 / 2 - 1), lxn = (fx & 1) ? lx + 1 : lx - 1;
            ipos[k] = se.in[k] ? (uint32_t)(ly * kCX + lx) | (uint32_t)(ly * kCX + lxn) << 8 |
                                     (uint32_t)(lyn * kCX + lx) << 16 | (uint32_t)(lyn * kCX + lxn) << 24
                               : 0u;
        }
        // loads run two steps ahead: fine-plane labels, the coarse plane the
        // next even step writes, the cell operands of the plane a step computes
        const float cm0 = coarse(m0 - 1), cm1 = coarse(m0);
        float cpre = coarse(m0 + 1);
        auto lA = labels(z0 - 1);
        auto lB = labels(z0);
        UpCell<ND> oA, oB;
        if (first) {
            __asm__ volatile("" ::: "memory");
            if (done) return;
            first = false;
        }
        __syncthreads();   // the previous footprint's reads of the ring and the coarse planes are done
        put_coarse(m0 - 1, cm0);
        put_coarse(m0, cm1);
        __syncthreads();
        auto step = [&](int s, auto& lpre, UpCell<ND>& ops) {
            // stage fine plane s: interpolation from coarse planes s >> 1 and its neighbour on s's side
            uint2* buf = ring + (s & 3) * kPlaneP;
            const bool zin = s >= 0 && s < g.nz;
            const int jz = s >> 1, jzn = (s & 1) ? jz + 1 : jz - 1;   // virtual planes, clamped when staged
            const float* cz0 = csh[(jz + 3) % 3];
            const float* cz1 = csh[(jzn + 3) % 3];
#pragma unroll
            for (int k = 0; k < StageElems::K; ++k) {
                const int i = threadIdx.x + k * kBlock;
                float val = 0.0f;
                if (zin && se.in[k] && i < kPlane) {
                    const uint32_t w = ipos[k];
                    const int a00 = w & 255, a01 = (w >> 8) & 255, a10 = (w >> 16) & 255, a11 = w >> 24;
                    auto bil = [&](const float* p) {
                        const float a = fmaf(0.25f, p[a01] - p[a00], p[a00]);
                        const float b = fmaf(0.25f, p[a11] - p[a10], p[a10]);
                        return fmaf(0.25f, b - a, a);
                    };
                    const float v0 = bil(cz0), v1 = bil(cz1);
                    val = fmaf(0.25f, v1 - v0, v0);
                }
                // the CConv_2 input is not masked (only the level's output is)
                buf[i] = uint2{bits(val), feat_word<KM, true>(lpre.v[k])};
            }
            // an even step writes coarse plane (s >> 1) + 1, which the odd fine plane s + 1 needs
            if (!(s & 1) && s < z1) {
                put_coarse((s >> 1) + 1, cpre);
                if (s + 2 < z1) cpre = coarse((s >> 1) + 2);
            }
            if (s + 2 <= z1) lpre = labels(s + 2);
            const int c = s - 1;
            const uint32_t modes = c >= z0 ? __builtin_amdgcn_readfirstlane(mrow[(size_t)c * mstride]) : 0u;
            __syncthreads();   // plane s (and the coarse plane) staged
            if (c >= z0) {
                const float x2 = march_cconv<KM>(ring, c, modes, mc);
                const bool fl = ring[(c & 3) * kPlaneP + own].y == fluid_word;
                const float out = fl ? (c1 * ops.x1 + c2 * x2) * scale : 0.0f;
                if (col) {
                    dhat[(size_t)c * pstride + own_off] = out;
#pragma unroll
                    for (int j = 0; j < ND; ++j)
                        if (j < ndots) v[j] = fma((double)out, (double)ops.ad[j], v[j]);
                }
            }
            if (s + 1 < z1) ops = cell_ops(s + 1, own_off);   // plane s + 1, formed at step s + 2
        };
        // z1 - z0 is even, so the steps z0 - 1 .. z1 come in pairs
        for (int s = z0 - 1; s <= z1; s += 2) {
            step(s, lA, oA);
            step(s + 1, lB, oB);
        }
    }
    if (!HOOK && !done) block_partials<kBlock>(v, partials);
}

}  // namespace nps
