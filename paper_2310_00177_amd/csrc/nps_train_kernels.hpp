// Backward kernels of the network (training loss of Sec. "Training").
//
// With g the gradient of a CConv block's output, r its input, I the image:
//   dL/dB_t      = sum_p g(p) r(p + a_t)                        (= U_t)
//   dL/dW[t,c,o] = sum_p g(p) r(p + a_t) I_c(p + o)
//   dL/dr(q)     = sum_t K_t(q - a_t) g(q - a_t)                 (transposed apply)
// In count form I_c = n_c / 8^(l-1) for fluid and air, and the solid channel
// follows from sum_c I_c = 1 (also for the solid padding):
//   dL/dW[t,solid,o] = U_t - dL/dW[t,fluid,o] - dL/dW[t,air,o].
// Each block accumulates the 27 x 55 sums (54 counts and the constant 1) of
// its tiles and writes them as one partial; a reduce kernel sums the partials
// in block order into the double gradient blob.  All levels use kernels K
// formed at setup (tap-major), so the transposed apply is a gather.
#pragma once

#include "nps_kernels.hpp"

#include <type_traits>

namespace nps {

constexpr int kFeat = 2 * kTaps + 1;            // 54 counts + the constant
constexpr int kWGrad = kTaps * kFeat;           // 1485 sums per CConv block
constexpr int kWPart = kWGrad + 3;              // + dL/dc1, dL/dc2 partials, padding
constexpr int kTrainBlocks = 1024;              // grid of the backward tile kernels
constexpr int kUStride = kBlock + 1;            // padded row of the u table in LDS

// Accumulate this tile's contribution to the 27 x 55 sums.  u_s[t][p] holds
// g(p) r(p + a_t) for the tile's cells (row stride kUStride), img_s the
// haloed image.  Thread i owns sums i, i + kBlock, ...
template <class T, bool L1>
__device__ __forceinline__ void accumulate_wgrad(const T* u_s, const uint32_t* img_s, T (&acc)[(kWGrad + kBlock - 1) / kBlock]) {
    constexpr int NO = (kWGrad + kBlock - 1) / kBlock;
#pragma unroll
    for (int j = 0; j < NO; ++j) {
        const int idx = threadIdx.x + j * kBlock;
        if (idx >= kWGrad) break;
        const int t = idx / kFeat, k = idx % kFeat;
        T s = T(0);
        if (k == kFeat - 1) {
            for (int p = 0; p < kBlock; ++p) s += u_s[t * kUStride + p];
        } else {
            const int o = k >> 1, c = k & 1;
            const int off = halo_off_rt(o);
            for (int p = 0; p < kBlock; ++p) {
                const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                uint32_t n0, n1;
                counts_of<L1>(img_s[halo_base(lx, ly, lz) + off], n0, n1);
                const uint32_t n = c ? n1 : n0;
                if (n) s += u_s[t * kUStride + p] * (T)n;
            }
        }
        acc[j] += s;
    }
}

// Float: the tile's contribution as a matrix product on the matrix cores,
// sums[t][f] += sum_p U[t][p] F[f][p] with U[t][p] = g(p) r(p + a_t) (from
// u_s) and F[f][p] the f-th count feature of cell p (f = 2 o + c: count of
// channel c at window position o; f = 54 the constant 1), contracted over the
// tile's 256 cells four at a time on v_mfma_f32_16x16x4_f32 (exact fp32
// products, fp32 accumulation).  Wave w owns the feature block f = 16 w ..
// 16 w + 15 and both tap blocks; lane (k, n) supplies U[16 mb + n][p0 + k]
// and F[16 w + n][p0 + k].  acc[mb][i] ends as sums[16 mb + 4 k + i][16 w + n].
template <bool L1>
__device__ __forceinline__ void accumulate_wgrad_mfma(const float* u_s, const uint32_t* img_s, f32x4 (&acc)[2]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = lane & 15, k = lane >> 4;
    const int f = 16 * wv + n, o = min(f >> 1, kTaps - 1), ch = f & 1;
    const int off = halo_off_rt(o);
    // unrolled so that several steps' LDS reads are in flight ahead of their MFMAs
#pragma unroll 8
    for (int p0 = 0; p0 < kBlock; p0 += 4) {
        const int p = p0 + k;
        const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
        float b;
        if (f < 2 * kTaps) {
            uint32_t n0, n1;
            counts_of<L1>(img_s[halo_base(lx, ly, lz) + off], n0, n1);
            b = (float)(ch ? n1 : n0);
        } else {
            b = f == 2 * kTaps ? 1.0f : 0.0f;
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int t = 16 * mb + n;
            const float a = t < kTaps ? u_s[t * kUStride + p] : 0.0f;
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[mb], 0, 0, 0);
        }
    }
}

// The same product with bf16 operands and fp32 accumulation (the bf16
// training leg): v_mfma_f32_16x16x32_bf16 contracts 32 cells at a time, lane
// (k, n) supplying U and F at cells p0 + 8 k .. p0 + 8 k + 7 (U rounded to
// nearest even; the counts are small integers, exact).
__device__ __forceinline__ uint16_t bf16_bits_rne(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <bool L1>
__device__ __forceinline__ void accumulate_wgrad_bf16(const float* u_s, const uint32_t* img_s, f32x4 (&acc)[2]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = lane & 15, k = lane >> 4;
    const int f = 16 * wv + n, o = min(f >> 1, kTaps - 1), ch = f & 1;
    const int off = halo_off_rt(o);
#pragma unroll 2
    for (int p0 = 0; p0 < kBlock; p0 += 32) {
        u16x8 b, a[2];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int p = p0 + 8 * k + j;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            float fv;
            if (f < 2 * kTaps) {
                uint32_t n0, n1;
                counts_of<L1>(img_s[halo_base(lx, ly, lz) + off], n0, n1);
                fv = (float)(ch ? n1 : n0);
            } else {
                fv = f == 2 * kTaps ? 1.0f : 0.0f;
            }
            b[j] = bf16_bits_rne(fv);
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const int t = 16 * mb + n;
                a[mb][j] = bf16_bits_rne(t < kTaps ? u_s[t * kUStride + p] : 0.0f);
            }
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[mb]),
                                                              __builtin_bit_cast(bf16x8, b), acc[mb], 0, 0, 0);
    }
}

__device__ __forceinline__ void write_wgrad_partial_mfma(const f32x4 (&acc)[2], double* part, double gc1, double gc2) {
    double* mine = part + (size_t)blockIdx.x * kWPart;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = lane & 15, k = lane >> 4, f = 16 * wv + n;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = 16 * mb + 4 * k + i;
            if (t < kTaps && f < kFeat) mine[t * kFeat + f] = (double)acc[mb][i];
        }
    if (threadIdx.x == 0) {
        mine[kWGrad] = gc1;
        mine[kWGrad + 1] = gc2;
        mine[kWGrad + 2] = 0.0;
    }
}

// How the parameter sums are contracted: per-thread sums on the vector ALU
// (double), fp32 matrix cores (float), bf16 matrix cores with fp32
// accumulation (the bf16 training leg).
enum WgradPath : int { kWgVector = 0, kWgMfma32 = 1, kWgMfmaBf16 = 2 };

// Per-block accumulator of a CConv block's parameter sums.
template <class T, int WP = std::is_same<T, float>::value ? kWgMfma32 : kWgVector>
struct WgradAcc {
    static constexpr bool kMfma = WP != kWgVector;
    static_assert(!kMfma || std::is_same<T, float>::value, "matrix-core sums are float");
    T v[kMfma ? 1 : (kWGrad + kBlock - 1) / kBlock];
    f32x4 m[kMfma ? 2 : 1];
    __device__ __forceinline__ void init() {
        if constexpr (kMfma) {
            m[0] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            m[1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        } else {
#pragma unroll
            for (int j = 0; j < (kWGrad + kBlock - 1) / kBlock; ++j) v[j] = T(0);
        }
    }
    template <bool L1>
    __device__ __forceinline__ void add(const T* u_s, const uint32_t* img_s) {
        if constexpr (WP == kWgMfmaBf16) accumulate_wgrad_bf16<L1>(u_s, img_s, m);
        else if constexpr (WP == kWgMfma32) accumulate_wgrad_mfma<L1>(u_s, img_s, m);
        else accumulate_wgrad<T, L1>(u_s, img_s, v);
    }
};

template <class T>
__device__ __forceinline__ void write_wgrad_partial_vec(const T (&acc)[(kWGrad + kBlock - 1) / kBlock], double* part,
                                           double gc1, double gc2) {
    constexpr int NO = (kWGrad + kBlock - 1) / kBlock;
    double* mine = part + (size_t)blockIdx.x * kWPart;
#pragma unroll
    for (int j = 0; j < NO; ++j) {
        const int idx = threadIdx.x + j * kBlock;
        if (idx < kWGrad) mine[idx] = (double)acc[j];
    }
    if (threadIdx.x == 0) {
        mine[kWGrad] = gc1;
        mine[kWGrad + 1] = gc2;
        mine[kWGrad + 2] = 0.0;
    }
}

template <class T, int WP>
__device__ __forceinline__ void write_wgrad_partial(const WgradAcc<T, WP>& a, double* part, double gc1, double gc2) {
    if constexpr (WgradAcc<T, WP>::kMfma) write_wgrad_partial_mfma(a.m, part, gc1, gc2);
    else write_wgrad_partial_vec<T>(a.v, part, gc1, gc2);
}

// Backward of one up block at level l:  x = c1 x1 + c2 CConv_2(Interp(xc)).
// Given gx = dL/dx: writes gx1 = c1 gx (the x1 share), gr2 = CConv_2^T(c2 gx),
// and (WGRAD) a partial of the CConv_2 parameter sums and of dL/dc1 = gx.x1,
// dL/dc2 = gx.x2.  Level 1 (L1): gx is masked to fluid first.  Without
// WGRAD this is the up block's part of the adjoint P^T (xc, x1, x2 and part
// are not read).
template <class T, bool L1, bool WGRAD, int WP = std::is_same<T, float>::value ? kWgMfma32 : kWgVector>
__global__ __launch_bounds__(kBlock) void k_bwd_up(const void* __restrict__ img, Grid g, const T* __restrict__ gx_in,
                                                   const T* __restrict__ xc, const T* __restrict__ x1,
                                                   const T* __restrict__ x2, const T* __restrict__ k2, const State* st,
                                                   int lvl, T* __restrict__ gx1, T* __restrict__ gr2, double* part) {
    const T c1 = (T)st->c1[lvl], c2 = (T)st->c2[lvl];
    __shared__ uint32_t img_s[kHaloP];
    __shared__ T r_s[WGRAD ? kHaloP : 1];       // Interp(xc): the block's input
    __shared__ T g_s[kHaloP];       // gx (masked at level 1); the block's output gradient is c2 gx
    __shared__ T c_s[WGRAD ? kCoarseTileP : 1];
    __shared__ T u_s[WGRAD ? kTaps * kUStride : 1];
    WgradAcc<T, WP> acc;
    acc.init();
    double gc1 = 0.0, gc2 = 0.0;
    const Tiles tl = tiles_of(g);
    const size_t n = ncells(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    for (TileSpan sp = tile_span(tl.count()); sp.t0 < sp.t1; sp.t0 += sp.step) {
        const TileOrigin o = tile_origin(sp.t0, tl);
        __syncthreads();
        if constexpr (WGRAD) stage_image_interp<L1, kStored, T>(img_s, nullptr, img, r_s, c_s, xc, g, o);
        else stage_image<L1>(img_s, img, g, o);
        for (int i = threadIdx.x; i < kHalo; i += kBlock) {
            const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
            const int xx = o.x0 + hx - 1, yy = o.y0 + hy - 1, zz = o.z0 + hz - 1;
            T v = T(0);
            if (in_grid(g, zz, yy, xx)) {
                const size_t q = cell_index(g, zz, yy, xx);
                v = gx_in[q];
                if (L1 && static_cast<const uint8_t*>(img)[q] != kFluid) v = T(0);
            }
            g_s[i] = v;
        }
        __syncthreads();
        const int xx = o.x0 + lx, yy = o.y0 + ly, zz = o.z0 + lz;
        const bool active = in_grid(g, zz, yy, xx);
        const size_t idx = active ? cell_index(g, zz, yy, xx) : 0;
        const T gxp = g_s[base];
        const T gself = c2 * gxp;    // dL/dx2(p)
        if constexpr (WGRAD)
            for (int t = 0; t < kTaps; ++t) u_s[t * kUStride + threadIdx.x] = active ? gself * r_s[base + halo_off(t)] : T(0);
        if (active) {
            gx1[idx] = c1 * gxp;
            if constexpr (WGRAD) {
                gc1 += (double)gxp * (double)x1[idx];
                gc2 += (double)gxp * (double)x2[idx];
            }
            T s = T(0);
#pragma unroll
            for (int t = 0; t < kTaps; ++t) {
                const int qz = zz - (t / 9 - 1), qy = yy - ((t / 3) % 3 - 1), qx = xx - (t % 3 - 1);
                if (in_grid(g, qz, qy, qx)) s = fma(k2[(size_t)t * n + cell_index(g, qz, qy, qx)], c2 * g_s[base - halo_off(t)], s);
            }
            gr2[idx] = s;
        }
        if constexpr (WGRAD) {
            __syncthreads();
            acc.template add<L1>(u_s, img_s);
        }
    }
    if constexpr (!WGRAD) return;
    // dL/dc partials: block sums
    double v[kRedWidth] = {gc1, gc2, 0.0, 0.0};
    __shared__ double sh[kRedWidth][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int w = 0; w < 2; ++w) v[w] = wave_sum(v[w]);
    __syncthreads();
    if (lane == 0) {
        sh[0][wid] = v[0];
        sh[1][wid] = v[1];
    }
    __syncthreads();
    double b1 = 0.0, b2 = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) {
        b1 += sh[0][i];
        b2 += sh[1][i];
    }
    write_wgrad_partial(acc, part, b1, b2);
}

// Backward of one down block at level l:  x1 = CConv_1(r1).  The output
// gradient is gx1 plus, below the coarsest level, the pool adjoint of the
// next level's input gradient (gr_next / 8 of the parent cell).  Writes
// gr1 = CConv_1^T(g) (unless gr1 is null; at level 1 restricted to fluid,
// where the input was) and (WGRAD) a partial of the parameter sums.
// Without WGRAD this is the down block's part of the adjoint P^T (r1 and
// part are not read).
template <class T, bool L1, bool WGRAD, int WP = std::is_same<T, float>::value ? kWgMfma32 : kWgVector>
__global__ __launch_bounds__(kBlock) void k_bwd_down(const void* __restrict__ img, Grid g, const T* __restrict__ gx1,
                                                     const T* __restrict__ gr_next, const T* __restrict__ r1,
                                                     const T* __restrict__ k1, T* __restrict__ gr1, double* part) {
    __shared__ uint32_t img_s[kHaloP];
    __shared__ T r_s[WGRAD ? kHaloP : 1];
    __shared__ T g_s[kHaloP];
    __shared__ T u_s[WGRAD ? kTaps * kUStride : 1];
    WgradAcc<T, WP> acc;
    acc.init();
    const Tiles tl = tiles_of(g);
    const size_t n = ncells(g);
    const Grid gc = coarser(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    for (TileSpan sp = tile_span(tl.count()); sp.t0 < sp.t1; sp.t0 += sp.step) {
        const TileOrigin o = tile_origin(sp.t0, tl);
        __syncthreads();
        stage_image<L1>(img_s, img, g, o);
        for (int i = threadIdx.x; i < kHalo; i += kBlock) {
            const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
            const int xx = o.x0 + hx - 1, yy = o.y0 + hy - 1, zz = o.z0 + hz - 1;
            T gv = T(0), rv = T(0);
            if (in_grid(g, zz, yy, xx)) {
                const size_t q = cell_index(g, zz, yy, xx);
                gv = gx1[q];
                if (gr_next) gv += gr_next[cell_index(gc, zz >> 1, yy >> 1, xx >> 1)] * T(0.125);
                if constexpr (WGRAD) {
                    rv = r1[q];
                    if (L1 && static_cast<const uint8_t*>(img)[q] != kFluid) rv = T(0);   // input padded with zeros
                }
            }
            g_s[i] = gv;
            if constexpr (WGRAD) r_s[i] = rv;
        }
        __syncthreads();
        const int xx = o.x0 + lx, yy = o.y0 + ly, zz = o.z0 + lz;
        const bool active = in_grid(g, zz, yy, xx);
        const T gself = g_s[base];
        if constexpr (WGRAD)
            for (int t = 0; t < kTaps; ++t) u_s[t * kUStride + threadIdx.x] = active ? gself * r_s[base + halo_off(t)] : T(0);
        if (active && gr1) {
            T s = T(0);
#pragma unroll
            for (int t = 0; t < kTaps; ++t) {
                const int qz = zz - (t / 9 - 1), qy = yy - ((t / 3) % 3 - 1), qx = xx - (t % 3 - 1);
                if (in_grid(g, qz, qy, qx)) s = fma(k1[(size_t)t * n + cell_index(g, qz, qy, qx)], g_s[base - halo_off(t)], s);
            }
            if (L1 && img_s[base] != (uint32_t)kFluid) s = T(0);
            gr1[cell_index(g, zz, yy, xx)] = s;
        }
        if constexpr (WGRAD) {
            __syncthreads();
            acc.template add<L1>(u_s, img_s);
        }
    }
    if constexpr (WGRAD) write_wgrad_partial(acc, part, 0.0, 0.0);
}

// Adjoint of the 2x trilinear upsampling: gc(j) = sum over fine cells f of
// w(f -> j) gf(f).  Along one axis a fine cell f feeds f/2 with 3/4 and its
// neighbour on f's side (clamped) with 1/4, so coarse j collects f = 2j, 2j+1
// (3/4), 2j-1, 2j+2 (1/4), and at the ends the clamped quarter of f = 0 or
// f = 2n-1 once more.
__device__ __forceinline__ int up_adjoint_axis(int j, int nc, int* f, double* w) {
    int m = 0;
    f[m] = 2 * j; w[m++] = 0.75;
    f[m] = 2 * j + 1; w[m++] = 0.75;
    if (j > 0) { f[m] = 2 * j - 1; w[m++] = 0.25; }
    else { f[m] = 0; w[m++] = 0.25; }
    if (j < nc - 1) { f[m] = 2 * j + 2; w[m++] = 0.25; }
    else { f[m] = 2 * nc - 1; w[m++] = 0.25; }
    return m;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_bwd_interp(Grid gcoarse, const T* __restrict__ gf, T* __restrict__ gcout) {
    const Grid gfine{2 * gcoarse.nz, 2 * gcoarse.ny, 2 * gcoarse.nx};
    const size_t n = ncells(gcoarse);
    for (size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (size_t)gridDim.x * kBlock) {
        const int x = (int)(q % gcoarse.nx), y = (int)((q / gcoarse.nx) % gcoarse.ny),
                  z = (int)(q / ((size_t)gcoarse.nx * gcoarse.ny));
        int fx[4], fy[4], fz[4];
        double wx[4], wy[4], wz[4];
        const int mx = up_adjoint_axis(x, gcoarse.nx, fx, wx), my = up_adjoint_axis(y, gcoarse.ny, fy, wy),
                  mz = up_adjoint_axis(z, gcoarse.nz, fz, wz);
        double s = 0.0;
        for (int a = 0; a < mz; ++a)
            for (int bb = 0; bb < my; ++bb)
                for (int c = 0; c < mx; ++c)
                    s += wz[a] * wy[bb] * wx[c] * (double)gf[cell_index(gfine, fz[a], fy[bb], fx[c])];
        gcout[q] = (T)s;
    }
}

// The per-block partials of the parameter sums are reduced in two passes
// of fixed order: k_wgrad_chunks sums each chunk of kWChunk consecutive rows
// into the chunk's first row (in place: no other block reads that chunk),
// then k_wgrad_reduce sums the first rows in chunk order.  One workgroup
// summing every row itself had 12 MB to read per CConv block.
constexpr int kWChunk = 32;

__global__ __launch_bounds__(kBlock) void k_wgrad_chunks(double* __restrict__ part, int nparts) {
    const int idx = blockIdx.y * kBlock + threadIdx.x;   // column
    const int b0 = blockIdx.x * kWChunk, b1 = min(b0 + kWChunk, nparts);
    if (idx >= kWPart) return;
    constexpr int U = 8;
    double s = 0.0;
    for (int b = b0; b < b1; b += U) {
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = b + u < b1 ? part[(size_t)(b + u) * kWPart + idx] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) s += t[u];
    }
    part[(size_t)b0 * kWPart + idx] = s;
}

// Sums the chunk sums (rows 0, kWChunk, 2 kWChunk, ... below nparts) of one
// CConv block's parameter sums into the gradient blob: W[t][c][o] (c =
// fluid, air scaled by 1/8^(l-1); solid from U_t), B[t] = U_t.  Also
// returns dL/dc1, dL/dc2 into dc.
__global__ __launch_bounds__(kBlock) void k_wgrad_reduce(const double* __restrict__ part, int nparts, double scale,
                                                         double* __restrict__ gW, double* __restrict__ gB,
                                                         double* __restrict__ dc) {
    __shared__ double sums[kWPart];
    const int nchunks = (nparts + kWChunk - 1) / kWChunk;
    for (int idx = threadIdx.x; idx < kWPart; idx += kBlock) {
        constexpr int U = 8;
        double s = 0.0;
        for (int c = 0; c < nchunks; c += U) {
            double t[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                t[u] = c + u < nchunks ? part[(size_t)(c + u) * kWChunk * kWPart + idx] : 0.0;
#pragma unroll
            for (int u = 0; u < U; ++u) s += t[u];
        }
        sums[idx] = s;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kTaps * kTaps; idx += kBlock) {   // (t, o)
        const int t = idx / kTaps, o = idx % kTaps;
        const double u = sums[t * kFeat + kFeat - 1];
        const double gf = scale * sums[t * kFeat + 2 * o], ga = scale * sums[t * kFeat + 2 * o + 1];
        gW[(t * 3 + kFluid) * kTaps + o] += gf;
        gW[(t * 3 + kAir) * kTaps + o] += ga;
        gW[(t * 3 + kSolid) * kTaps + o] += u - gf - ga;
    }
    for (int t = threadIdx.x; t < kTaps; t += kBlock) gB[t] += sums[t * kFeat + kFeat - 1];
    if (threadIdx.x == 0 && dc) {
        dc[0] = sums[kWGrad];
        dc[1] = sums[kWGrad + 1];
    }
}

// Image-window sums S[c][o] = sum_p I_c(p + o) of one level (solid padding),
// the derivative of an Aff scalar with respect to its weights times 27 n_l.
// The channels are counts times 8^-(l-1), so the fluid and air sums are
// accumulated as integer counts (exact, in registers); the solid channel
// follows from I_solid = 1 - I_fluid - I_air, which the padding satisfies
// too: S[solid][o] = (cells) - S[fluid][o] - S[air][o].  Every partial is a
// multiple of 8^-(l-1) below 2^32, exact in double, so the sums do not depend
// on their order.
template <bool L1>
__global__ __launch_bounds__(kBlock) void k_image_sums(const void* __restrict__ img, Grid g, double inv_full,
                                                       double* __restrict__ part) {
    const size_t n = ncells(g);
    uint32_t s0[kTaps], s1[kTaps], cells = 0;
#pragma unroll
    for (int o = 0; o < kTaps; ++o) s0[o] = s1[o] = 0u;
    for (size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (size_t)gridDim.x * kBlock) {
        const int x = (int)(p % g.nx), y = (int)((p / g.nx) % g.ny), z = (int)(p / ((size_t)g.nx * g.ny));
        cells += 1u;
#pragma unroll
        for (int o = 0; o < kTaps; ++o) {
            const int qz = z + o / 9 - 1, qy = y + (o / 3) % 3 - 1, qx = x + o % 3 - 1;
            if (in_grid(g, qz, qy, qx)) {
                const size_t q = cell_index(g, qz, qy, qx);
                const uint32_t v = L1 ? (uint32_t)static_cast<const uint8_t*>(img)[q] : static_cast<const uint32_t*>(img)[q];
                uint32_t c0, c1;
                counts_of<L1>(v, c0, c1);
                s0[o] += c0;
                s1[o] += c1;
            }
        }
    }
    // every wave reduces its sums, then one barrier and one thread per sum
    // adds the waves in order
    __shared__ uint32_t sh[kBlock / 64][2 * kTaps + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    auto wave_total = [](uint32_t v) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off, 64);
        return v;
    };
#pragma unroll
    for (int o = 0; o < kTaps; ++o) {
        const uint32_t a = wave_total(s0[o]), b = wave_total(s1[o]);
        if (lane == 0) {
            sh[wid][o] = a;
            sh[wid][kTaps + o] = b;
        }
    }
    const uint32_t c = wave_total(cells);
    if (lane == 0) sh[wid][2 * kTaps] = c;
    __syncthreads();
    for (int o = threadIdx.x; o < kTaps; o += kBlock) {
        uint32_t a = 0u, b = 0u, m = 0u;
        for (int k = 0; k < kBlock / 64; ++k) {
            a += sh[k][o];
            b += sh[k][kTaps + o];
            m += sh[k][2 * kTaps];
        }
        double* dst = part + (size_t)blockIdx.x * 3 * kTaps;
        const double f = (double)a * inv_full, ai = (double)b * inv_full;
        dst[o] = f;
        dst[kTaps + o] = ai;
        dst[2 * kTaps + o] = (double)m - f - ai;
    }
}

// Aff gradients of one level: dL/dWbar = dL/dc * S / (27 n_l), dL/dBbar = dL/dc,
// for Aff_1 (dc[0]) and Aff_2 (dc[1]); S summed from the k_image_sums partials.
// One block per weight entry e = c * 27 + o (81 blocks): the block adds the
// entry's partials (exact, see k_image_sums: the order does not matter) and
// updates its gradient; block 0 also updates Bbar.
__global__ __launch_bounds__(kBlock) void k_aff_grad(const double* __restrict__ spart, int nparts,
                                                     const double* __restrict__ dc, double n27,
                                                     double* __restrict__ gA1, double* __restrict__ gA2) {
    const int e = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) s += spart[(size_t)b * 3 * kTaps + e];
    __shared__ double sh[kBlock / 64];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) t += sh[k];
        gA1[e] += dc[0] * t / n27;   // Wbar[c][o]
        gA2[e] += dc[1] * t / n27;
        if (e == 0) {
            gA1[3 * kTaps] += dc[0];   // Bbar
            gA2[3 * kTaps] += dc[1];
        }
    }
}

// Training loss of one system: res = b - A y on fluid cells; partial ||res||^2,
// and A res (whose scaled negative is dL/dy) written to ares.
template <class T>
__global__ __launch_bounds__(kBlock) void k_train_residual(const uint8_t* __restrict__ lab, Grid g,
                                                           const T* __restrict__ b, const T* __restrict__ y,
                                                           T* __restrict__ res, double* partials) {
    __shared__ uint32_t lab_s[kHaloP];
    __shared__ T y_s[kHaloP];
    const Tiles tl = tiles_of(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    double v[kRedWidth] = {0.0, 0.0, 0.0, 0.0};
    for (TileSpan sp = tile_span(tl.count()); sp.t0 < sp.t1; sp.t0 += sp.step) {
        const TileOrigin o = tile_origin(sp.t0, tl);
        __syncthreads();
        stage_image<true>(lab_s, lab, g, o);
        for (int i = threadIdx.x; i < kHalo; i += kBlock) {
            const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
            const int xx = o.x0 + hx - 1, yy = o.y0 + hy - 1, zz = o.z0 + hz - 1;
            y_s[i] = in_grid(g, zz, yy, xx) ? y[cell_index(g, zz, yy, xx)] : T(0);
        }
        __syncthreads();
        const int xx = o.x0 + lx, yy = o.y0 + ly, zz = o.z0 + lz;
        if (in_grid(g, zz, yy, xx)) {
            const size_t idx = cell_index(g, zz, yy, xx);
            T rv = T(0);
            if (lab_s[base] == (uint32_t)kFluid) rv = b[idx] - apply_A<T, T, uint32_t>(lab_s, y_s, base, HX, HX * HY);
            res[idx] = rv;
            v[0] += (double)rv * (double)rv;
        }
    }
    block_partials<kBlock>(v, partials);
}

// dL/dy = -w A res / ||res|| (A is symmetric), from the residual and its
// norm in st->rr; w weighs the system in a batch mean (1 alone).
template <class T>
__global__ __launch_bounds__(kBlock) void k_train_gy(const uint8_t* __restrict__ lab, Grid g, const T* __restrict__ res,
                                                     const State* st, T* __restrict__ gy, double w) {
    __shared__ uint32_t lab_s[kHaloP];
    __shared__ T r_s[kHaloP];
    const T inv = (T)(-w / sqrt(st->rr));
    const Tiles tl = tiles_of(g);
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int base = halo_base(lx, ly, lz);
    for (TileSpan sp = tile_span(tl.count()); sp.t0 < sp.t1; sp.t0 += sp.step) {
        const TileOrigin o = tile_origin(sp.t0, tl);
        __syncthreads();
        stage_image<true>(lab_s, lab, g, o);
        for (int i = threadIdx.x; i < kHalo; i += kBlock) {
            const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
            const int xx = o.x0 + hx - 1, yy = o.y0 + hy - 1, zz = o.z0 + hz - 1;
            r_s[i] = in_grid(g, zz, yy, xx) ? res[cell_index(g, zz, yy, xx)] : T(0);
        }
        __syncthreads();
        const int xx = o.x0 + lx, yy = o.y0 + ly, zz = o.z0 + lz;
        if (in_grid(g, zz, yy, xx)) gy[cell_index(g, zz, yy, xx)] = inv * apply_A<T, T, uint32_t>(lab_s, r_s, base, HX, HX * HY);
    }
}

// acc = 0 (set) or acc += w ||res|| of the system just evaluated (one thread).
__global__ void k_loss_accumulate(const State* st, double* acc, double w, int set) {
    const double v = w * sqrt(st->rr);
    *acc = set ? 0.0 : *acc + v;
}

}  // namespace nps
