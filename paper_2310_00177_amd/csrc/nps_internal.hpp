// Internal declarations shared by the HIP kernels and the C-ABI host code.
//
// Notation (arXiv 2310.00177): level l = 1..L of the network (Alg. 2), the
// image I^l of level l stored as two integer channel counts per cell (fluid,
// air: the solid channel is implied because the three channels of an
// average-pooled one-hot image sum to one), Krylov vectors of Alg. 1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace nps {

constexpr int kMaxLevels = 6;   // counts of level 6 reach 8^5 = 32768 < 2^16
constexpr int kMaxOrtho = 4;
constexpr int kRing = kMaxOrtho + 1;
constexpr int kTaps = 27;
constexpr int kRedWidth = 4;          // doubles reduced per block at most
constexpr int kMaxRedBlocks = 16384;  // cap on blocks of reducing kernels (partials per value)
constexpr int kXcds = 8;              // accelerator dies; workgroups are dealt to them round-robin
constexpr int kBlock = 256;           // threads per block of the stencil kernels
constexpr int kCtlBlock = 1024;       // threads of the control kernel
constexpr int kStoreMaxCells = 32768; // levels at most this large keep their kernels K in HBM
constexpr int kBottomMaxCells = 512;  // levels at most this large run in one workgroup
constexpr int kMfmaMaxLevel = 3;      // counts <= 64: exact in bf16 and fp16
constexpr int kPieces = 3;            // bf16 pieces of an fp32 weight (sum is exact to fp32)

enum Label : uint8_t { kFluid = 0, kAir = 1, kSolid = 2 };

// How a level generates its per-cell kernels.
enum KMode : int { kVector = 0, kStored = 1, kMfmaBf16x3 = 2, kMfmaBf16 = 3, kMfmaF16 = 4 };

struct Grid {
    int nz, ny, nx;
};

__host__ __device__ inline size_t ncells(Grid g) { return (size_t)g.nz * g.ny * g.nx; }
__host__ __device__ inline Grid coarser(Grid g) { return Grid{g.nz / 2, g.ny / 2, g.nx / 2}; }

// A CConv block in "count form".  With n_c(q) the number of level-1 cells of
// label c inside coarse cell q (1 or 0 at level 1), the per-cell kernel of
// Sec. "Architecture" is
//   K_t(p) = C[t] + sum_o D[o][t][0] n_fluid(p+o) + D[o][t][1] n_air(p+o),
// where C[t] = B_t + sum_o W[t,solid,o] and D = (W[t,c,o] - W[t,solid,o]) / 8^(l-1)
// (the solid channel is eliminated with sum_c I_c = 1, which also holds for
// the solid padding).  Kpure[c] is the kernel of a window made only of pure
// label-c cells.
template <class T>
struct CConvW {
    T C[kTaps];
    T D[kTaps][kTaps][2];   // [window offset o][tap t][fluid, air]
    T Kpure[3][kTaps];
};

// The same block as the A operand of v_mfma_f32_16x16x32_{bf16,f16}:
// A[m][k] with m = tap (27 padded to 32), k = feature (2o + c for the 54
// counts, 54 the constant 1 carrying C, 55..63 zero), pre-arranged per lane
// (lane l holds m = 16 mb + l % 16, k = 32 ks + 8 (l / 16) + i, i < 8).
// bf16[p] are the three bf16 pieces of the fp32 value (p = 0 alone is the
// bf16 rounding), f16 the fp16 rounding.
struct MfmaW {
    uint16_t bf16[kPieces][2][2][64][8];   // [piece][mb][ks][lane][i]
    uint16_t f16[2][2][64][8];
};

// Aff block (Sec. "Architecture"): Bbar + (1/(27 n_l)) sum_p sum_c sum_o Wbar[c,o] I_c(p+o).
struct AffW {
    double w[3][kTaps];
    double b;
};

// Device-side solver state (lives in the caller's workspace).  Written only
// by the one-block control kernel; read by every other kernel at entry.
struct State {
    double bb;                 // ||b||^2 over fluid cells
    double tol2bb;             // tol^2 ||b||^2
    double rr;                 // ||b - A x||^2 of the current iterate
    double scale;              // 1 / ||r||: the network input normalisation
    double alpha;              // step length of the pending direction
    double beta[kMaxOrtho];    // orthogonalisation coefficients of this iteration
    double dAd[kRing];         // d . A d per ring slot
    double rd;                 // r . d of the newest direction
    double c1[kMaxLevels], c2[kMaxLevels];
    int iter;                  // completed iterations
    int xcur;                  // which of the two solution buffers holds the current iterate
    int nprev;                 // previous directions to orthogonalise against
    int pending;               // 1: x += alpha d_(iter+1) not yet applied
    int done;                  // 1: stop, kernels become no-ops
    int status;                // nps_status
    int n_fluid, bad_label, nonfinite;
    int max_iter, fixed, n_ortho;
    int method;                // nps_method
    int sym;                   // 1: preconditioner P^T o P (the symmetric variant)
    int ndots;                 // partial dots the level-1 up kernel forms this iteration
    double rho, rho_prev;      // PCG forms: r . P(r)/||r|| of this and of the previous iteration
    int nlive;                 // work items of the 7-point kernels that hold fluid
};

// Tile geometry of the stencil kernels: TX x TY x TZ cells, one per thread.
// A wave covers one z-plane of the tile: 16 x-consecutive cells in 4 rows,
// i.e. four 16-cell groups, the N dimension of a 16x16x32 MFMA.
constexpr int TX = 16, TY = 4, TZ = 4;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int kHalo = HX * HY * HZ;
static_assert(TX * TY * TZ == kBlock, "one cell per thread");

// LDS arrays filled by a batched staging hold whole rounds of kBlock elements
// (the surplus of the last round lands in the padding).
constexpr int pad_block(int n) { return (n + kBlock - 1) / kBlock * kBlock; }
constexpr int kHaloP = pad_block(kHalo);

struct Tiles {
    int ntx, nty, ntz;
    __host__ __device__ int count() const { return ntx * nty * ntz; }
};

__host__ __device__ inline Tiles tiles_of(Grid g) {
    return Tiles{(g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, (g.nz + TZ - 1) / TZ};
}

// Grid of a tile kernel: one block per tile up to kMaxRedBlocks, rounded up
// to a multiple of kXcds so that every die owns an equal, contiguous range of
// tiles (see tile_span).
inline int tile_blocks(int tiles) {
    int g = tiles < 1 ? 1 : tiles;
    if (g > kXcds) g = (g + kXcds - 1) / kXcds * kXcds;
    return g < kMaxRedBlocks ? g : kMaxRedBlocks;
}

inline int red_blocks(int work_blocks) {
    return work_blocks < kMaxRedBlocks ? (work_blocks > 0 ? work_blocks : 1) : kMaxRedBlocks;
}

// Host-visible copy of the stopping decision, written by the control kernel.
struct HostFlags {
    int done;
    int iter;
};

// Control-kernel stages.
enum Stage : int { kStageScan = 0, kStageAff = 1, kStageResidual = 2, kStageDots = 3, kStageStep = 4, kStageLoss = 5 };

}  // namespace nps
