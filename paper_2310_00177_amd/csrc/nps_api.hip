// C-ABI of the neural-preconditioned Poisson solver (declared in include/nps.h).
//
// Host-side responsibilities: argument validation, conversion of the weight
// blob into the count form and the MFMA operand layout the kernels use,
// carving the caller's workspace, the per-solve setup (image pyramid, Aff
// scalars, kernels of the small levels), and the Alg. 1 loop, which enqueues
// one iteration's kernels at a time.  Convergence is decided on the device;
// the host polls a copy of the device state one iteration behind, so the GPU
// never waits for the host.
#include "nps.h"
#include "nps_internal.hpp"
#include "nps_kernels.hpp"
#include "nps_march_kernels.hpp"
#include "nps_train_kernels.hpp"
#include "nps_lanczos_kernels.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

using namespace nps;

struct nps_net {
    int levels = 0;
    char* dev = nullptr;
    size_t off_w64 = 0, off_w32 = 0, off_mfma = 0, off_aff = 0;
    size_t off_wbf = 0, off_wbf32 = 0;   // count form with C and D rounded to bf16 (the bf16 training leg)
    double aff_b[2 * kMaxLevels] = {};   // Bbar of Aff_1^l, Aff_2^l (host copy)
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define NPS_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(NPS_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

#define NPS_TRY(expr)            \
    do {                         \
        const int rc_ = (expr);  \
        if (rc_) return rc_;     \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

Grid level_grid(nps_dims d, int level) {  // level 1 = finest
    const int s = level - 1;
    return Grid{d.nz >> s, d.ny >> s, d.nx >> s};
}

// Positive dims and at most 1e9 cells (cell indices are formed in 32 bits).
int check_grid(nps_dims d) {
    if (d.nz <= 0 || d.ny <= 0 || d.nx <= 0) return fail(NPS_ESHAPE, "dims must be positive");
    if ((double)d.nz * d.ny * d.nx > 1.0e9) return fail(NPS_ESHAPE, "grid too large");
    return NPS_OK;
}

int check_dims(nps_dims d, int levels) {
    if (levels < 2 || levels > kMaxLevels)
        return fail(NPS_EINVAL, "levels must be in [2, %d], got %d", kMaxLevels, levels);
    NPS_TRY(check_grid(d));
    const int m = 1 << (levels - 1);
    if (d.nz % m || d.ny % m || d.nx % m)
        return fail(NPS_ESHAPE, "dims (%d,%d,%d) not divisible by 2^(levels-1) = %d", d.nz, d.ny, d.nx, m);
    return NPS_OK;
}

size_t vec_bytes(int precision) { return precision == NPS_FP64 ? 8 : 4; }
size_t x_bytes(int precision) { return precision == NPS_FP32 ? 4 : 8; }

// How each level evaluates its CConv blocks.
struct Plan {
    int L;
    int lb;                      // first level run by the one-workgroup bottom kernel (L + 1: none)
    int km[kMaxLevels + 2];      // KMode per level
};

// LDS elements the bottom workgroup needs for levels lb..levels (two padded
// slots per level).
size_t bottom_footprint(nps_dims d, int lb, int levels) {
    size_t e = 0;
    for (int l = lb; l <= levels; ++l) e += 2 * (size_t)padded_cells(level_grid(d, l));
    return e;
}

Plan make_plan(nps_dims d, int levels, int precision, bool all_stored = false) {
    Plan p = {};
    p.L = levels;
    p.lb = levels + 1;
    for (int l = 1; l <= levels; ++l) {
        const size_t n = ncells(level_grid(d, l));
        if (all_stored) {   // training: every level keeps its kernels, no one-workgroup bottom
            p.km[l] = kStored;
            continue;
        }
        if (n <= (size_t)kStoreMaxCells) p.km[l] = kStored;
        else if (precision == NPS_FP64 || l > kMfmaMaxLevel) p.km[l] = kVector;
        else if (precision == NPS_FP32) p.km[l] = kMfmaBf16x3;
        else if (precision == NPS_MIXED_BF16) p.km[l] = kMfmaBf16;
        else p.km[l] = kMfmaF16;
        if (l >= 2 && p.lb > levels && n <= (size_t)kBottomMaxCells &&
            bottom_footprint(d, l, levels) <= (size_t)kBottomLds)
            p.lb = l;
    }
    return p;
}

// Workspace carving, shared by nps_workspace_bytes, nps_solve and nps_apply_precond.
struct Layout {
    size_t state, partials;
    size_t dots;   // partials of the up kernel's dots (the next kernel writes partials while reading these)
    size_t counts[kMaxLevels + 1];
    size_t x1[kMaxLevels + 1];
    size_t rb[kMaxLevels + 1];
    size_t k1[kMaxLevels + 1], k2[kMaxLevels + 1];
    size_t dhat, dring[kRing], adring[kRing], x[2], r[2];
    size_t wmode[kMaxLevels + 1][2];   // per-wave CConv modes: [level][down, up (level 1)]
    size_t gmode[2];                   // level 1 on matrix cores: per-group modes [down, up]
    size_t izero[2];                   // and per-item zero flags [down, up]
    size_t live, items;                // 7-point work items: fluid flags, the list of those with fluid
    size_t total;
};

Layout make_layout(nps_dims d, int levels, int precision, int n_ortho, bool solve, bool all_stored = false) {
    Layout L = {};
    const Plan p = make_plan(d, levels, precision, all_stored);
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes);
        return at;
    };
    const size_t s = vec_bytes(precision);
    const size_t n = ncells(level_grid(d, 1));
    L.state = put(sizeof(State));
    L.partials = put(sizeof(double) * kRedWidth * kMaxRedBlocks);
    L.dots = put(sizeof(double) * kRedWidth * kMaxRedBlocks);
    for (int l = 2; l <= levels; ++l) L.counts[l] = put(sizeof(uint32_t) * ncells(level_grid(d, l)));
    for (int l = 1; l <= levels; ++l) L.x1[l] = put(s * ncells(level_grid(d, l)));
    for (int l = 2; l <= levels; ++l) L.rb[l] = put(s * ncells(level_grid(d, l)));
    for (int l = 1; l <= levels; ++l) {
        if (p.km[l] != kStored) continue;
        const size_t nl = ncells(level_grid(d, l));
        L.k1[l] = put(s * kTaps * nl);
        if (l < levels) L.k2[l] = put(s * kTaps * nl);
    }
    for (int l = 1; l <= levels; ++l) {
        const size_t waves = (size_t)tiles_of(level_grid(d, l)).count() * TZ;
        L.wmode[l][0] = put(waves);
        if (l == 1) L.wmode[l][1] = put(waves);
    }
    if (is_mfma(p.km[1])) {
        L.gmode[0] = put(group_mode_bytes(level_grid(d, 1)));
        L.gmode[1] = put(group_mode_bytes(level_grid(d, 1)));
        L.izero[0] = put((size_t)march_columns(level_grid(d, 1)).count());
        L.izero[1] = put((size_t)march_columns(level_grid(d, 1)).count());
    }
    L.dhat = put(s * n);
    if (solve) {
        for (int i = 0; i <= n_ortho; ++i) {
            L.dring[i] = put(s * n);
            L.adring[i] = put(s * n);
        }
        L.x[0] = put(x_bytes(precision) * n);
        L.x[1] = put(x_bytes(precision) * n);
        L.r[0] = put(s * n);   // residuals of alternate iterations (flexible PCG reads both)
        L.r[1] = put(s * n);
        const size_t nitems = (size_t)columns_of(level_grid(d, 1)).count();
        L.live = put(nitems);
        L.items = put(sizeof(uint32_t) * nitems);
    }
    L.total = off;
    return L;
}

// Training (and symmetric-variant) workspace: the base layout with stored
// kernels at every level, plus the adjoint sweep's per-level gradients.
struct TrainLayout {
    Layout base;                 // state, partials, counts, x1, rb (= down inputs), stored K
    size_t xup[kMaxLevels + 1], x2[kMaxLevels + 1];
    size_t gx[kMaxLevels + 1], gx1[kMaxLevels + 1], gr1[kMaxLevels + 1], gr2[kMaxLevels + 1];
    size_t wpart, spart, dc, res;
    size_t y, gy, lacc;          // the batch step: network output, its loss gradient, the loss sum
    size_t dsym;                 // solve with P^T o P: the direction after P^T
    size_t total;
};

constexpr int kSumBlocks = 1024;  // most blocks of k_image_sums (five per CU fit)
int sum_blocks(Grid g) { return (int)std::min<size_t>(kSumBlocks, std::max<size_t>((ncells(g) + kBlock - 1) / kBlock, 1)); }

TrainLayout make_train_layout(nps_dims d, int levels, int precision, bool solve = false, int n_ortho = 0) {
    TrainLayout t = {};
    t.base = make_layout(d, levels, precision, n_ortho, solve, true);
    size_t off = t.base.total;
    auto put = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes);
        return at;
    };
    const size_t s = vec_bytes(precision);
    for (int l = 1; l <= levels; ++l) {
        const size_t nl = ncells(level_grid(d, l));
        if (l >= 2 && l < levels) t.xup[l] = put(s * nl);
        if (l < levels) {
            t.x2[l] = put(s * nl);
            t.gx1[l] = put(s * nl);
            t.gr2[l] = put(s * nl);
        }
        if (l >= 2) {
            t.gx[l] = put(s * nl);
            t.gr1[l] = put(s * nl);
        }
    }
    t.wpart = put(sizeof(double) * kWPart * kTrainBlocks);
    t.spart = put(sizeof(double) * 3 * kTaps * kSumBlocks * levels);
    t.dc = put(sizeof(double) * 2 * levels);
    t.res = put(s * ncells(level_grid(d, 1)));
    t.y = put(s * ncells(level_grid(d, 1)));
    t.gy = put(s * ncells(level_grid(d, 1)));
    t.lacc = put(sizeof(double));
    if (solve) t.dsym = put(s * ncells(level_grid(d, 1)));
    t.total = off;
    return t;
}

int tile_grid(Grid g) { return tile_blocks(tiles_of(g).count()); }

// Grid of a pipelined tile kernel: the blocks that fit on the device at once
// (the kernel's occupancy times the compute units), at most one per tile,
// rounded to a multiple of kXcds; each block then walks its share of tiles.
// Occupancy per kernel and the unit count per device are cached.
template <class K>
int persist_grid_n(K* kern, int items) {
    thread_local std::unordered_map<const void*, int> occ;
    thread_local int units[64] = {0};
    const void* f = reinterpret_cast<const void*>(kern);
    auto it = occ.find(f);
    int nb = 1;
    if (it != occ.end()) {
        nb = it->second;
    } else {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
        occ[f] = nb;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (units[dev] == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1) cu = 1;
        units[dev] = cu;
    }
    const long want = (long)nb * units[dev];
    return tile_blocks((int)std::min<long>(items, want));
}
// Persistent grid of a tile kernel on grid g.
template <class K>
int persist_grid(K* kern, Grid g) {
    return persist_grid_n(kern, tiles_of(g).count());
}
int red_elem_grid(size_t n) { return red_blocks((int)std::min<size_t>((n + kBlock - 1) / kBlock, 1u << 30)); }
int elem_grid(size_t n) { return (int)std::min<size_t>(std::max<size_t>((n + kBlock - 1) / kBlock, 1), 65536); }

// Pinned host memory: a mirror of the device state (read at setup and exit)
// and the stopping flags the control kernel writes every iteration.
struct HostMirror {
    State* state = nullptr;
    HostFlags* flags = nullptr;     // host address
    HostFlags* flags_d = nullptr;   // its device address
};

HostMirror* host_mirror() {
    thread_local HostMirror m;
    if (!m.state) {
        void* p = nullptr;
        if (hipHostMalloc(&p, sizeof(State) + 256, hipHostMallocMapped) != hipSuccess) return nullptr;
        m.state = static_cast<State*>(p);
        m.flags = reinterpret_cast<HostFlags*>(static_cast<char*>(p) + ((sizeof(State) + 63) / 64) * 64);
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, m.flags, 0) != hipSuccess) {
            m.state = nullptr;
            return nullptr;
        }
        m.flags_d = static_cast<HostFlags*>(d);
    }
    return &m;
}

// Optional per-kernel timing: an event pair around every launch.
struct ProfRec {
    const char* name;
    int ev0, ev1;
    double cells;
};
struct Prof {
    bool on = false;
    bool overflow = false;
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    std::vector<ProfRec> recs;
};
thread_local Prof g_prof;
constexpr size_t kMaxProfEvents = 2000000;

int prof_mark(hipStream_t s) {
    Prof& p = g_prof;
    if (p.next >= kMaxProfEvents) {
        p.overflow = true;
        return -1;
    }
    if (p.next == p.pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        p.pool.push_back(e);
    }
    if (hipEventRecord(p.pool[p.next], s) != hipSuccess) return -1;
    return (int)p.next++;
}

// Launch through f(); checks the launch and records timing events if enabled.
template <class F>
int launch(const char* name, double cells, hipStream_t s, F&& f) {
    int e0 = -1;
    if (g_prof.on) e0 = prof_mark(s);
    f();
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(NPS_EDEVICE, "launch of %s failed: %s", name, hipGetErrorString(e));
    if (g_prof.on && e0 >= 0) {
        const int e1 = prof_mark(s);
        if (e1 >= 0) g_prof.recs.push_back(ProfRec{name, e0, e1, cells});
    }
    return NPS_OK;
}

size_t net_sizes(int levels, size_t* o64, size_t* o32, size_t* omf, size_t* oaff, size_t* obf = nullptr,
                 size_t* obf32 = nullptr) {
    const int nb = 2 * levels - 1;
    size_t off = 0;
    *o64 = off;
    off += align256(sizeof(CConvW<double>) * nb);
    if (obf) *obf = off;
    off += align256(sizeof(CConvW<double>) * nb);
    if (obf32) *obf32 = off;
    off += align256(sizeof(CConvW<float>) * nb);
    *o32 = off;
    off += align256(sizeof(CConvW<float>) * nb);
    *omf = off;
    off += align256(sizeof(MfmaW) * nb);
    *oaff = off;
    off += align256(sizeof(AffW) * 2 * (levels - 1));
    return off;
}

// CConv block b: CConv_1^l is b = l - 1 (l = 1..L), CConv_2^l is b = L + l - 1.
int block_down(int l) { return l - 1; }
int block_up(const nps_net* net, int l) { return net->levels + l - 1; }

template <class T>
const CConvW<T>* cconv_block(const nps_net* net, int b) {
    const size_t off = sizeof(T) == 8 ? net->off_w64 : net->off_w32;
    return reinterpret_cast<const CConvW<T>*>(net->dev + off) + b;
}
// The count form rounded to bf16 (values held as doubles or floats).
template <class T>
const CConvW<T>* cconv_block_bf16(const nps_net* net, int b) {
    const size_t off = sizeof(T) == 8 ? net->off_wbf : net->off_wbf32;
    return reinterpret_cast<const CConvW<T>*>(net->dev + off) + b;
}
const MfmaW* mfma_block(const nps_net* net, int b) {
    return reinterpret_cast<const MfmaW*>(net->dev + net->off_mfma) + b;
}
const AffW* aff_block(const nps_net* net, int level, int which) {  // which: 0 -> Aff_1, 1 -> Aff_2
    return reinterpret_cast<const AffW*>(net->dev + net->off_aff) + 2 * (level - 1) + which;
}

// Count form of one CConv block (see CConvW): double precision on the host.
void to_count_form(const double* W, const double* B, int level, CConvW<double>& out) {
    const double s = std::ldexp(1.0, -3 * (level - 1));   // 1 / 8^(l-1)
    auto w = [&](int t, int c, int o) { return W[(t * 3 + c) * kTaps + o]; };
    for (int t = 0; t < kTaps; ++t) {
        double c = B[t];
        for (int o = 0; o < kTaps; ++o) c += w(t, kSolid, o);
        out.C[t] = c;
        double kf = c, ka = c;
        for (int o = 0; o < kTaps; ++o) {
            const double d0 = w(t, kFluid, o) - w(t, kSolid, o);
            const double d1 = w(t, kAir, o) - w(t, kSolid, o);
            out.D[o][t][0] = d0 * s;
            out.D[o][t][1] = d1 * s;
            kf += d0;
            ka += d1;
        }
        out.Kpure[kFluid][t] = kf;
        out.Kpure[kAir][t] = ka;
        out.Kpure[kSolid][t] = c;
    }
}

uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
double bf16_value(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
uint16_t f16_rne(double v) {
    const _Float16 h = (_Float16)(float)v;
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

// The count-form block as the MFMA A operand, in per-lane order (see MfmaW).
void to_mfma(const CConvW<double>& cw, MfmaW& m) {
    for (int mb = 0; mb < 2; ++mb)
        for (int ks = 0; ks < 2; ++ks)
            for (int lane = 0; lane < 64; ++lane)
                for (int i = 0; i < 8; ++i) {
                    const int tap = 16 * mb + lane % 16, k = 32 * ks + 8 * (lane / 16) + i;
                    double v = 0.0;
                    if (tap < kTaps) {
                        if (k < 2 * kTaps) v = cw.D[k / 2][tap][k % 2];
                        else if (k == 2 * kTaps) v = cw.C[tap];
                    }
                    double rest = v;
                    for (int p = 0; p < kPieces; ++p) {
                        const uint16_t h = bf16_rne((float)rest);
                        m.bf16[p][mb][ks][lane][i] = h;
                        rest -= bf16_value(h);
                    }
                    m.f16[mb][ks][lane][i] = f16_rne(v);
                }
}

template <class T>
const T* cptr(void* ws, size_t off) {
    return reinterpret_cast<const T*>(static_cast<char*>(ws) + off);
}
template <class T>
T* mptr(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

uint32_t full_count(int l) { return 1u << (3 * (l - 1)); }

// Image pyramid as counts, Aff scalars, and the stored kernels of small levels.
template <class T>
int run_setup(const nps_net* net, const uint8_t* labels, nps_dims d, const Plan& plan, const Layout& lay,
              void* ws, hipStream_t s, bool bf16w = false) {
    const int L = net->levels;
    State* st = mptr<State>(ws, lay.state);
    double* partials = mptr<double>(ws, lay.partials);
    for (int l = 2; l <= L; ++l) {
        const Grid gin = level_grid(d, l - 1), gout = level_grid(d, l);
        uint32_t* out = mptr<uint32_t>(ws, lay.counts[l]);
        const int grid = elem_grid(ncells(gout));
        if (l == 2)
            NPS_TRY(launch("setup_pool_counts", (double)ncells(gout), s, [&] {
                k_pool_counts<true><<<grid, kBlock, 0, s>>>(labels, gin, out, gout);
            }));
        else
            NPS_TRY(launch("setup_pool_counts", (double)ncells(gout), s, [&] {
                k_pool_counts<false><<<grid, kBlock, 0, s>>>(cptr<uint32_t>(ws, lay.counts[l - 1]), gin, out, gout);
            }));
    }
    auto img = [&](int l) -> const void* {
        return l == 1 ? static_cast<const void*>(labels) : static_cast<const void*>(cptr<uint32_t>(ws, lay.counts[l]));
    };
    for (int l = 1; l < L; ++l) {
        const Grid g = level_grid(d, l);
        const double inv_full = std::ldexp(1.0, -3 * (l - 1));
        const int grid = red_elem_grid(ncells(g));
        if (l == 1)
            NPS_TRY(launch("setup_aff", (double)ncells(g), s, [&] {
                k_aff<true><<<grid, kBlock, 0, s>>>(img(l), g, inv_full, aff_block(net, l, 0), aff_block(net, l, 1), partials);
            }));
        else
            NPS_TRY(launch("setup_aff", (double)ncells(g), s, [&] {
                k_aff<false><<<grid, kBlock, 0, s>>>(img(l), g, inv_full, aff_block(net, l, 0), aff_block(net, l, 1), partials);
            }));
        const double b1 = net->aff_b[2 * (l - 1)], b2 = net->aff_b[2 * (l - 1) + 1];
        NPS_TRY(launch("control", 0, s, [&] {
            k_control<kStageAff><<<1, kCtlBlock, 0, s>>>(st, partials, grid, l - 1, 0, 0, 0, b1, b2, 27.0 * (double)ncells(g),
                                                           nullptr);
        }));
    }
    if (is_mfma(plan.km[1])) {
        const Grid g = level_grid(d, 1);
        const size_t threads = group_mode_bytes(g) * 16;
        NPS_TRY(launch("setup_group_modes", (double)ncells(g), s, [&] {
            k_group_modes<<<(unsigned)((threads + kBlock - 1) / kBlock), kBlock, 0, s>>>(
                labels, g, mptr<uint8_t>(ws, lay.gmode[0]), mptr<uint8_t>(ws, lay.gmode[1]));
        }));
        const int items = march_columns(g).count();
        NPS_TRY(launch("setup_item_zero", (double)items, s, [&] {
            k_item_zero<<<(unsigned)((items + kBlock - 1) / kBlock), kBlock, 0, s>>>(
                g, cptr<uint32_t>(ws, lay.gmode[0]), cptr<uint32_t>(ws, lay.gmode[1]), mptr<uint8_t>(ws, lay.izero[0]),
                mptr<uint8_t>(ws, lay.izero[1]));
        }));
    }
    for (int l = 1; l <= L; ++l) {
        const Grid g = level_grid(d, l);
        const int grid = tile_grid(g);
        int8_t* md = mptr<int8_t>(ws, lay.wmode[l][0]);
        if (l == 1 && is_mfma(plan.km[1])) continue;   // the marching kernels use the group modes
        if (l == 1)
            NPS_TRY(launch("setup_wave_modes", (double)ncells(g), s, [&] {
                k_wave_modes<true><<<grid, kBlock, 0, s>>>(img(l), g, 1u, md, mptr<int8_t>(ws, lay.wmode[l][1]));
            }));
        else
            NPS_TRY(launch("setup_wave_modes", (double)ncells(g), s, [&] {
                k_wave_modes<false><<<grid, kBlock, 0, s>>>(img(l), g, full_count(l), md, nullptr);
            }));
    }
    for (int l = 1; l <= L; ++l) {
        if (plan.km[l] != kStored) continue;
        const Grid g = level_grid(d, l);
        // one thread per (tap, cell) on levels the solve stores; one per cell
        // (its window read once for all taps) on larger ones (training)
        const bool per_cell = ncells(g) > (size_t)kStoreMaxCells;
        const int grid = elem_grid((per_cell ? 1 : (size_t)kTaps) * ncells(g));
        for (int which = 0; which < (l < L ? 2 : 1); ++which) {
            T* out = mptr<T>(ws, which == 0 ? lay.k1[l] : lay.k2[l]);
            const int blk = which == 0 ? block_down(l) : block_up(net, l);
            const CConvW<double>* w = bf16w ? cconv_block_bf16<double>(net, blk) : cconv_block<double>(net, blk);
            auto go = [&](auto l1, auto tg) {
                constexpr bool L1 = decltype(l1)::value;
                constexpr int TG = decltype(tg)::value;
                return launch("setup_kgen", (double)ncells(g), s, [&] {
                    k_kgen_store<T, L1, TG><<<grid, kBlock, 0, s>>>(img(l), g, w, out);
                });
            };
            using one = std::integral_constant<int, 1>;
            using all = std::integral_constant<int, kTaps>;
            if constexpr (std::is_same_v<T, float>) {
                // levels above 4096 cells whose counts are exact in bf16: matrix
                // cores, the pieces of the solve's FP32 mode or the bf16 leg's
                // single piece
                if (ncells(g) > 4096 && l <= kMfmaMaxLevel) {
                    const MfmaW* wm = mfma_block(net, blk);
                    const int mg = elem_grid(((size_t)g.nz * g.ny * ((g.nx + 15) / 16)) * 64);
                    auto mf = [&](auto km, auto l1) {
                        constexpr int KM = decltype(km)::value;
                        constexpr bool L1 = decltype(l1)::value;
                        return launch("setup_kgen", (double)ncells(g), s, [&] {
                            k_kgen_store_mfma<KM, L1><<<mg, kBlock, 0, s>>>(img(l), g, wm, out);
                        });
                    };
                    using x3 = std::integral_constant<int, kMfmaBf16x3>;
                    using b1 = std::integral_constant<int, kMfmaBf16>;
                    if (bf16w) NPS_TRY(l == 1 ? mf(b1{}, std::true_type{}) : mf(b1{}, std::false_type{}));
                    else NPS_TRY(l == 1 ? mf(x3{}, std::true_type{}) : mf(x3{}, std::false_type{}));
                    continue;
                }
            }
            if (l == 1) NPS_TRY(per_cell ? go(std::true_type{}, all{}) : go(std::true_type{}, one{}));
            else NPS_TRY(per_cell ? go(std::false_type{}, all{}) : go(std::false_type{}, one{}));
        }
    }
    return NPS_OK;
}

// Kernel dispatch over the per-level KMode (MFMA modes exist for float only).
template <class T, class F>
int with_kmode(int km, F&& f) {
    switch (km) {
        case kVector: return f(std::integral_constant<int, kVector>());
        case kStored: return f(std::integral_constant<int, kStored>());
        default: break;
    }
    if constexpr (std::is_same_v<T, float>) {
        switch (km) {
            case kMfmaBf16x3: return f(std::integral_constant<int, kMfmaBf16x3>());
            case kMfmaBf16: return f(std::integral_constant<int, kMfmaBf16>());
            case kMfmaF16: return f(std::integral_constant<int, kMfmaF16>());
            default: break;
        }
    }
    return fail(NPS_EINVAL, "kernel mode %d not available for this precision", km);
}

// Alg. 2 below level 1: coarse down levels, bottom workgroup, coarse up
// levels.  On return *x2 points at x^2, the input of level 1's up block.
// res_partials (with res_np and hf): the iteration's Residual stage, run by
// the bottom workgroup (the caller runs it itself when plan.lb > L).
template <class T>
int run_coarse(const nps_net* net, nps_dims d, const Plan& plan, const Layout& lay, void* ws, hipStream_t s,
               const T** x2, const double* res_partials = nullptr, int res_np = 0, HostFlags* hf = nullptr) {
    static const char* const kDownName[kMaxLevels + 1] = {"", "", "net_down_l2", "net_down_l3", "net_down_l4",
                                                          "net_down_l5", "net_down_l6"};
    static const char* const kUpName[kMaxLevels + 1] = {"", "", "net_up_l2", "net_up_l3", "net_up_l4", "net_up_l5",
                                                        "net_up_l6"};
    const int L = net->levels;
    State* st = mptr<State>(ws, lay.state);
    const int last_down = std::min(plan.lb - 1, L);   // levels handled by k_down
    for (int l = 2; l <= last_down; ++l) {
        const Grid g = level_grid(d, l);
        const uint32_t* cnt = cptr<uint32_t>(ws, lay.counts[l]);
        const T* rin = cptr<T>(ws, lay.rb[l]);
        T* x1 = mptr<T>(ws, lay.x1[l]);
        T* rnext = l < L ? mptr<T>(ws, lay.rb[l + 1]) : nullptr;
        const CConvW<T>* w = cconv_block<T>(net, block_down(l));
        const MfmaW* wm = mfma_block(net, block_down(l));
        const T* kst = plan.km[l] == kStored ? cptr<T>(ws, lay.k1[l]) : nullptr;
        const double cells = (double)ncells(g);
        NPS_TRY(with_kmode<T>(plan.km[l], [&](auto km) {
            constexpr int KM = decltype(km)::value;
            const int grid = persist_grid(l < L ? &k_down<T, KM, true> : &k_down<T, KM, false>, g);
            if (l < L)
                return launch(kDownName[l], cells, s, [&] {
                    k_down<T, KM, true><<<grid, kBlock, 0, s>>>(cnt, g, full_count(l), rin, x1, rnext, w, wm, kst, st,
                                                                 cptr<int8_t>(ws, lay.wmode[l][0]));
                });
            return launch("net_coarsest", cells, s, [&] {
                k_down<T, KM, false><<<grid, kBlock, 0, s>>>(cnt, g, full_count(l), rin, x1, nullptr, w, wm, kst, st,
                                                              cptr<int8_t>(ws, lay.wmode[l][0]));
            });
        }));
    }
    if (plan.lb <= L) {
        BottomArgs<T> a = {};
        a.lb = plan.lb;
        a.L = L;
        if (bottom_footprint(d, plan.lb, L) > (size_t)kBottomLds)
            return fail(NPS_EINVAL, "bottom levels exceed the workgroup buffer");
        size_t cells = 0;
        int off = 0;
        for (int l = plan.lb; l <= L; ++l) {
            const Grid g = level_grid(d, l);
            const int pc = padded_cells(g);
            BottomLevel& v = a.lv[l];
            v.g = g;
            v.n = (int)ncells(g);
            v.sy = g.nx + 2;
            v.sz = (g.ny + 2) * (g.nx + 2);
            v.r = off;
            v.x1 = off + pc;
            v.mx = div_magic(g.nx);
            v.mxy = div_magic(g.nx * g.ny);
            off += 2 * pc;
            a.k1[l] = cptr<T>(ws, lay.k1[l]);
            a.k2[l] = l < L ? cptr<T>(ws, lay.k2[l]) : nullptr;
            cells += ncells(g);
        }
        a.used = off;
        a.rin = cptr<T>(ws, lay.rb[plan.lb]);
        a.xout = mptr<T>(ws, lay.rb[plan.lb]);
        a.res_partials = res_partials;
        a.res_nparts = res_np;
        a.hf = hf;
        NPS_TRY(launch("net_bottom", (double)cells, s, [&] { k_bottom<T><<<1, kBottomThreads, 0, s>>>(a, st); }));
    }
    auto x_of = [&](int l) -> const T* {   // x^l, the up-sweep output of level l
        return (l == L && plan.lb > L) ? cptr<T>(ws, lay.x1[L]) : cptr<T>(ws, lay.rb[l]);
    };
    const int first_up = std::min(plan.lb - 1, L - 1);
    for (int l = first_up; l >= 2; --l) {
        const Grid g = level_grid(d, l);
        const uint32_t* cnt = cptr<uint32_t>(ws, lay.counts[l]);
        const T* xc = x_of(l + 1);
        const T* x1 = cptr<T>(ws, lay.x1[l]);
        T* xo = mptr<T>(ws, lay.rb[l]);
        const CConvW<T>* w = cconv_block<T>(net, block_up(net, l));
        const MfmaW* wm = mfma_block(net, block_up(net, l));
        const T* kst = plan.km[l] == kStored ? cptr<T>(ws, lay.k2[l]) : nullptr;
        NPS_TRY(with_kmode<T>(plan.km[l], [&](auto km) {
            constexpr int KM = decltype(km)::value;
            const int grid = persist_grid(&k_up<T, KM>, g);
            return launch(kUpName[l], (double)ncells(g), s, [&] {
                k_up<T, KM><<<grid, kBlock, 0, s>>>(cnt, g, full_count(l), xc, x1, xo, w, wm, kst, l - 1, st, nullptr,
                                                    cptr<int8_t>(ws, lay.wmode[l][0]));
            });
        }));
    }
    *x2 = x_of(2);
    return NPS_OK;
}

// Level-1 down kernel: x1 = CConv_1(r), r^2 = Pool(x1), r the network input.
template <class T>
int run_down_l1(const nps_net* net, const uint8_t* labels, nps_dims d, const Plan& plan, const Layout& lay, void* ws,
                const T* r, hipStream_t s, bool bf16w = false) {
    const Grid g = level_grid(d, 1);
    State* st = mptr<State>(ws, lay.state);
    T* x1 = mptr<T>(ws, lay.x1[1]);
    T* rnext = mptr<T>(ws, lay.rb[2]);
    const CConvW<T>* w = bf16w ? cconv_block_bf16<T>(net, block_down(1)) : cconv_block<T>(net, block_down(1));
    const MfmaW* wm = mfma_block(net, block_down(1));
    const T* kst = plan.km[1] == kStored ? cptr<T>(ws, lay.k1[1]) : nullptr;
    return with_kmode<T>(plan.km[1], [&](auto km) {
        constexpr int KM = decltype(km)::value;
        if constexpr (is_mfma(KM)) {
            // as many blocks as fit (the down kernel's registers allow five per CU)
            const int grid = persist_grid_n(&k_down_l1m<KM>, march_columns(g).count());
            return launch("net_down_l1", (double)ncells(g), s, [&] {
                k_down_l1m<KM><<<grid, kBlock, 0, s>>>(labels, g, r, x1, rnext, w, wm, st,
                                                       cptr<uint32_t>(ws, lay.gmode[0]), cptr<uint8_t>(ws, lay.izero[0]));
            });
        } else {
            const int grid = persist_grid(&k_down_l1<T, KM>, g);
            return launch("net_down_l1", (double)ncells(g), s, [&] {
                k_down_l1<T, KM><<<grid, kBlock, 0, s>>>(labels, g, r, x1, rnext, w, wm, kst, st,
                                                         cptr<int8_t>(ws, lay.wmode[1][0]));
            });
        }
    });
}

// Level-1 up kernel; its partial dots go to lay.dots, *nparts receives its
// grid (the number of partials).
template <class T, bool HOOK>
int run_up_l1(const nps_net* net, const uint8_t* labels, nps_dims d, const Plan& plan, const Layout& lay, void* ws,
              const T* x2, T* dhat, const T* const* ad, hipStream_t s, int* nparts, int max_dots = 0) {
    const Grid g = level_grid(d, 1);
    State* st = mptr<State>(ws, lay.state);
    double* partials = mptr<double>(ws, lay.dots);
    const T* x1 = cptr<T>(ws, lay.x1[1]);
    const CConvW<T>* w = cconv_block<T>(net, block_up(net, 1));
    const MfmaW* wm = mfma_block(net, block_up(net, 1));
    const T* kst = plan.km[1] == kStored ? cptr<T>(ws, lay.k2[1]) : nullptr;
    return with_kmode<T>(plan.km[1], [&](auto km) {
        constexpr int KM = decltype(km)::value;
        if constexpr (is_mfma(KM)) {
            // the kernel keeps registers for at most max_dots dot operands
            auto go = [&](auto nd) {
                constexpr int ND = decltype(nd)::value;
                constexpr bool H = HOOK;
                const int grid = persist_grid_n(&k_up_l1m<KM, H, H ? 0 : ND>, march_columns(g).count() / 2);
                if (nparts) *nparts = grid;
                return launch("net_up_l1", (double)ncells(g), s, [&] {
                    k_up_l1m<KM, H, H ? 0 : ND><<<grid, kBlock, 0, s>>>(labels, g, x2, x1, dhat, w, wm, st, partials,
                                                                       ad[0], ad[1], ad[2], ad[3],
                                                                       cptr<uint32_t>(ws, lay.gmode[1]),
                                                                       cptr<uint8_t>(ws, lay.izero[1]));
                });
            };
            if (HOOK || max_dots <= 0) return go(std::integral_constant<int, 0>());
            if (max_dots == 1) return go(std::integral_constant<int, 1>());
            if (max_dots == 2) return go(std::integral_constant<int, 2>());
            if (max_dots == 3) return go(std::integral_constant<int, 3>());
            return go(std::integral_constant<int, 4>());
        } else {
            const int grid = persist_grid(&k_up_l1<T, KM, HOOK>, g);
            if (nparts) *nparts = grid;
            return launch("net_up_l1", (double)ncells(g), s, [&] {
                k_up_l1<T, KM, HOOK><<<grid, kBlock, 0, s>>>(labels, g, x2, x1, dhat, w, wm, kst, st, partials, ad[0], ad[1],
                                                            ad[2], ad[3], nullptr, cptr<int8_t>(ws, lay.wmode[1][1]));
            });
        }
    });
}

// y = P^T g, the adjoint of the network in its input vector (P is linear in
// it): Alg. 2 backwards with each linear step replaced by its adjoint, on
// the stored kernels of every level (the setup of the layout tl must have
// run).  g and y are level-1 vectors; tl's gradient buffers are scratch.
template <class T>
int adjoint_apply(const nps_net* net, const uint8_t* labels, nps_dims d, const TrainLayout& tl, void* ws,
                  const T* g_in, T* y, hipStream_t s) {
    const int L = net->levels;
    const Layout& lay = tl.base;
    const State* st = cptr<State>(ws, lay.state);
    auto img = [&](int l) -> const void* {
        return l == 1 ? static_cast<const void*>(labels) : static_cast<const void*>(cptr<uint32_t>(ws, lay.counts[l]));
    };
    for (int l = 1; l < L; ++l) {   // up sweep, reversed
        const Grid g = level_grid(d, l);
        const int grid = tile_grid(g);
        const T* gin = l == 1 ? g_in : cptr<T>(ws, tl.gx[l]);
        const T* k2 = cptr<T>(ws, lay.k2[l]);
        T* gx1 = mptr<T>(ws, tl.gx1[l]);
        T* gr2 = mptr<T>(ws, tl.gr2[l]);
        if (l == 1)
            NPS_TRY(launch("adj_up", (double)ncells(g), s, [&] {
                k_bwd_up<T, true, false><<<grid, kBlock, 0, s>>>(img(l), g, gin, nullptr, nullptr, nullptr, k2, st, l - 1,
                                                                 gx1, gr2, nullptr);
            }));
        else
            NPS_TRY(launch("adj_up", (double)ncells(g), s, [&] {
                k_bwd_up<T, false, false><<<grid, kBlock, 0, s>>>(img(l), g, gin, nullptr, nullptr, nullptr, k2, st, l - 1,
                                                                  gx1, gr2, nullptr);
            }));
        const Grid gc = level_grid(d, l + 1);
        T* gxc = mptr<T>(ws, tl.gx[l + 1]);
        NPS_TRY(launch("adj_interp", (double)ncells(gc), s, [&] {
            k_bwd_interp<T><<<elem_grid(ncells(gc)), kBlock, 0, s>>>(gc, gr2, gxc);
        }));
    }
    for (int l = L; l >= 1; --l) {   // down sweep, reversed (the coarsest output gradient is gx^L)
        const Grid g = level_grid(d, l);
        const int grid = tile_grid(g);
        const T* gx1 = l == L ? cptr<T>(ws, tl.gx[L]) : cptr<T>(ws, tl.gx1[l]);
        const T* gr_next = l < L ? cptr<T>(ws, tl.gr1[l + 1]) : nullptr;
        const T* k1 = cptr<T>(ws, lay.k1[l]);
        T* gr1 = l > 1 ? mptr<T>(ws, tl.gr1[l]) : y;
        if (l == 1)
            NPS_TRY(launch("adj_down", (double)ncells(g), s, [&] {
                k_bwd_down<T, true, false><<<grid, kBlock, 0, s>>>(img(l), g, gx1, gr_next, nullptr, k1, gr1, nullptr);
            }));
        else
            NPS_TRY(launch("adj_down", (double)ncells(g), s, [&] {
                k_bwd_down<T, false, false><<<grid, kBlock, 0, s>>>(img(l), g, gx1, gr_next, nullptr, k1, gr1, nullptr);
            }));
    }
    return NPS_OK;
}

int check_opts(const nps_opts& o) {
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(NPS_EINVAL, "tol must be positive and finite");
    if (o.max_iter < 0) return fail(NPS_EINVAL, "max_iter must be >= 0");
    if (o.n_ortho < 0 || o.n_ortho > kMaxOrtho) return fail(NPS_EINVAL, "n_ortho must be in [0, %d]", kMaxOrtho);
    if (o.precision < NPS_FP64 || o.precision > NPS_MIXED_FP16) return fail(NPS_EINVAL, "unknown precision %d", o.precision);
    if (o.method < NPS_NPSDO || o.method > NPS_FPCG) return fail(NPS_EINVAL, "unknown method %d", o.method);
    if (o.method != NPS_NPSDO && o.n_ortho != 1) return fail(NPS_EINVAL, "PCG and flexible PCG need n_ortho = 1");
    if (o.symmetric != 0 && o.symmetric != 1) return fail(NPS_EINVAL, "symmetric must be 0 or 1");
    return NPS_OK;
}

// Plan and workspace layout of a solve: the symmetric variant keeps the
// kernels of every level in HBM (its P^T sweep gathers them) and carries the
// adjoint's buffers.
struct SolveLayout {
    Plan plan;
    Layout lay;
    TrainLayout tl;
    size_t total;
};

SolveLayout solve_layout(nps_dims d, int levels, const nps_opts& o) {
    SolveLayout r{};
    if (o.symmetric) {
        r.plan = make_plan(d, levels, o.precision, true);
        r.tl = make_train_layout(d, levels, o.precision, true, o.n_ortho);
        r.lay = r.tl.base;
        r.total = r.tl.total;
    } else {
        r.plan = make_plan(d, levels, o.precision);
        r.lay = make_layout(d, levels, o.precision, o.n_ortho, true);
        r.total = r.lay.total;
    }
    return r;
}

// One solve in flight, as enqueue steps on one stream: nps_solve drives a
// single solver to completion; the request server keeps one per slot.
struct Solver {
    const nps_net* net = nullptr;
    const uint8_t* labels = nullptr;
    const double* b = nullptr;
    nps_dims d{};
    nps_opts o{};
    Plan plan{};
    Layout lay{};
    TrainLayout tl{};             // symmetric variant only
    void* ws = nullptr;
    hipStream_t s = nullptr;
    State* hs = nullptr;          // pinned host mirror of the device state
    HostFlags* hf = nullptr;      // pinned flags written by the control kernel
    HostFlags* hf_d = nullptr;    // device address of hf
    virtual ~Solver() {}
    virtual int enqueue_validate() = 0;            // scan, then copy the state to hs
    virtual int enqueue_setup() = 0;               // pyramid, Aff, stored kernels
    virtual int enqueue_body(int k) = 0;           // iteration k (see below)
    virtual int enqueue_finalize(double* x_out) = 0;   // x_out, then copy the state to hs
};

// Validation verdict from the state mirror after enqueue_validate completed.
int validation_status(const State* hs) {
    if (hs->bad_label) return fail(NPS_ELABEL, "%d labels outside {0,1,2}", hs->bad_label);
    if (hs->n_fluid == 0) return fail(NPS_ENOFLUID, "no fluid cell");
    if (hs->nonfinite) return fail(NPS_ENONFINITE, "%d non-finite entries of b on fluid cells", hs->nonfinite);
    return NPS_OK;
}

// nps_info from the state mirror after enqueue_finalize completed.
int fill_info(const State* hs, nps_info* info) {
    info->n_fluid = hs->n_fluid;
    if (hs->bb == 0.0) {
        info->iterations = 0;
        info->status = NPS_OK;
        info->rel_residual = info->rel_residual_rec = 0.0;
        info->refinements = 0;
        return NPS_OK;
    }
    info->iterations = hs->iter;
    info->status = hs->done ? hs->status : NPS_NOT_CONVERGED;
    info->rel_residual = std::sqrt(hs->rr / hs->bb);
    info->rel_residual_rec = info->rel_residual;
    info->refinements = hs->iter + 1;
    if (info->status == NPS_EBREAKDOWN)
        fail(NPS_EBREAKDOWN, "breakdown: d.Ad <= 0 or not finite at iteration %d", hs->iter + 1);
    return info->status;
}

template <class T, class X>
struct SolverT : Solver {
    int enqueue_validate() override {
        const size_t n = ncells(level_grid(d, 1));
        State* st = mptr<State>(ws, lay.state);
        double* partials = mptr<double>(ws, lay.partials);
        X* x = mptr<X>(ws, lay.x[0]);
        const int max_iter = std::max(o.max_iter, 0);
        NPS_TRY(launch("state_init", 0, s, [&] {
            k_state_init<<<1, 64, 0, s>>>(st, max_iter, o.fixed_iters ? 1 : 0, o.n_ortho, o.method, o.symmetric);
        }));
        const int sgrid = red_elem_grid(n);
        NPS_TRY(launch("setup_scan", (double)n, s, [&] { k_scan<X><<<sgrid, kBlock, 0, s>>>(labels, b, n, x, partials); }));
        NPS_TRY(launch("control", 0, s, [&] {
            k_control<kStageScan><<<1, kCtlBlock, 0, s>>>(st, partials, sgrid, 0, 0, 0, 0, o.tol, 0.0, 0.0, nullptr);
        }));
        // the 7-point kernels' live items; the others get zeros in the vectors
        // those kernels write (and read back) there
        const Grid g = level_grid(d, 1);
        const int nitems = columns_of(g).count();
        ZeroBufs zb{};
        auto zero = [&](void* p, int bytes) {
            zb.p[zb.n] = p;
            zb.bytes[zb.n++] = bytes;
        };
        zero(mptr<X>(ws, lay.x[1]), (int)sizeof(X));
        zero(mptr<T>(ws, lay.r[0]), (int)sizeof(T));
        zero(mptr<T>(ws, lay.r[1]), (int)sizeof(T));
        for (int i = 0; i <= o.n_ortho; ++i) {
            zero(mptr<T>(ws, lay.dring[i]), (int)sizeof(T));
            zero(mptr<T>(ws, lay.adring[i]), (int)sizeof(T));
        }
        uint8_t* live = mptr<uint8_t>(ws, lay.live);
        NPS_TRY(launch("setup_items", (double)n, s, [&] { k_item_live<<<nitems, kBlock, 0, s>>>(labels, g, live, zb); }));
        NPS_TRY(launch("setup_item_list", 0, s, [&] {
            k_item_list<<<1, kBlock, 0, s>>>(live, nitems, mptr<uint32_t>(ws, lay.items), st);
        }));
        NPS_HIP(hipMemcpyAsync(hs, st, sizeof(State), hipMemcpyDeviceToHost, s));
        return NPS_OK;
    }

    int enqueue_setup() override {
        hf->done = 0;
        hf->iter = 0;
        nlive = hs->nlive;   // the validation copy has completed
        return run_setup<T>(net, labels, d, plan, lay, ws, s);
    }

    int nlive = 0;   // live items of the 7-point kernels (set-up)

    // The ortho kernel's grid (the count of its partials, which the next
    // body's residual kernel sums).
    int ortho_grid() const {
        switch (o.n_ortho) {
            case 0: return persist_grid_n(&k_ortho<T, 0>, nlive);
            case 1: return persist_grid_n(&k_ortho<T, 1>, nlive);
            case 2: return persist_grid_n(&k_ortho<T, 2>, nlive);
            case 3: return persist_grid_n(&k_ortho<T, 3>, nlive);
            default: return persist_grid_n(&k_ortho<T, 4>, nlive);
        }
    }

    // Body k finishes step k-1 (its length from the previous body's dots),
    // forms x_(k-1) and r_(k-1) = b - A x_(k-1), tests convergence, then forms
    // the direction d_k and the dots of its step.
    int enqueue_body(int k) override {
        const Grid g = level_grid(d, 1);
        const double cells = (double)ncells(g);
        State* st = mptr<State>(ws, lay.state);
        double* partials = mptr<double>(ws, lay.partials);
        double* pdots = mptr<double>(ws, lay.dots);
        X* x0 = mptr<X>(ws, lay.x[0]);
        X* x1b = mptr<X>(ws, lay.x[1]);
        T* r = mptr<T>(ws, lay.r[k & 1]);
        const T* r_prev = cptr<T>(ws, lay.r[(k + 1) & 1]);
        T* dhat = mptr<T>(ws, lay.dhat);
        const int R = o.n_ortho + 1;

        const int slot = k % R;
        const T* ad[kMaxOrtho] = {nullptr, nullptr, nullptr, nullptr};
        const T* dp[kMaxOrtho] = {nullptr, nullptr, nullptr, nullptr};
        int sl[kMaxOrtho] = {0, 0, 0, 0};
        for (int j = 0; j < o.n_ortho; ++j) {
            sl[j] = ((k - 1 - j) % R + R) % R;
            dp[j] = cptr<T>(ws, lay.dring[sl[j]]);
            ad[j] = cptr<T>(ws, lay.adring[sl[j]]);
        }
        if (o.method != NPS_NPSDO) {   // PCG forms: the up kernel dots P(r) with r (and r_(k-1))
            ad[0] = r;
            ad[1] = r_prev;
        }
        const T* dpend = cptr<T>(ws, lay.dring[((k - 1) % R + R) % R]);
        T* dk = mptr<T>(ws, lay.dring[slot]);
        T* adk = mptr<T>(ws, lay.adring[slot]);
        const T* x2 = nullptr;
        int np = 0;
        // x += alpha d and r = b - A x (one-cell halo), then the network on r
        // (from body 2 on it first runs the Step stage of the previous body, on
        // the ortho kernel's partials; its own ||r||^2 partials go to the dots
        // buffer, which the Residual stage consumes before the up kernel refills it)
        const uint32_t* items = cptr<uint32_t>(ws, lay.items);
        const int np_res = persist_grid_n(&k_residual<T, X>, nlive);
        const int snp = k > 1 ? ortho_grid() : 0;
        NPS_TRY(launch("residual", cells, s, [&] {
            // body k reads the iterate from buffer (k - 1) & 1 (state.xcur, which
            // every Residual stage flips) and writes the other
            const bool odd = ((k - 1) & 1) != 0;
            k_residual<T, X><<<np_res, kBlock, 0, s>>>(labels, g, b, odd ? x1b : x0, odd ? x0 : x1b, dpend, r, st,
                                                       partials, snp, ((k - 1) % R + R) % R, hf_d, pdots, items,
                                                       nlive);
        }));
        // The Residual stage (convergence test, 1/||r||, the dots the up
        // kernel forms) is first needed by the up sweep, and the network is
        // linear in r: the bottom workgroup runs it when there is one.
        const bool res_in_bottom = plan.lb <= net->levels;
        if (!res_in_bottom)
            NPS_TRY(launch("control", 0, s, [&] {
                k_control<kStageResidual><<<1, kCtlBlock, 0, s>>>(st, pdots, np_res, 0, 0, 0, 0, 0.0, 0.0, 0.0, hf_d);
            }));
        NPS_TRY(run_down_l1<T>(net, labels, d, plan, lay, ws, r, s));
        if (res_in_bottom) NPS_TRY(run_coarse<T>(net, d, plan, lay, ws, s, &x2, pdots, np_res, hf_d));
        else NPS_TRY(run_coarse<T>(net, d, plan, lay, ws, s, &x2));
        NPS_TRY((run_up_l1<T, false>(net, labels, d, plan, lay, ws, x2, dhat, ad, s, &np,
                                     o.symmetric ? 0 : (o.method == NPS_NPSDO ? o.n_ortho : o.method == NPS_PCG ? 1 : 2))));
        if (o.symmetric) {   // d^ = P^T P(r)/||r||, then the dots the up kernel left out
            T* dsym = mptr<T>(ws, tl.dsym);
            NPS_TRY(adjoint_apply<T>(net, labels, d, tl, ws, dhat, dsym, s));
            const size_t n = ncells(g);
            np = red_elem_grid(n);
            NPS_TRY(launch("sym_dots", cells, s, [&] {
                k_dots<T><<<np, kBlock, 0, s>>>(n, dsym, ad[0], ad[1], ad[2], ad[3], st, pdots);
            }));
            dhat = dsym;
        }
        // the Dots stage runs inside the ortho kernel (every block sums the dots)
        const int dnp = o.n_ortho > 0 ? np : 0;
        const int ogrid = ortho_grid();
        NPS_TRY(launch("ortho_matvec", cells, s, [&] {
            auto go = [&](auto no) {
                k_ortho<T, decltype(no)::value><<<ogrid, kBlock, 0, s>>>(labels, g, dhat, dp[0], dp[1], dp[2], dp[3], r,
                                                                         dk, adk, st, pdots, dnp, sl[0], sl[1], sl[2],
                                                                         sl[3], partials, items, nlive);
            };
            switch (o.n_ortho) {
                case 0: go(std::integral_constant<int, 0>{}); break;
                case 1: go(std::integral_constant<int, 1>{}); break;
                case 2: go(std::integral_constant<int, 2>{}); break;
                case 3: go(std::integral_constant<int, 3>{}); break;
                default: go(std::integral_constant<int, 4>{}); break;
            }
        }));
        // the Step stage (alpha) runs at the start of the next body's residual kernel
        return NPS_OK;
    }

    int enqueue_finalize(double* x_out) override {
        const size_t n = ncells(level_grid(d, 1));
        State* st = mptr<State>(ws, lay.state);
        const X* x0 = cptr<X>(ws, lay.x[0]);
        const X* x1b = cptr<X>(ws, lay.x[1]);
        NPS_TRY(launch("finalize", (double)n, s, [&] {
            k_finalize<X><<<elem_grid(n), kBlock, 0, s>>>(n, labels, x0, x1b, st, x_out);
        }));
        NPS_HIP(hipMemcpyAsync(hs, st, sizeof(State), hipMemcpyDeviceToHost, s));
        return NPS_OK;
    }
};

Solver* make_solver(int precision) {
    switch (precision) {
        case NPS_FP64: return new SolverT<double, double>();
        case NPS_FP32: return new SolverT<float, float>();
        default: return new SolverT<float, double>();
    }
}

// nps_solve: validate, set up, iterate with a one-body-behind poll, finalize.
// Events bracketing a solve's phases on its stream (created once per thread).
struct SolveEvents {
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};   // start, setup done, end
    bool ok = false;
    SolveEvents() {
        ok = true;
        for (auto& e : ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    }
};

int run_solve(Solver& sv, double* x_out, nps_info* info) {
    thread_local SolveEvents tev;
    if (!tev.ok) return fail(NPS_EDEVICE, "hipEventCreate failed");
    NPS_HIP(hipEventRecord(tev.ev[0], sv.s));
    NPS_TRY(sv.enqueue_validate());
    NPS_HIP(hipStreamSynchronize(sv.s));
    NPS_TRY(validation_status(sv.hs));
    if (sv.hs->bb != 0.0) {
        NPS_TRY(sv.enqueue_setup());
        NPS_HIP(hipEventRecord(tev.ev[1], sv.s));
        const int max_iter = std::max(sv.o.max_iter, 0);
        volatile HostFlags* hf = sv.hf;
        for (int k = 1; k <= max_iter + 1; ++k) {
            NPS_TRY(sv.enqueue_body(k));
            if (k < 2) continue;
            // Keep about two bodies queued: wait until body k-1 has passed its
            // residual test (the control kernel mirrors the completed
            // iteration count, k-2 by then, and the stop flag to pinned host
            // memory), with no marker in the stream.  An idle stream ends the
            // wait too (the flags have then been written for good).
            for (long spin = 0; !hf->done && hf->iter < k - 2; ++spin) {
                if ((spin & 255) == 255) {
                    const hipError_t q = hipStreamQuery(sv.s);
                    if (q == hipSuccess) break;
                    if (q != hipErrorNotReady) return fail(NPS_EDEVICE, "stream failed: %s", hipGetErrorString(q));
                }
            }
            if (hf->done) break;
        }
    } else {
        NPS_HIP(hipEventRecord(tev.ev[1], sv.s));
    }
    NPS_TRY(sv.enqueue_finalize(x_out));
    NPS_HIP(hipEventRecord(tev.ev[2], sv.s));
    NPS_HIP(hipStreamSynchronize(sv.s));
    const int rc = fill_info(sv.hs, info);
    float setup_ms = 0.0f, iter_ms = 0.0f;
    NPS_HIP(hipEventElapsedTime(&setup_ms, tev.ev[0], tev.ev[1]));
    NPS_HIP(hipEventElapsedTime(&iter_ms, tev.ev[1], tev.ev[2]));
    info->t_setup_ms = setup_ms;
    info->t_iter_ms = info->iterations > 0 ? iter_ms / info->iterations : 0.0;
    return rc;
}

template <class T>
int precond_impl(const nps_net* net, const uint8_t* labels, nps_dims d, const T* r_in, T* d_out, void* ws,
                 const Plan& plan, const Layout& lay, hipStream_t s) {
    State* st = mptr<State>(ws, lay.state);
    NPS_TRY(launch("state_init", 0, s, [&] { k_state_init<<<1, 64, 0, s>>>(st, 0, 0, 0, 0, 0); }));
    NPS_TRY(run_setup<T>(net, labels, d, plan, lay, ws, s));
    NPS_TRY(run_down_l1<T>(net, labels, d, plan, lay, ws, r_in, s));
    const T* x2 = nullptr;
    NPS_TRY(run_coarse<T>(net, d, plan, lay, ws, s, &x2));
    const T* none[kMaxOrtho] = {nullptr, nullptr, nullptr, nullptr};
    return run_up_l1<T, true>(net, labels, d, plan, lay, ws, x2, d_out, none, s, nullptr);
}


// ---------------------------------------------------------------------------
// request server
// ---------------------------------------------------------------------------
// Pinned host buffers reused by exact size (request grids repeat).  Only
// admitted and finished-but-unpolled requests hold one, so the pinned
// footprint stays near max_slots requests however long the queue grows.
struct PinnedPool {
    std::multimap<size_t, void*> free_;
    void* get(size_t bytes) {
        auto it = free_.find(bytes);
        if (it != free_.end()) {
            void* p = it->second;
            free_.erase(it);
            return p;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        return p;
    }
    void put(size_t bytes, void* p) {
        if (p) free_.emplace(bytes, p);
    }
    ~PinnedPool() {
        for (auto& kv : free_) (void)hipHostFree(kv.second);
    }
};

// First-fit allocator over the device arena (offsets, 256-byte granules).
struct Arena {
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t size) { free_ = {{0, size}}; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

using Clock = std::chrono::steady_clock;

struct Request {
    enum Phase { kQueued, kValidating, kRunning, kFinishing, kDone };
    uint64_t id = 0;
    nps_dims d{};
    nps_opts o{};
    size_t n = 0;
    const uint8_t* lab_u = nullptr;   // the caller's inputs, read once at admission
    const double* b_u = nullptr;
    uint8_t* lab_h = nullptr;   // pinned staging of the inputs (admission to validation)
    double* b_h = nullptr;
    double* x_h = nullptr;      // pinned result (from the finalize step until polled)
    bool x_ready = false;       // x_h was written (the request reached its finalize step)
    Phase phase = kQueued;
    int status = NPS_OK;
    nps_info info{};
    Clock::time_point t_submit, t_done;
    int slot = -1;
    size_t off = 0, bytes = 0;  // arena region
    int k = 0;                  // last body enqueued
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    State* hs = nullptr;
    HostFlags* hf = nullptr;
    HostFlags* hf_d = nullptr;
    Solver* sv = nullptr;
    Request* req = nullptr;
};

struct RequestLayout {
    size_t ws, lab, b, x, total;
};

RequestLayout request_layout(nps_dims d, int levels, const nps_opts& o) {
    RequestLayout r{};
    const size_t n = ncells(level_grid(d, 1));
    r.ws = 0;
    r.lab = align256(solve_layout(d, levels, o).total);
    r.b = r.lab + align256(n);
    r.x = r.b + align256(8 * n);
    r.total = r.x + align256(8 * n);
    return r;
}

}  // namespace

struct nps_server {
    const nps_net* net = nullptr;
    char* arena_d = nullptr;
    size_t budget = 0;
    Arena arena;
    std::vector<Slot> slots;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, Request*> live;   // every request not yet polled
    uint64_t next_id = 1;
    PinnedPool pool;
    void* mirror = nullptr;   // pinned mapped block of the slots' state mirrors and flags
};

namespace {

void release_inputs(nps_server* srv, Request* r) {
    srv->pool.put(r->n, r->lab_h);
    srv->pool.put(8 * r->n, r->b_h);
    r->lab_h = nullptr;
    r->b_h = nullptr;
}

// The request leaves its slot and arena region; its result waits for a poll.
void retire(nps_server* srv, Slot& sl, int status) {
    Request* r = sl.req;
    r->status = status;
    r->t_done = Clock::now();
    r->phase = Request::kDone;
    release_inputs(srv, r);
    srv->arena.release(r->off, r->bytes);
    delete sl.sv;
    sl.sv = nullptr;
    sl.req = nullptr;
}

int admit(nps_server* srv, Slot& sl, Request* r) {
    r->lab_h = static_cast<uint8_t*>(srv->pool.get(r->n));
    r->b_h = static_cast<double*>(srv->pool.get(8 * r->n));
    if (!r->lab_h || !r->b_h) {   // nothing enqueued yet: the request ends here
        release_inputs(srv, r);
        srv->arena.release(r->off, r->bytes);
        r->status = fail(NPS_EDEVICE, "pinned host allocation failed");
        r->t_done = Clock::now();
        r->phase = Request::kDone;
        return NPS_OK;
    }
    std::memcpy(r->lab_h, r->lab_u, r->n);
    std::memcpy(r->b_h, r->b_u, 8 * r->n);
    r->lab_u = nullptr;
    r->b_u = nullptr;
    const RequestLayout rl = request_layout(r->d, srv->net->levels, r->o);
    char* base = srv->arena_d + r->off;
    Solver* sv = make_solver(r->o.precision);
    sv->net = srv->net;
    sv->labels = reinterpret_cast<const uint8_t*>(base + rl.lab);
    sv->b = reinterpret_cast<const double*>(base + rl.b);
    sv->d = r->d;
    sv->o = r->o;
    const SolveLayout sol = solve_layout(r->d, srv->net->levels, r->o);
    sv->plan = sol.plan;
    sv->lay = sol.lay;
    sv->tl = sol.tl;
    sv->ws = base + rl.ws;
    sv->s = sl.s;
    sv->hs = sl.hs;
    sv->hf = sl.hf;
    sv->hf_d = sl.hf_d;
    sl.sv = sv;
    sl.req = r;
    r->slot = (int)(&sl - srv->slots.data());
    NPS_HIP(hipMemcpyAsync(base + rl.lab, r->lab_h, r->n, hipMemcpyHostToDevice, sl.s));
    NPS_HIP(hipMemcpyAsync(base + rl.b, r->b_h, 8 * r->n, hipMemcpyHostToDevice, sl.s));
    NPS_TRY(sv->enqueue_validate());
    NPS_HIP(hipEventRecord(sl.ev[0], sl.s));
    r->phase = Request::kValidating;
    return NPS_OK;
}

int enqueue_finish(nps_server* srv, Slot& sl) {
    Request* r = sl.req;
    const RequestLayout rl = request_layout(r->d, srv->net->levels, r->o);
    double* x_d = reinterpret_cast<double*>(srv->arena_d + r->off + rl.x);
    r->x_h = static_cast<double*>(srv->pool.get(8 * r->n));
    if (!r->x_h) {   // let the slot's stream drain before its arena region is reused
        NPS_HIP(hipStreamSynchronize(sl.s));
        retire(srv, sl, fail(NPS_EDEVICE, "pinned host allocation failed"));
        return NPS_OK;
    }
    NPS_TRY(sl.sv->enqueue_finalize(x_d));
    NPS_HIP(hipMemcpyAsync(r->x_h, x_d, 8 * r->n, hipMemcpyDeviceToHost, sl.s));
    NPS_HIP(hipEventRecord(sl.ev[0], sl.s));
    r->x_ready = true;
    r->phase = Request::kFinishing;
    return NPS_OK;
}

bool event_done(hipEvent_t e) { return hipEventQuery(e) == hipSuccess; }

// Advance one slot without blocking; returns a hard error only for device failures.
int advance(nps_server* srv, Slot& sl) {
    Request* r = sl.req;
    switch (r->phase) {
        case Request::kValidating: {
            if (!event_done(sl.ev[0])) return NPS_OK;
            release_inputs(srv, r);
            const int v = validation_status(sl.hs);
            if (v != NPS_OK) {
                retire(srv, sl, v);
                return NPS_OK;
            }
            if (sl.hs->bb == 0.0) return enqueue_finish(srv, sl);
            NPS_TRY(sl.sv->enqueue_setup());
            const int last = std::max(r->o.max_iter, 0) + 1;
            for (int k = 1; k <= std::min(2, last); ++k) {
                NPS_TRY(sl.sv->enqueue_body(k));
                NPS_HIP(hipEventRecord(sl.ev[k & 1], sl.s));
                r->k = k;
            }
            r->phase = Request::kRunning;
            return NPS_OK;
        }
        case Request::kRunning: {
            const int last = std::max(r->o.max_iter, 0) + 1;
            const int watch = r->k < last ? r->k - 1 : r->k;   // one behind, or the final body
            if (watch >= 1 && !event_done(sl.ev[watch & 1])) return NPS_OK;
            if (watch < 1 && !event_done(sl.ev[r->k & 1])) return NPS_OK;
            volatile HostFlags* hf = sl.hf;
            if (hf->done || r->k >= last) return enqueue_finish(srv, sl);
            r->k += 1;
            NPS_TRY(sl.sv->enqueue_body(r->k));
            NPS_HIP(hipEventRecord(sl.ev[r->k & 1], sl.s));
            return NPS_OK;
        }
        case Request::kFinishing: {
            if (!event_done(sl.ev[0])) return NPS_OK;
            nps_info info{};
            const int st = fill_info(sl.hs, &info);
            r->info = info;
            retire(srv, sl, st);
            return NPS_OK;
        }
        default:
            return NPS_OK;
    }
}


// ---------------------------------------------------------------------------
// training: forward with saved activations, backward, loss
// ---------------------------------------------------------------------------
size_t off_c1(int l) { return (size_t)(l - 1) * (27 * 81 + 27); }
size_t off_c2(int L, int l) { return (size_t)(L + l - 1) * (27 * 81 + 27); }
size_t off_aff(int L, int l) { return (size_t)(2 * L - 1) * (27 * 81 + 27) + (size_t)(l - 1) * 164; }

template <class T>
int train_forward(const nps_net* net, const uint8_t* labels, nps_dims d, const TrainLayout& tl, void* ws,
                  const T* r, T* y, hipStream_t s, bool bf16w = false) {
    const int L = net->levels;
    const Layout& lay = tl.base;
    const Plan plan = make_plan(d, L, vec_bytes(NPS_FP32) == sizeof(T) ? NPS_FP32 : NPS_FP64, true);
    State* st = mptr<State>(ws, lay.state);
    auto wblock = [&](int b) { return bf16w ? cconv_block_bf16<T>(net, b) : cconv_block<T>(net, b); };
    NPS_TRY(launch("state_init", 0, s, [&] { k_state_init<<<1, 64, 0, s>>>(st, 0, 0, 0, 0, 0); }));
    NPS_TRY(run_setup<T>(net, labels, d, plan, lay, ws, s, bf16w));
    auto img = [&](int l) -> const void* {
        return l == 1 ? static_cast<const void*>(labels) : static_cast<const void*>(cptr<uint32_t>(ws, lay.counts[l]));
    };
    for (int l = 1; l < L; ++l) {   // image-window sums for the Aff gradients
        const Grid g = level_grid(d, l);
        double* sp = mptr<double>(ws, tl.spart) + (size_t)(l - 1) * 3 * kTaps * kSumBlocks;
        const double inv_full = std::ldexp(1.0, -3 * (l - 1));
        if (l == 1)
            NPS_TRY(launch("train_image_sums", (double)ncells(g), s, [&] { k_image_sums<true><<<sum_blocks(g), kBlock, 0, s>>>(img(l), g, inv_full, sp); }));
        else
            NPS_TRY(launch("train_image_sums", (double)ncells(g), s, [&] { k_image_sums<false><<<sum_blocks(g), kBlock, 0, s>>>(img(l), g, inv_full, sp); }));
    }
    NPS_TRY(run_down_l1<T>(net, labels, d, plan, lay, ws, r, s, bf16w));
    for (int l = 2; l <= L; ++l) {
        const Grid g = level_grid(d, l);
        const int grid = tile_grid(g);
        const uint32_t* cnt = cptr<uint32_t>(ws, lay.counts[l]);
        const T* rin = cptr<T>(ws, lay.rb[l]);
        T* x1 = mptr<T>(ws, lay.x1[l]);
        T* rnext = l < L ? mptr<T>(ws, lay.rb[l + 1]) : nullptr;
        const T* kst = cptr<T>(ws, lay.k1[l]);
        const CConvW<T>* w = wblock(block_down(l));
        if (l < L)
            NPS_TRY(launch("net_down", (double)ncells(g), s, [&] {
                k_down<T, kStored, true><<<grid, kBlock, 0, s>>>(cnt, g, full_count(l), rin, x1, rnext, w, nullptr, kst, st,
                                                                  nullptr);
            }));
        else
            NPS_TRY(launch("net_coarsest", (double)ncells(g), s, [&] {
                k_down<T, kStored, false><<<grid, kBlock, 0, s>>>(cnt, g, full_count(l), rin, x1, nullptr, w, nullptr, kst,
                                                                   st, nullptr);
            }));
    }
    auto x_of = [&](int l) -> const T* { return l == L ? cptr<T>(ws, lay.x1[L]) : cptr<T>(ws, tl.xup[l]); };
    for (int l = L - 1; l >= 2; --l) {
        const Grid g = level_grid(d, l);
        const int grid = tile_grid(g);
        const uint32_t* cnt = cptr<uint32_t>(ws, lay.counts[l]);
        const T* xc = x_of(l + 1);
        const T* x1 = cptr<T>(ws, lay.x1[l]);
        T* xo = mptr<T>(ws, tl.xup[l]);
        T* x2o = mptr<T>(ws, tl.x2[l]);
        const T* kst = cptr<T>(ws, lay.k2[l]);
        const CConvW<T>* w = wblock(block_up(net, l));
        NPS_TRY(launch("net_up", (double)ncells(g), s, [&] {
            k_up<T, kStored><<<grid, kBlock, 0, s>>>(cnt, g, full_count(l), xc, x1, xo, w, nullptr, kst, l - 1, st, x2o,
                                                         nullptr);
        }));
    }
    {
        const Grid g = level_grid(d, 1);
        const int grid = tile_grid(g);
        const T* xc = x_of(2);
        const T* x1 = cptr<T>(ws, lay.x1[1]);
        T* x2o = mptr<T>(ws, tl.x2[1]);
        const T* kst = cptr<T>(ws, lay.k2[1]);
        const CConvW<T>* w = wblock(block_up(net, 1));
        double* partials = mptr<double>(ws, lay.partials);
        NPS_TRY(launch("net_up_l1", (double)ncells(g), s, [&] {
            k_up_l1<T, kStored, true><<<grid, kBlock, 0, s>>>(labels, g, xc, x1, y, w, nullptr, kst, st, partials, nullptr,
                                                            nullptr, nullptr, nullptr, x2o, nullptr);
        }));
    }
    return NPS_OK;
}

// The weight-gradient sums of one CConv block from nparts per-block rows:
// chunk sums in place, then the final reduction into gW (and dc).
int wgrad_reduce(double* wpart, int nparts, double scale, double* gW, double* dc, hipStream_t s) {
    const dim3 cgrid((nparts + kWChunk - 1) / kWChunk, (kWPart + kBlock - 1) / kBlock);
    NPS_TRY(launch("train_wgrad_chunks", 0, s, [&] { k_wgrad_chunks<<<cgrid, kBlock, 0, s>>>(wpart, nparts); }));
    return launch("train_wgrad_reduce", 0, s, [&] {
        k_wgrad_reduce<<<1, kBlock, 0, s>>>(wpart, nparts, scale, gW, gW + 27 * 81, dc);
    });
}

template <class T, int WP = std::is_same<T, float>::value ? kWgMfma32 : kWgVector>
int train_backward(const nps_net* net, const uint8_t* labels, nps_dims d, const TrainLayout& tl, void* ws,
                   const T* r, const T* gy, double* grad, hipStream_t s) {
    const int L = net->levels;
    const Layout& lay = tl.base;
    State* st = mptr<State>(ws, lay.state);
    double* wpart = mptr<double>(ws, tl.wpart);
    double* dc = mptr<double>(ws, tl.dc);
    auto img = [&](int l) -> const void* {
        return l == 1 ? static_cast<const void*>(labels) : static_cast<const void*>(cptr<uint32_t>(ws, lay.counts[l]));
    };
    auto x_of = [&](int l) -> const T* { return l == L ? cptr<T>(ws, lay.x1[L]) : cptr<T>(ws, tl.xup[l]); };
    // up sweep, reversed
    for (int l = 1; l < L; ++l) {
        const Grid g = level_grid(d, l);
        const int grid = std::min(tile_grid(g), kTrainBlocks);
        const T* gin = l == 1 ? gy : cptr<T>(ws, tl.gx[l]);
        const T* xc = x_of(l + 1);
        const T* x1 = cptr<T>(ws, lay.x1[l]);
        const T* x2 = cptr<T>(ws, tl.x2[l]);
        const T* k2 = cptr<T>(ws, lay.k2[l]);
        T* gx1 = mptr<T>(ws, tl.gx1[l]);
        T* gr2 = mptr<T>(ws, tl.gr2[l]);
        if (l == 1)
            NPS_TRY(launch("train_bwd_up", (double)ncells(g), s, [&] {
                k_bwd_up<T, true, true, WP><<<grid, kBlock, 0, s>>>(img(l), g, gin, xc, x1, x2, k2, st, l - 1, gx1, gr2, wpart);
            }));
        else
            NPS_TRY(launch("train_bwd_up", (double)ncells(g), s, [&] {
                k_bwd_up<T, false, true, WP><<<grid, kBlock, 0, s>>>(img(l), g, gin, xc, x1, x2, k2, st, l - 1, gx1, gr2, wpart);
            }));
        const double scale = std::ldexp(1.0, -3 * (l - 1));
        double* gW = grad + off_c2(L, l);
        double* dcl = dc + 2 * (l - 1);
        NPS_TRY(wgrad_reduce(wpart, grid, scale, gW, dcl, s));
        const double* sp = cptr<double>(ws, tl.spart) + (size_t)(l - 1) * 3 * kTaps * kSumBlocks;
        double* ga = grad + off_aff(L, l);
        const double n27 = 27.0 * (double)ncells(g);
        NPS_TRY(launch("train_aff_grad", 0, s, [&] { k_aff_grad<<<3 * kTaps, kBlock, 0, s>>>(sp, sum_blocks(g), dcl, n27, ga, ga + 82); }));
        const Grid gc = level_grid(d, l + 1);
        T* gxc = mptr<T>(ws, tl.gx[l + 1]);
        NPS_TRY(launch("train_bwd_interp", (double)ncells(gc), s, [&] {
            k_bwd_interp<T><<<elem_grid(ncells(gc)), kBlock, 0, s>>>(gc, gr2, gxc);
        }));
    }
    // down sweep, reversed (the coarsest level's output gradient is gx^L)
    for (int l = L; l >= 1; --l) {
        const Grid g = level_grid(d, l);
        const int grid = std::min(tile_grid(g), kTrainBlocks);
        const T* gx1 = l == L ? cptr<T>(ws, tl.gx[L]) : cptr<T>(ws, tl.gx1[l]);
        const T* gr_next = l < L ? cptr<T>(ws, tl.gr1[l + 1]) : nullptr;
        const T* r1 = l == 1 ? r : cptr<T>(ws, lay.rb[l]);
        const T* k1 = cptr<T>(ws, lay.k1[l]);
        T* gr1 = l > 1 ? mptr<T>(ws, tl.gr1[l]) : nullptr;
        if (l == 1)
            NPS_TRY(launch("train_bwd_down", (double)ncells(g), s, [&] {
                k_bwd_down<T, true, true, WP><<<grid, kBlock, 0, s>>>(img(l), g, gx1, gr_next, r1, k1, gr1, wpart);
            }));
        else
            NPS_TRY(launch("train_bwd_down", (double)ncells(g), s, [&] {
                k_bwd_down<T, false, true, WP><<<grid, kBlock, 0, s>>>(img(l), g, gx1, gr_next, r1, k1, gr1, wpart);
            }));
        const double scale = std::ldexp(1.0, -3 * (l - 1));
        double* gW = grad + off_c1(l);
        NPS_TRY(wgrad_reduce(wpart, grid, scale, gW, nullptr, s));
    }
    (void)st;
    return NPS_OK;
}

template <class T>
int train_loss(const uint8_t* labels, nps_dims d, const TrainLayout& tl, void* ws, const T* b, const T* y, T* gy,
               double* loss_h, hipStream_t s) {
    const Layout& lay = tl.base;
    const Grid g = level_grid(d, 1);
    State* st = mptr<State>(ws, lay.state);
    double* partials = mptr<double>(ws, lay.partials);
    T* res = mptr<T>(ws, tl.res);
    const int grid = tile_grid(g);
    NPS_TRY(launch("train_residual", (double)ncells(g), s, [&] {
        k_train_residual<T><<<grid, kBlock, 0, s>>>(labels, g, b, y, res, partials);
    }));
    NPS_TRY(launch("control", 0, s, [&] {
        k_control<kStageLoss><<<1, kCtlBlock, 0, s>>>(st, partials, grid, 0, 0, 0, 0, 0.0, 0.0, 0.0, nullptr);
    }));
    NPS_TRY(launch("train_gy", (double)ncells(g), s, [&] { k_train_gy<T><<<grid, kBlock, 0, s>>>(labels, g, res, st, gy, 1.0); }));
    double rr = 0.0;
    NPS_HIP(hipMemcpyAsync(&rr, &st->rr, sizeof(double), hipMemcpyDeviceToHost, s));
    NPS_HIP(hipStreamSynchronize(s));
    *loss_h = std::sqrt(rr);
    return NPS_OK;
}

// One step over a batch (the mean loss of Sec. "Training"): the systems run
// one after another in the same workspace, each forward keeping its per-level
// activations for its own backward; the loss gradient of each is weighed by
// 1/batch, so the backward passes add the gradient of the mean.
template <class T, int WP>
int train_step(const nps_net* net, const uint8_t* labels, nps_dims d, int batch, const T* b, double* grad,
               double* loss_h, const TrainLayout& tl, void* ws, hipStream_t s, bool bf16w) {
    const Layout& lay = tl.base;
    const Grid g = level_grid(d, 1);
    const size_t n = ncells(g);
    State* st = mptr<State>(ws, lay.state);
    double* partials = mptr<double>(ws, lay.partials);
    T* res = mptr<T>(ws, tl.res);
    T* y = mptr<T>(ws, tl.y);
    T* gy = mptr<T>(ws, tl.gy);
    double* lacc = mptr<double>(ws, tl.lacc);
    const double w = 1.0 / batch;
    const int grid = tile_grid(g);
    NPS_TRY(launch("train_loss_sum", 0, s, [&] { k_loss_accumulate<<<1, 1, 0, s>>>(st, lacc, 0.0, 1); }));
    for (int i = 0; i < batch; ++i) {
        const uint8_t* lab = labels + (size_t)i * n;
        const T* bi = b + (size_t)i * n;
        NPS_TRY(train_forward<T>(net, lab, d, tl, ws, bi, y, s, bf16w));
        NPS_TRY(launch("train_residual", (double)n, s, [&] {
            k_train_residual<T><<<grid, kBlock, 0, s>>>(lab, g, bi, y, res, partials);
        }));
        NPS_TRY(launch("control", 0, s, [&] {
            k_control<kStageLoss><<<1, kCtlBlock, 0, s>>>(st, partials, grid, 0, 0, 0, 0, 0.0, 0.0, 0.0, nullptr);
        }));
        NPS_TRY(launch("train_gy", (double)n, s, [&] { k_train_gy<T><<<grid, kBlock, 0, s>>>(lab, g, res, st, gy, w); }));
        NPS_TRY(launch("train_loss_sum", 0, s, [&] { k_loss_accumulate<<<1, 1, 0, s>>>(st, lacc, w, 0); }));
        NPS_TRY((train_backward<T, WP>(net, lab, d, tl, ws, bi, gy, grad, s)));
    }
    NPS_HIP(hipMemcpyAsync(loss_h, lacc, sizeof(double), hipMemcpyDeviceToHost, s));
    NPS_HIP(hipStreamSynchronize(s));
    return NPS_OK;
}

// Training precisions: NPS_FP64 (double vectors, vector-ALU parameter sums),
// NPS_FP32 (float vectors, fp32 matrix-core sums), NPS_MIXED_BF16 (float
// vectors, kernels from bf16-rounded weights, bf16 matrix-core sums with fp32
// accumulation).
bool train_precision_ok(int p) { return p == NPS_FP64 || p == NPS_FP32 || p == NPS_MIXED_BF16; }

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of the no-allocation entry point
// ---------------------------------------------------------------------------
// The workspace of nps_apply_precond_noalloc: a file-scope device array that
// every GPU the library runs on holds until the process ends.  In host code
// `scratch` is only a stand-in symbol: its device address, different on each
// device, comes from hipGetSymbolAddress, taken once per device with that
// device current and kept in g_scratch_dev.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of the current device's scratch.
int scratch_address(void** out) {
    int dev = 0;
    NPS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NPS_EDEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(NPS_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return NPS_OK;
}

}  // namespace

extern "C" {

size_t nps_param_count(int levels) {
    if (levels < 1) return 0;
    return (size_t)(2 * levels - 1) * (27 * 81 + 27) + (size_t)2 * (levels - 1) * (81 + 1);
}

size_t nps_net_bytes(int levels) {
    if (levels < 2 || levels > kMaxLevels) return 0;
    size_t a, b, c, e;
    return net_sizes(levels, &a, &b, &c, &e);
}

int nps_net_levels(const nps_net* net) { return net ? net->levels : 0; }

int nps_net_create(const double* params_h, size_t n_params, int levels, void* dev_buf_d, size_t dev_bytes,
                   void* stream, nps_net** out) {
    if (!params_h || !dev_buf_d || !out) return fail(NPS_EINVAL, "null argument");
    if (levels < 2 || levels > kMaxLevels) return fail(NPS_EINVAL, "levels must be in [2, %d]", kMaxLevels);
    if (n_params != nps_param_count(levels))
        return fail(NPS_EINVAL, "blob has %zu parameters, expected %zu", n_params, nps_param_count(levels));
    if (reinterpret_cast<uintptr_t>(dev_buf_d) % 256) return fail(NPS_EINVAL, "device buffer not 256-byte aligned");
    size_t o64, o32, omf, oaff, obf, obf32;
    const size_t need = net_sizes(levels, &o64, &o32, &omf, &oaff, &obf, &obf32);
    if (dev_bytes < need) return fail(NPS_ENOMEM, "device buffer has %zu bytes, needs %zu", dev_bytes, need);
    for (size_t i = 0; i < n_params; ++i)
        if (!std::isfinite(params_h[i])) return fail(NPS_ENONFINITE, "parameter %zu is not finite", i);

    std::vector<char> host(need, 0);
    const int nb = 2 * levels - 1;
    auto* w64 = reinterpret_cast<CConvW<double>*>(host.data() + o64);
    auto* w32 = reinterpret_cast<CConvW<float>*>(host.data() + o32);
    auto* wmf = reinterpret_cast<MfmaW*>(host.data() + omf);
    auto* aff = reinterpret_cast<AffW*>(host.data() + oaff);
    auto* wbf = reinterpret_cast<CConvW<double>*>(host.data() + obf);
    auto* wbf32 = reinterpret_cast<CConvW<float>*>(host.data() + obf32);
    nps_net* net = new nps_net();
    const double* p = params_h;
    const size_t cw = 27 * 81, cb = 27;
    for (int l = 1; l <= levels; ++l) {              // CConv_1^l
        to_count_form(p, p + cw, l, w64[l - 1]);
        p += cw + cb;
    }
    for (int l = 1; l < levels; ++l) {               // CConv_2^l
        to_count_form(p, p + cw, l, w64[levels + l - 1]);
        p += cw + cb;
    }
    for (int l = 1; l < levels; ++l) {               // Aff_1^l, Aff_2^l
        for (int which = 0; which < 2; ++which) {
            AffW& a = aff[2 * (l - 1) + which];
            for (int c = 0; c < 3; ++c)
                for (int o = 0; o < kTaps; ++o) a.w[c][o] = p[c * kTaps + o];
            a.b = p[81];
            net->aff_b[2 * (l - 1) + which] = p[81];
            p += 82;
        }
    }
    for (int b = 0; b < nb; ++b) {
        const CConvW<double>& s = w64[b];
        CConvW<float>& t = w32[b];
        for (int i = 0; i < kTaps; ++i) t.C[i] = (float)s.C[i];
        for (int o = 0; o < kTaps; ++o)
            for (int i = 0; i < kTaps; ++i)
                for (int c = 0; c < 2; ++c) t.D[o][i][c] = (float)s.D[o][i][c];
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < kTaps; ++i) t.Kpure[c][i] = (float)s.Kpure[c][i];
        to_mfma(s, wmf[b]);
        // bf16-rounded count form: the single bf16 piece the mixed path's matrix
        // cores use; the pure-window kernels follow from the rounded values
        CConvW<double>& r = wbf[b];
        const int lvl = b < levels ? b + 1 : b - levels + 1;
        const double full = std::ldexp(1.0, 3 * (lvl - 1));
        for (int t = 0; t < kTaps; ++t) {
            r.C[t] = bf16_value(bf16_rne((float)s.C[t]));
            double kf = r.C[t], ka = r.C[t];
            for (int o = 0; o < kTaps; ++o)
                for (int c = 0; c < 2; ++c) {
                    r.D[o][t][c] = bf16_value(bf16_rne((float)s.D[o][t][c]));
                    (c == 0 ? kf : ka) += r.D[o][t][c] * full;
                }
            r.Kpure[kFluid][t] = kf;
            r.Kpure[kAir][t] = ka;
            r.Kpure[kSolid][t] = r.C[t];
        }
        CConvW<float>& r32 = wbf32[b];
        for (int i = 0; i < kTaps; ++i) r32.C[i] = (float)r.C[i];
        for (int o = 0; o < kTaps; ++o)
            for (int i = 0; i < kTaps; ++i)
                for (int c = 0; c < 2; ++c) r32.D[o][i][c] = (float)r.D[o][i][c];
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < kTaps; ++i) r32.Kpure[c][i] = (float)r.Kpure[c][i];
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(dev_buf_d, host.data(), need, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete net;
        return fail(NPS_EDEVICE, "copy of the network to the device failed: %s", hipGetErrorString(e));
    }
    net->levels = levels;
    net->dev = static_cast<char*>(dev_buf_d);
    net->off_w64 = o64;
    net->off_w32 = o32;
    net->off_mfma = omf;
    net->off_aff = oaff;
    net->off_wbf = obf;
    net->off_wbf32 = obf32;
    *out = net;
    return NPS_OK;
}

void nps_net_destroy(nps_net* net) { delete net; }

size_t nps_workspace_bytes(nps_dims dims, int levels, int precision, int n_ortho) {
    if (check_dims(dims, levels) != NPS_OK) return 0;
    if (precision < NPS_FP64 || precision > NPS_MIXED_FP16) return 0;
    if (n_ortho < 0 || n_ortho > kMaxOrtho) return 0;
    return make_layout(dims, levels, precision, n_ortho, true).total;
}

size_t nps_solve_workspace_bytes(nps_dims dims, int levels, const nps_opts* opts) {
    if (!opts || check_dims(dims, levels) != NPS_OK || check_opts(*opts) != NPS_OK) return 0;
    return solve_layout(dims, levels, *opts).total;
}

int nps_solve(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const double* b_d, double* x_d,
              const nps_opts* opts, nps_info* info, void* ws_d, size_t ws_bytes, void* stream) {
    if (!net || !labels_d || !b_d || !x_d || !opts || !info || !ws_d) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_dims(dims, net->levels));
    const nps_opts& o = *opts;
    NPS_TRY(check_opts(o));
    const SolveLayout sl = solve_layout(dims, net->levels, o);
    if (ws_bytes < sl.total) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, sl.total);
    if (reinterpret_cast<uintptr_t>(ws_d) % 256) return fail(NPS_EINVAL, "workspace not 256-byte aligned");
    std::memset(info, 0, sizeof(*info));
    HostMirror* hm = host_mirror();
    if (!hm) return fail(NPS_EDEVICE, "hipHostMalloc of the host mirror failed");
    Solver* sv = make_solver(o.precision);
    sv->net = net;
    sv->labels = labels_d;
    sv->b = b_d;
    sv->d = dims;
    sv->o = o;
    sv->plan = sl.plan;
    sv->lay = sl.lay;
    sv->tl = sl.tl;
    sv->ws = ws_d;
    sv->s = static_cast<hipStream_t>(stream);
    sv->hs = hm->state;
    sv->hf = hm->flags;
    sv->hf_d = hm->flags_d;
    const int rc = run_solve(*sv, x_d, info);
    delete sv;
    return rc;
}

int nps_apply_laplacian(const uint8_t* labels_d, nps_dims dims, const void* x_d, void* y_d, int precision,
                        void* stream) {
    if (!labels_d || !x_d || !y_d) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_grid(dims));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid g{dims.nz, dims.ny, dims.nx};
    const int grid = std::min(tile_grid(g), 65536);
    const double cells = (double)ncells(g);
    if (precision == NPS_FP64)
        return launch("laplacian", cells, s, [&] {
            k_laplacian<double><<<grid, kBlock, 0, s>>>(labels_d, g, static_cast<const double*>(x_d),
                                                        static_cast<double*>(y_d));
        });
    if (precision == NPS_FP32)
        return launch("laplacian", cells, s, [&] {
            k_laplacian<float><<<grid, kBlock, 0, s>>>(labels_d, g, static_cast<const float*>(x_d),
                                                       static_cast<float*>(y_d));
        });
    return fail(NPS_EINVAL, "precision must be NPS_FP64 or NPS_FP32");
}

int nps_apply_precond(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* r_d, void* d_d,
                      int precision, void* ws_d, size_t ws_bytes, void* stream) {
    if (!net || !labels_d || !r_d || !d_d || !ws_d) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_dims(dims, net->levels));
    if (precision < NPS_FP64 || precision > NPS_MIXED_FP16) return fail(NPS_EINVAL, "unknown precision %d", precision);
    const Plan plan = make_plan(dims, net->levels, precision);
    const Layout lay = make_layout(dims, net->levels, precision, 0, false);
    if (ws_bytes < lay.total) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);
    if (reinterpret_cast<uintptr_t>(ws_d) % 256) return fail(NPS_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == NPS_FP64)
        return precond_impl<double>(net, labels_d, dims, static_cast<const double*>(r_d), static_cast<double*>(d_d),
                                    ws_d, plan, lay, s);
    return precond_impl<float>(net, labels_d, dims, static_cast<const float*>(r_d), static_cast<float*>(d_d), ws_d,
                               plan, lay, s);
}


int nps_apply_precond_noalloc(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* r_d, void* d_d,
                              int precision, void* stream) {
    if (!net || !labels_d || !r_d || !d_d) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_dims(dims, net->levels));
    if (precision < NPS_FP64 || precision > NPS_MIXED_FP16) return fail(NPS_EINVAL, "unknown precision %d", precision);
    const size_t need = make_layout(dims, net->levels, precision, 0, false).total;
    if (need > kScratchBytes)
        return fail(NPS_ENOMEM, "needs %zu bytes of scratch, the static buffer holds %zu", need, kScratchBytes);
    void* ws = nullptr;
    NPS_TRY(scratch_address(&ws));
    return nps_apply_precond(net, labels_d, dims, r_d, d_d, precision, ws, kScratchBytes, stream);
}

size_t nps_train_workspace_bytes(nps_dims dims, int levels, int precision) {
    if (check_dims(dims, levels) != NPS_OK) return 0;
    if (!train_precision_ok(precision)) return 0;
    return make_train_layout(dims, levels, precision).total;
}

int nps_net_forward(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* r_d, void* y_d,
                    int precision, void* ws_d, size_t ws_bytes, void* stream) {
    if (!net || !labels_d || !r_d || !y_d || !ws_d) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_dims(dims, net->levels));
    if (!train_precision_ok(precision)) return fail(NPS_EINVAL, "training precision must be FP64, FP32 or MIXED_BF16");
    const TrainLayout tl = make_train_layout(dims, net->levels, precision);
    if (ws_bytes < tl.total) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, tl.total);
    if (reinterpret_cast<uintptr_t>(ws_d) % 256) return fail(NPS_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == NPS_FP64)
        return train_forward<double>(net, labels_d, dims, tl, ws_d, static_cast<const double*>(r_d), static_cast<double*>(y_d), s);
    return train_forward<float>(net, labels_d, dims, tl, ws_d, static_cast<const float*>(r_d), static_cast<float*>(y_d), s,
                                precision == NPS_MIXED_BF16);
}

int nps_net_backward(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* r_d, const void* gy_d,
                     double* grad_d, int precision, void* ws_d, size_t ws_bytes, void* stream) {
    if (!net || !labels_d || !r_d || !gy_d || !grad_d || !ws_d) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_dims(dims, net->levels));
    if (!train_precision_ok(precision)) return fail(NPS_EINVAL, "training precision must be FP64, FP32 or MIXED_BF16");
    const TrainLayout tl = make_train_layout(dims, net->levels, precision);
    if (ws_bytes < tl.total) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, tl.total);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == NPS_FP64)
        return train_backward<double>(net, labels_d, dims, tl, ws_d, static_cast<const double*>(r_d),
                                      static_cast<const double*>(gy_d), grad_d, s);
    if (precision == NPS_MIXED_BF16)
        return train_backward<float, kWgMfmaBf16>(net, labels_d, dims, tl, ws_d, static_cast<const float*>(r_d),
                                                  static_cast<const float*>(gy_d), grad_d, s);
    return train_backward<float>(net, labels_d, dims, tl, ws_d, static_cast<const float*>(r_d),
                                 static_cast<const float*>(gy_d), grad_d, s);
}

int nps_train_step(const nps_net* net, const uint8_t* labels_d, nps_dims dims, int batch, const void* b_d,
                   double* grad_d, double* loss_h, int precision, void* ws_d, size_t ws_bytes, void* stream) {
    if (!net || !labels_d || !b_d || !grad_d || !loss_h || !ws_d) return fail(NPS_EINVAL, "null argument");
    if (batch < 1) return fail(NPS_EINVAL, "batch must be at least 1");
    NPS_TRY(check_dims(dims, net->levels));
    if (!train_precision_ok(precision)) return fail(NPS_EINVAL, "training precision must be FP64, FP32 or MIXED_BF16");
    const TrainLayout tl = make_train_layout(dims, net->levels, precision);
    if (ws_bytes < tl.total) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, tl.total);
    if (reinterpret_cast<uintptr_t>(ws_d) % 256) return fail(NPS_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == NPS_FP64)
        return train_step<double, kWgVector>(net, labels_d, dims, batch, static_cast<const double*>(b_d), grad_d, loss_h,
                                             tl, ws_d, s, false);
    if (precision == NPS_MIXED_BF16)
        return train_step<float, kWgMfmaBf16>(net, labels_d, dims, batch, static_cast<const float*>(b_d), grad_d, loss_h,
                                              tl, ws_d, s, true);
    return train_step<float, kWgMfma32>(net, labels_d, dims, batch, static_cast<const float*>(b_d), grad_d, loss_h, tl,
                                        ws_d, s, false);
}

int nps_train_loss(const uint8_t* labels_d, nps_dims dims, int levels, const void* b_d, const void* y_d, void* gy_d,
                   double* loss_h, int precision, void* ws_d, size_t ws_bytes, void* stream) {
    if (!labels_d || !b_d || !y_d || !gy_d || !loss_h || !ws_d) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_dims(dims, levels));
    if (!train_precision_ok(precision)) return fail(NPS_EINVAL, "training precision must be FP64, FP32 or MIXED_BF16");
    const TrainLayout tl = make_train_layout(dims, levels, precision);
    if (ws_bytes < tl.total) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, tl.total);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == NPS_FP64)
        return train_loss<double>(labels_d, dims, tl, ws_d, static_cast<const double*>(b_d), static_cast<const double*>(y_d),
                                  static_cast<double*>(gy_d), loss_h, s);
    return train_loss<float>(labels_d, dims, tl, ws_d, static_cast<const float*>(b_d), static_cast<const float*>(y_d),
                             static_cast<float*>(gy_d), loss_h, s);
}

int nps_apply_precond_transpose(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* g_d,
                                void* y_d, int precision, void* ws_d, size_t ws_bytes, void* stream) {
    if (!net || !labels_d || !g_d || !y_d || !ws_d) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_dims(dims, net->levels));
    if (precision != NPS_FP64 && precision != NPS_FP32) return fail(NPS_EINVAL, "precision must be FP64 or FP32");
    const TrainLayout tl = make_train_layout(dims, net->levels, precision);
    if (ws_bytes < tl.total) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, tl.total);
    if (reinterpret_cast<uintptr_t>(ws_d) % 256) return fail(NPS_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Plan plan = make_plan(dims, net->levels, precision, true);
    State* st = mptr<State>(ws_d, tl.base.state);
    NPS_TRY(launch("state_init", 0, s, [&] { k_state_init<<<1, 64, 0, s>>>(st, 0, 0, 0, 0, 0); }));
    if (precision == NPS_FP64) {
        NPS_TRY(run_setup<double>(net, labels_d, dims, plan, tl.base, ws_d, s));
        return adjoint_apply<double>(net, labels_d, dims, tl, ws_d, static_cast<const double*>(g_d),
                                     static_cast<double*>(y_d), s);
    }
    NPS_TRY(run_setup<float>(net, labels_d, dims, plan, tl.base, ws_d, s));
    return adjoint_apply<float>(net, labels_d, dims, tl, ws_d, static_cast<const float*>(g_d), static_cast<float*>(y_d),
                                s);
}

int nps_asymmetry(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* x_d, const void* y_d,
                  void* px_d, void* py_d, int precision, void* ws_d, size_t ws_bytes, double* s_h, void* stream) {
    if (!net || !labels_d || !x_d || !y_d || !px_d || !py_d || !ws_d || !s_h) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_dims(dims, net->levels));
    if (precision < NPS_FP64 || precision > NPS_MIXED_FP16) return fail(NPS_EINVAL, "unknown precision %d", precision);
    const Plan plan = make_plan(dims, net->levels, precision);
    const Layout lay = make_layout(dims, net->levels, precision, 0, false);
    if (ws_bytes < lay.total + 256) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total + 256);
    if (reinterpret_cast<uintptr_t>(ws_d) % 256) return fail(NPS_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = ncells(level_grid(dims, 1));
    double* partials = mptr<double>(ws_d, lay.partials);
    double* sums = mptr<double>(ws_d, lay.total);   // 4 doubles past the layout
    const int grid = red_elem_grid(n);
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        NPS_TRY(precond_impl<T>(net, labels_d, dims, static_cast<const T*>(x_d), static_cast<T*>(px_d), ws_d, plan, lay, s));
        NPS_TRY(precond_impl<T>(net, labels_d, dims, static_cast<const T*>(y_d), static_cast<T*>(py_d), ws_d, plan, lay, s));
        NPS_TRY(launch("asym_dots", (double)n, s, [&] {
            k_dot4<T><<<grid, kBlock, 0, s>>>(n, static_cast<const T*>(x_d), static_cast<const T*>(y_d),
                                              static_cast<const T*>(px_d), static_cast<const T*>(py_d), partials);
        }));
        return NPS_OK;
    };
    NPS_TRY(precision == NPS_FP64 ? run(0.0) : run(0.0f));
    NPS_TRY(launch("asym_sum", 0, s, [&] { k_sum_partials<<<1, kBlock, 0, s>>>(partials, grid, sums); }));
    double v[4];
    NPS_HIP(hipMemcpyAsync(v, sums, sizeof(v), hipMemcpyDeviceToHost, s));
    NPS_HIP(hipStreamSynchronize(s));
    const double den = std::sqrt(std::fabs(v[2]) * std::fabs(v[3]));
    *s_h = den > 0.0 ? std::fabs(v[0] - v[1]) / den : 0.0;
    return NPS_OK;
}

// ---------------------------------------------------------------------------
// Ritz-vector right-hand sides (training data of Sec. "Training")
// ---------------------------------------------------------------------------
namespace {

// One rocBLAS handle per device and host thread, created at first use.
rocblas_handle blas_handle() {
    thread_local rocblas_handle h[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    if (!h[dev] && rocblas_create_handle(&h[dev]) != rocblas_status_success) h[dev] = nullptr;
    return h[dev];
}

struct LanczosLayout {
    size_t w, h, partials, total;
};

LanczosLayout lanczos_layout(size_t n, int m) {
    LanczosLayout L{};
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes);
        return at;
    };
    L.w = put(sizeof(double) * n);
    L.h = put(sizeof(double) * (size_t)m);
    L.partials = put(sizeof(double) * kRedWidth * kMaxRedBlocks);
    L.total = off;
    return L;
}

struct RitzLayout {
    size_t d, e, y, z, info, total;
};

RitzLayout ritz_layout(int m, int k) {
    RitzLayout L{};
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes);
        return at;
    };
    L.d = put(sizeof(double) * (size_t)m);
    L.e = put(sizeof(double) * (size_t)m);
    L.y = put(sizeof(double) * (size_t)m * m);
    L.z = put(sizeof(double) * (size_t)m * k);
    L.info = put(sizeof(int));
    L.total = off;
    return L;
}

#define NPS_BLAS(call)                                                                             \
    do {                                                                                           \
        const rocblas_status st_ = (call);                                                         \
        if (st_ != rocblas_status_success)                                                         \
            return fail(NPS_EDEVICE, "%s failed: %s", #call, rocblas_status_to_string(st_));       \
    } while (0)

}  // namespace

size_t nps_lanczos_workspace_bytes(nps_dims dims, int m) {
    if (dims.nz <= 0 || dims.ny <= 0 || dims.nx <= 0 || m < 1) return 0;
    return lanczos_layout((size_t)dims.nz * dims.ny * dims.nx, m).total;
}

int nps_lanczos(const uint8_t* labels_d, nps_dims dims, int m, int reorth, const double* v0_d, double* V_d,
                double* alpha_d, double* beta_d, int* steps_h, void* ws_d, size_t ws_bytes, void* stream) {
    if (!labels_d || !v0_d || !V_d || !alpha_d || !beta_d || !steps_h || !ws_d) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_grid(dims));
    const size_t n = (size_t)dims.nz * dims.ny * dims.nx;
    if (m < 1 || n > (size_t)INT32_MAX) return fail(NPS_EINVAL, "need m >= 1 and fewer than 2^31 cells");
    const LanczosLayout L = lanczos_layout(n, m);
    if (ws_bytes < L.total) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (reinterpret_cast<uintptr_t>(ws_d) % 256) return fail(NPS_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    rocblas_handle hb = blas_handle();
    if (!hb) return fail(NPS_EDEVICE, "rocblas_create_handle failed");
    NPS_BLAS(rocblas_set_stream(hb, s));
    NPS_BLAS(rocblas_set_pointer_mode(hb, rocblas_pointer_mode_host));
    const Grid g{dims.nz, dims.ny, dims.nx};
    double* w = mptr<double>(ws_d, L.w);
    double* h = mptr<double>(ws_d, L.h);
    double* partials = mptr<double>(ws_d, L.partials);
    const int eg = std::min<int>(kLzBlocks, (int)((n + kBlock - 1) / kBlock));
    const int lg = std::min(tile_grid(g), 65536);
    const int ni = (int)n;
    const double one = 1.0, zero = 0.0, minus_one = -1.0;
    auto col = [&](int j) { return V_d + (size_t)j * n; };
    // v_1 = v0 restricted to fluid, normalised
    NPS_TRY(launch("lanczos_vec", (double)n, s, [&] { k_lz_mask<<<eg, kBlock, 0, s>>>(n, labels_d, v0_d, w); }));
    NPS_TRY(launch("lanczos_dot", (double)n, s, [&] { k_lz_dot<<<eg, kBlock, 0, s>>>(n, w, w, partials); }));
    NPS_TRY(launch("lanczos_reduce", 0, s, [&] { k_lz_reduce<true><<<1, kBlock, 0, s>>>(partials, eg, h); }));
    NPS_TRY(launch("lanczos_vec", (double)n, s, [&] { k_lz_scale<<<eg, kBlock, 0, s>>>(n, w, h, col(0)); }));
    for (int j = 0; j < m; ++j) {
        // w = A v_j; alpha_j = w . v_j; w -= alpha_j v_j + beta_(j-1) v_(j-1)
        NPS_TRY(launch("lanczos_matvec", (double)n, s, [&] { k_laplacian<double><<<lg, kBlock, 0, s>>>(labels_d, g, col(j), w); }));
        NPS_TRY(launch("lanczos_dot", (double)n, s, [&] { k_lz_dot<<<eg, kBlock, 0, s>>>(n, w, col(j), partials); }));
        NPS_TRY(launch("lanczos_reduce", 0, s, [&] { k_lz_reduce<false><<<1, kBlock, 0, s>>>(partials, eg, alpha_d + j); }));
        NPS_TRY(launch("lanczos_vec", (double)n, s, [&] {
            k_lz_update<<<eg, kBlock, 0, s>>>(n, w, col(j), j > 0 ? col(j - 1) : nullptr, alpha_d + j,
                                              j > 0 ? beta_d + j - 1 : nullptr);
        }));
        // full reorthogonalisation against v_1..v_(j+1), twice
        for (int pass = 0; pass < (reorth ? 2 : 0); ++pass) {
            NPS_BLAS(rocblas_dgemv(hb, rocblas_operation_transpose, ni, j + 1, &one, V_d, ni, w, 1, &zero, h, 1));
            NPS_BLAS(rocblas_dgemv(hb, rocblas_operation_none, ni, j + 1, &minus_one, V_d, ni, h, 1, &one, w, 1));
        }
        // beta_j = ||w||; v_(j+1) = w / beta_j
        NPS_TRY(launch("lanczos_dot", (double)n, s, [&] { k_lz_dot<<<eg, kBlock, 0, s>>>(n, w, w, partials); }));
        NPS_TRY(launch("lanczos_reduce", 0, s, [&] { k_lz_reduce<true><<<1, kBlock, 0, s>>>(partials, eg, beta_d + j); }));
        if (j + 1 < m)
            NPS_TRY(launch("lanczos_vec", (double)n, s, [&] {
                k_lz_next<<<eg, kBlock, 0, s>>>(n, w, beta_d + j, alpha_d, col(j + 1));
            }));
    }
    // steps: the first j whose beta fell below the threshold, plus one
    std::vector<double> a(m), b(m);
    NPS_HIP(hipMemcpyAsync(a.data(), alpha_d, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    NPS_HIP(hipMemcpyAsync(b.data(), beta_d, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    NPS_HIP(hipStreamSynchronize(s));
    const double thr = 1e-12 * std::max(std::fabs(a[0]), 1.0);
    int steps = m;
    for (int j = 0; j < m; ++j)
        if (!(b[j] >= thr)) {
            steps = j + 1;
            break;
        }
    *steps_h = steps;
    return NPS_OK;
}

size_t nps_ritz_workspace_bytes(int m, int k) {
    if (m < 1 || k < 1) return 0;
    return ritz_layout(m, k).total;
}

int nps_ritz_rhs(const double* V_d, nps_dims dims, int m, const double* alpha_d, const double* beta_d,
                 const double* coef_d, int k, double* rhs_d, double* theta_d, void* ws_d, size_t ws_bytes, void* stream) {
    if (!V_d || !alpha_d || !beta_d || !coef_d || !rhs_d || !theta_d || !ws_d) return fail(NPS_EINVAL, "null argument");
    if (dims.nz <= 0 || dims.ny <= 0 || dims.nx <= 0) return fail(NPS_ESHAPE, "dims must be positive");
    const size_t n = (size_t)dims.nz * dims.ny * dims.nx;
    if (m < 1 || k < 1 || n > (size_t)INT32_MAX) return fail(NPS_EINVAL, "need m, k >= 1 and fewer than 2^31 cells");
    const RitzLayout L = ritz_layout(m, k);
    if (ws_bytes < L.total) return fail(NPS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (reinterpret_cast<uintptr_t>(ws_d) % 256) return fail(NPS_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    rocblas_handle hb = blas_handle();
    if (!hb) return fail(NPS_EDEVICE, "rocblas_create_handle failed");
    NPS_BLAS(rocblas_set_stream(hb, s));
    NPS_BLAS(rocblas_set_pointer_mode(hb, rocblas_pointer_mode_host));
    double* D = mptr<double>(ws_d, L.d);
    double* E = mptr<double>(ws_d, L.e);
    double* Y = mptr<double>(ws_d, L.y);
    double* Z = mptr<double>(ws_d, L.z);
    int* info_d = mptr<int>(ws_d, L.info);
    // Ritz pairs of T_m (eigenvalues ascending into D, eigenvectors into Y)
    NPS_HIP(hipMemcpyAsync(D, alpha_d, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    if (m > 1) NPS_HIP(hipMemcpyAsync(E, beta_d, sizeof(double) * (m - 1), hipMemcpyDeviceToDevice, s));
    NPS_TRY(launch("ritz_identity", 0, s, [&] {
        k_identity<<<std::min<int>(1024, (int)(((size_t)m * m + kBlock - 1) / kBlock)), kBlock, 0, s>>>(m, Y);
    }));
    NPS_BLAS(rocsolver_dstedc(hb, rocblas_evect_tridiagonal, m, D, E, Y, m, info_d));
    int info = 0;
    NPS_HIP(hipMemcpyAsync(&info, info_d, sizeof(int), hipMemcpyDeviceToHost, s));
    NPS_HIP(hipMemcpyAsync(theta_d, D, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    // Z = Y C (m x k), rhs = V Z (n x k), columns scaled to unit norm
    const double one = 1.0, zero = 0.0;
    NPS_BLAS(rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, m, k, m, &one, Y, m, coef_d, m, &zero, Z,
                           m));
    NPS_BLAS(rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, (int)n, k, m, &one, V_d, (int)n, Z, m,
                           &zero, rhs_d, (int)n));
    NPS_TRY(launch("ritz_unit_columns", (double)n * k, s, [&] { k_unit_columns<<<k, 1024, 0, s>>>(n, rhs_d); }));
    NPS_HIP(hipStreamSynchronize(s));
    if (info != 0) return fail(NPS_EBREAKDOWN, "tridiagonal eigensolver did not converge (%d)", info);
    return NPS_OK;
}

int nps_profile_enable(int on) {
    g_prof.on = on != 0;
    return NPS_OK;
}

int nps_profile_read(nps_kernel_stat* out_h, int max_records, int* n_records) {
    if (!n_records || (max_records > 0 && !out_h)) return fail(NPS_EINVAL, "null argument");
    Prof& p = g_prof;
    std::vector<nps_kernel_stat> agg;
    int rc = NPS_OK;
    if (!p.recs.empty()) {
        if (hipEventSynchronize(p.pool[p.recs.back().ev1]) != hipSuccess) rc = fail(NPS_EDEVICE, "event sync failed");
    }
    for (const ProfRec& r : p.recs) {
        if (rc) break;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.pool[r.ev0], p.pool[r.ev1]) != hipSuccess) {
            rc = fail(NPS_EDEVICE, "hipEventElapsedTime failed");
            break;
        }
        auto it = std::find_if(agg.begin(), agg.end(), [&](const nps_kernel_stat& k) { return !std::strcmp(k.name, r.name); });
        if (it == agg.end()) {
            nps_kernel_stat k = {};
            std::snprintf(k.name, sizeof k.name, "%s", r.name);
            agg.push_back(k);
            it = agg.end() - 1;
        }
        it->launches += 1;
        it->total_ms += ms;
        it->cells += r.cells;
    }
    const bool overflow = p.overflow;
    p.recs.clear();
    p.next = 0;
    p.overflow = false;
    *n_records = (int)agg.size();
    for (int i = 0; i < (int)agg.size() && i < max_records; ++i) out_h[i] = agg[i];
    if (rc) return rc;
    if (overflow) return fail(NPS_ENOMEM, "more than %zu timing events; later launches were not recorded", kMaxProfEvents / 2);
    return NPS_OK;
}


int nps_server_create(const nps_net* net, size_t hbm_budget, int max_slots, nps_server** out) {
    if (!net || !out) return fail(NPS_EINVAL, "null argument");
    if (max_slots < 1 || max_slots > 64) return fail(NPS_EINVAL, "max_slots must be in [1, 64]");
    if (hbm_budget < (1u << 20)) return fail(NPS_EINVAL, "hbm_budget too small");
    nps_server* srv = new nps_server();
    srv->net = net;
    srv->budget = align256(hbm_budget);
    if (hipMalloc((void**)&srv->arena_d, srv->budget) != hipSuccess) {
        delete srv;
        return fail(NPS_ENOMEM, "cannot allocate a %zu-byte arena", hbm_budget);
    }
    srv->arena.init(srv->budget);
    const size_t per = ((sizeof(State) + sizeof(HostFlags) + 255) / 256) * 256;
    if (hipHostMalloc(&srv->mirror, per * max_slots, hipHostMallocMapped) != hipSuccess) {
        (void)hipFree(srv->arena_d);
        delete srv;
        return fail(NPS_EDEVICE, "hipHostMalloc of the slot mirrors failed");
    }
    srv->slots.resize(max_slots);
    for (int i = 0; i < max_slots; ++i) {
        Slot& sl = srv->slots[i];
        char* m = static_cast<char*>(srv->mirror) + per * i;
        sl.hs = reinterpret_cast<State*>(m);
        sl.hf = reinterpret_cast<HostFlags*>(m + sizeof(State));
        void* d = nullptr;
        bool ok = hipHostGetDevicePointer(&d, sl.hf, 0) == hipSuccess;
        sl.hf_d = static_cast<HostFlags*>(d);
        ok = ok && hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&sl.ev[0], hipEventDisableTiming) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&sl.ev[1], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            nps_server_destroy(srv);
            return fail(NPS_EDEVICE, "stream/event creation failed");
        }
    }
    *out = srv;
    return NPS_OK;
}

void nps_server_destroy(nps_server* srv) {
    if (!srv) return;
    for (Slot& sl : srv->slots) {
        if (sl.s) (void)hipStreamSynchronize(sl.s);
        delete sl.sv;
        if (sl.ev[0]) (void)hipEventDestroy(sl.ev[0]);
        if (sl.ev[1]) (void)hipEventDestroy(sl.ev[1]);
        if (sl.s) (void)hipStreamDestroy(sl.s);
    }
    for (auto& kv : srv->live) {
        Request* r = kv.second;
        srv->pool.put(r->n, r->lab_h);
        srv->pool.put(8 * r->n, r->b_h);
        srv->pool.put(8 * r->n, r->x_h);
        delete r;
    }
    if (srv->arena_d) (void)hipFree(srv->arena_d);
    if (srv->mirror) (void)hipHostFree(srv->mirror);
    delete srv;
}

size_t nps_server_request_bytes(const nps_server* srv, nps_dims dims, const nps_opts* opts) {
    if (!srv || !opts || check_dims(dims, srv->net->levels) != NPS_OK || check_opts(*opts) != NPS_OK) return 0;
    return request_layout(dims, srv->net->levels, *opts).total;
}

int nps_server_submit(nps_server* srv, const uint8_t* labels_h, nps_dims dims, const double* b_h,
                      const nps_opts* opts, uint64_t* req_id) {
    if (!srv || !labels_h || !b_h || !opts || !req_id) return fail(NPS_EINVAL, "null argument");
    NPS_TRY(check_dims(dims, srv->net->levels));
    NPS_TRY(check_opts(*opts));
    const size_t bytes = request_layout(dims, srv->net->levels, *opts).total;
    if (bytes > srv->budget) return fail(NPS_ENOMEM, "request needs %zu bytes, the arena has %zu", bytes, srv->budget);
    Request* r = new Request();
    r->id = srv->next_id++;
    r->d = dims;
    r->o = *opts;
    r->n = ncells(level_grid(dims, 1));
    r->bytes = bytes;
    r->lab_u = labels_h;
    r->b_u = b_h;
    r->t_submit = Clock::now();
    srv->queue.push_back(r);
    srv->live[r->id] = r;
    *req_id = r->id;
    return NPS_OK;
}

int nps_server_step(nps_server* srv, int* n_active, int* n_queued) {
    if (!srv) return fail(NPS_EINVAL, "null argument");
    for (Slot& sl : srv->slots)
        if (sl.req) NPS_TRY(advance(srv, sl));
    // admission, first in first out, while a slot and arena space are free
    while (!srv->queue.empty()) {
        Request* r = srv->queue.front();
        Slot* free_slot = nullptr;
        for (Slot& sl : srv->slots)
            if (!sl.req) {
                free_slot = &sl;
                break;
            }
        if (!free_slot || !srv->arena.alloc(r->bytes, &r->off)) break;
        srv->queue.pop_front();
        NPS_TRY(admit(srv, *free_slot, r));
    }
    int active = 0;
    for (Slot& sl : srv->slots) active += sl.req != nullptr;
    if (n_active) *n_active = active;
    if (n_queued) *n_queued = (int)srv->queue.size();
    return NPS_OK;
}

int nps_server_poll(nps_server* srv, uint64_t req_id, double* x_h, nps_info* info, double* latency_ms) {
    if (!srv) return fail(NPS_EINVAL, "null argument");
    auto it = srv->live.find(req_id);
    if (it == srv->live.end()) return fail(NPS_EINVAL, "unknown request %llu", (unsigned long long)req_id);
    Request* r = it->second;
    if (r->phase != Request::kDone) return NPS_PENDING;
    // a request rejected before its solve ran leaves x_h untouched (hard error)
    if (x_h && r->x_ready) std::memcpy(x_h, r->x_h, 8 * r->n);
    if (info) *info = r->info;
    if (info) info->status = r->status;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    const int st = r->status;
    srv->pool.put(8 * r->n, r->x_h);
    srv->live.erase(it);
    delete r;
    return st;
}

const char* nps_last_error(void) { return g_err.c_str(); }

}  // extern "C"
