// msg_host.cpp -- C-ABI (include/msg.h) and host scheduler of the batched
// MSG solver: layout, workspace plan, the F-cycle level loop and the
// recursive mu-cycle, issuing the kernels of msg_kernels.hip.
//
// Paper: Robbe, Nuyens, Vandewalle, arXiv 1907.12334, Section 2 (Algorithm
// MSG mu-cycle, Algorithm MSG F-cycle).  Each grid (p,q) of F-cycle level L
// is one "problem": it is iterated with mu-cycles over its own rectangle
// [0..p] x [0..q]; problems with the same (p,q) form a "class" and share one
// launch per kernel, whatever samples they come from.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/msg.h"
#include "matern_kernels.hpp"
#include "msg_device.hpp"
#include "msg_internal.hpp"
#include "msg_kernels.hpp"

using namespace msg;

namespace {

thread_local std::string g_err;

msg_status fail(msg_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(MSG_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- validation
msg_status check_batch(const msg_batch_desc* b)
{
    if (!b) return fail(MSG_ERR_ARG, "batch descriptor is NULL");
    if (b->n_samples < 1) return fail(MSG_ERR_ARG, "n_samples must be >= 1 (got %d)", b->n_samples);
    if (b->c < 1 || b->c > 8) return fail(MSG_ERR_LAYOUT, "c must be in 1..8 (got %d)", b->c);
    if (!b->P || !b->Q) return fail(MSG_ERR_ARG, "P and Q arrays are required");
    for (int s = 0; s < b->n_samples; ++s) {
        const int P = b->P[s], Q = b->Q[s];
        if (P < 0 || Q < 0 || P > kMaxIndex || Q > kMaxIndex)
            return fail(MSG_ERR_LAYOUT, "sample %d: (P,Q) = (%d,%d) outside 0..%d", s, P, Q, kMaxIndex);
        if (((int64_t)b->c << P) > 32768 || ((int64_t)b->c << Q) > 32768)
            return fail(MSG_ERR_LAYOUT, "sample %d: finest grid side above 32768 cells", s);
    }
    return MSG_OK;
}

msg_status check_opts(const msg_solve_opts* o)
{
    if (!o) return fail(MSG_ERR_ARG, "options are NULL");
    if (o->mu < 1 || o->mu > 3) return fail(MSG_ERR_ARG, "mu must be 1..3");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 > 16 || o->nu2 > 16) return fail(MSG_ERR_ARG, "nu1, nu2 must be 0..16");
    if (o->max_cycles < 0 || o->max_cycles > 100000) return fail(MSG_ERR_ARG, "max_cycles out of range");
    if (!(o->tol >= 0.0)) return fail(MSG_ERR_ARG, "tol must be >= 0");
    if (!std::isfinite(o->omega)) return fail(MSG_ERR_ARG, "omega must be finite");
    if (o->precision != MSG_FP64 && o->precision != MSG_MIXED) return fail(MSG_ERR_ARG, "unknown precision");
    if (o->tail_levels < -1 || o->tail_levels > 8) return fail(MSG_ERR_ARG, "tail_levels must be -1..8");
    if (o->handoff < -1) return fail(MSG_ERR_ARG, "handoff must be >= -1");
    if (o->overlap < -1 || o->overlap > 2) return fail(MSG_ERR_ARG, "overlap must be -1..2");
    if (o->tail_budget != 0 && (o->tail_budget < 1024 || o->tail_budget > 153600))
        return fail(MSG_ERR_ARG, "tail_budget must be 0 or 1024..153600 bytes");
    if (o->tile_width != 0 && (o->tile_width < 4 || o->tile_width > 256 || (o->tile_width & (o->tile_width - 1))))
        return fail(MSG_ERR_ARG, "tile_width must be 0 or a power of two in 4..256");
    if (o->tile_cells != 0 && (o->tile_cells < 64 || o->tile_cells > 4096))
        return fail(MSG_ERR_ARG, "tile_cells must be 0 or 64..4096");
    if (o->tile_lds != 0 && (o->tile_lds < 256 || o->tile_lds > kRbgsLdsMax))
        return fail(MSG_ERR_ARG, "tile_lds must be 0 or 256..%d elements", kRbgsLdsMax);
    if (o->graphs < 0 || o->graphs > 1) return fail(MSG_ERR_ARG, "graphs must be 0 or 1");
    return MSG_OK;
}

// ---------------------------------------------------------------- layout
struct BatchLayout {
    int S, c;
    std::vector<int> P, Q;
    std::vector<int64_t> cell, xf, yf, grid, top;   // S+1 prefix arrays (top: finest-grid cells)
    int maxL;
};

BatchLayout make_layout(const msg_batch_desc* b)
{
    BatchLayout L;
    L.S = b->n_samples;
    L.c = b->c;
    L.P.assign(b->P, b->P + L.S);
    L.Q.assign(b->Q, b->Q + L.S);
    L.cell.assign(L.S + 1, 0);
    L.xf.assign(L.S + 1, 0);
    L.yf.assign(L.S + 1, 0);
    L.grid.assign(L.S + 1, 0);
    L.top.assign(L.S + 1, 0);
    L.maxL = 0;
    for (int s = 0; s < L.S; ++s) {
        const int P = L.P[s], Q = L.Q[s];
        L.cell[s + 1] = L.cell[s] + sample_cells(L.c, P, Q);
        L.xf[s + 1] = L.xf[s] + sample_xfaces(L.c, P, Q);
        L.yf[s + 1] = L.yf[s] + sample_yfaces(L.c, P, Q);
        L.grid[s + 1] = L.grid[s] + (int64_t)(P + 1) * (Q + 1);
        L.top[s + 1] = L.top[s] + ((int64_t)L.c << P) * ((int64_t)L.c << Q);
        L.maxL = std::max(L.maxL, P + Q);
    }
    return L;
}

// ---------------------------------------------------------------- plans
constexpr int kSideStreams = 4;   // W-cycles of sub-batches run on these, forked from the caller's stream
int g_side = 4;                   // side streams in use (at most kSideStreams; MSG_SIDE_STREAMS)
int g_fuse = 2;              // smoother sweeps fused per pass (1 or 2)
int g_rbgs_tw = 64;          // smoother tile: widest, most cells, LDS elements
int g_rbgs_cells = 1024;
int g_rbgs_lds = kRbgsLds;
int g_tail_lds = 20480;      // LDS budget of the W-cycle tail (sets its depth)
int g_split_inner = 0;       // overlap mode inside each concurrently solved half (0 or 1)
int g_handoff = 1024;        // hand a class's last cycling problems to one kernel at or below this count
int g_tail_reg_levels = kTailRegLevels;   // tail levels 1..n with register-resident slot state
int g_solve_lds = 65536;     // LDS budget under which a class is solved entirely in one kernel
bool g_tail_table = true;    // tails smooth from a red-black slot table (false: decode every slot)
bool g_fuse_restrict = true; // pre-smoothing passes of nu1 = 2 also restrict their residual
bool g_fuse_visits = true;   // consecutive W-cycle visits of a level share one pass (see mu_cycle)
int g_cr_tw = 0, g_cr_cells = 0, g_cr_lds = 0;   // tiles of that shared pass (0: derived from the plain ones)
bool g_debug_stages = false; // per-level timing on stderr
constexpr size_t kWideTailLds = (size_t)40 * 1024;      // tails above this run on four wavefronts
constexpr int kMaxGroups = kMaxIndex + 1;               // lockstep groups of one stage (at most its classes)

// LDS elements of a smoother tile tw x th with halo H: its iterate with H
// cells of halo towards a neighbouring tile and one wall cell where the tile
// spans the grid.
int rbgs_lds(int nx, int ny, int H, int tw, int th)
{
    const int Hx = tw < nx ? H : 1, Hy = th < ny ? H : 1;
    return (tw + 2 * Hx) * (th + 2 * Hy);
}

// Plan parameters a caller may tune (msg_solve_opts; 0 there = the defaults)
struct Tuning {
    int tail_budget;   // LDS bytes per problem of the cycle tail
    int tile_w;        // smoother tile: widest
    int tile_cells;    //   most cells
    int tile_lds;      //   LDS elements with halo
};

Tuning tuning_of(const msg_solve_opts& o)
{
    return Tuning{o.tail_budget > 0 ? o.tail_budget : g_tail_lds, o.tile_width > 0 ? o.tile_width : g_rbgs_tw,
                  o.tile_cells > 0 ? o.tile_cells : g_rbgs_cells, o.tile_lds > 0 ? o.tile_lds : g_rbgs_lds};
}

// Smoother tile of a grid: up to tile_w cells wide and tile_cells cells in
// all, within tile_lds elements of LDS.
void rbgs_tile(int nx, int ny, int H, const Tuning& tu, int& tw, int& th)
{
    tw = std::min(nx, tu.tile_w);
    th = 1;
    while (th * 2 <= ny && tw * th * 2 <= tu.tile_cells && rbgs_lds(nx, ny, H, tw, th * 2) <= tu.tile_lds) th *= 2;
    if (th < ny && th * 2 > ny) {
        // non-power-of-two heights: take the largest fitting height
        int t = ny;
        while (t > th && (tw * t > tu.tile_cells || rbgs_lds(nx, ny, H, tw, t) > tu.tile_lds)) --t;
        th = std::max(th, t);
    }
    // a tile too narrow for its halo still works; one that cannot hold a
    // single row with halo falls back to the smallest
    if (rbgs_lds(nx, ny, H, tw, th) > kRbgsLdsMax) {
        tw = std::min(nx, 16);
        th = 1;
    }
}

struct ClassPlan {
    int pc, qc, L;
    int ci = 0;                    // index of the class inside its level
    int K = 0;
    int first = 0;                 // first problem of the class in the stage table
    int64_t arena = 0;             // arena offset of the class
    int64_t stride = 0;            // arena cells per problem
    std::vector<int64_t> goff;     // arena offset per grid a*(qc+1)+b
    int tail_top = 0;
    KTail tail;
    size_t tail_lds = 0;
    int tail_threads = 64;         // workgroup of the cycle tail (one wavefront, or four for large tails)
    bool solve_in_tail = false;    // the whole adaptive level runs in one kernel (FP64)
    KTail tail64;
    size_t tail64_lds = 0;
    KLevel top1d;                  // the finest grid, 1-D tiles
    std::vector<KLevel> rb, rbc, pro, res;   // per level: smoother tiles (rbc: with the correction's
                                             // children), prolongation, restriction into level-1
    std::vector<KLevel> rbr;                 // per level: the restricting pre-smoothing pass
    std::vector<KLevel> rbcr;                // per level: post-smoothing of one W-cycle visit and the
                                             // restricting pre-smoothing of the next, fused (may be empty)
    int64_t part0 = 0;             // first partial-sum slot
    int64_t tpack = -1;            // element offset of the class's tail conductance images, -1 if none
    std::vector<int> samples;
};

struct StagePlan {
    int L;
    std::vector<ClassPlan> classes;
    int K = 0;
    int64_t arena_cells = 0;
    int64_t part_slots = 0;
    int64_t tpack_elems = 0;       // tail conductance images of the classes cycled on the host
    int64_t slot_entries = 0;      // red-black slot tables of the classes' tails
};

int64_t grid_cells(int c, int a, int b) { return ((int64_t)c << a) * ((int64_t)c << b); }

// A level's grids in 1-D tiles of bs consecutive cells (bs = 0: kBlock; -1:
// 64 when every grid of the level is small, else kBlock).
KLevel level_1d(int c, int pc, int qc, int lev, const std::vector<int64_t>& goff, int rel /*0 none, 1 children, 2 parents*/,
                int maxq, int bs = 0)
{
    KLevel K;
    std::memset(&K, 0, sizeof K);
    if (bs < 0) bs = grid_cells(c, 0, lev) < 1024 ? 64 : kBlock;
    if (bs == 0) bs = kBlock;
    K.bs = bs;
    int tiles = 0;
    for (int a = 0; a <= pc; ++a) {
        const int b = lev - a;
        if (b < 0 || b > qc) continue;
        KGrid& G = K.g[K.ngrids++];
        G.nx = c << a;
        G.ny = c << b;
        G.p = a;
        G.q = b;
        G.tw = G.nx;
        G.th = 1;
        G.tiles_x = 1;
        G.tile0 = tiles;
        G.aoff = goff[a * (maxq + 1) + b];
        G.aoff_x = G.aoff_y = -1;
        if (rel == 1) {
            if (a > 0) G.aoff_x = goff[(a - 1) * (maxq + 1) + b];
            if (b > 0) G.aoff_y = goff[a * (maxq + 1) + b - 1];
        } else if (rel == 2) {
            if (a + 1 <= pc) G.aoff_x = goff[(a + 1) * (maxq + 1) + b];
            if (b + 1 <= qc) G.aoff_y = goff[a * (maxq + 1) + b + 1];
        }
        tiles += (int)ceil_div(grid_cells(c, a, b), bs);
    }
    K.ntiles = tiles;
    return K;
}

KLevel level_rbgs(int c, int pc, int qc, int lev, const std::vector<int64_t>& goff, int H, const Tuning& tu)
{
    KLevel K;
    std::memset(&K, 0, sizeof K);
    int tiles = 0, area = 0;
    for (int a = 0; a <= pc; ++a) {
        const int b = lev - a;
        if (b < 0 || b > qc) continue;
        KGrid& G = K.g[K.ngrids++];
        G.nx = c << a;
        G.ny = c << b;
        G.p = a;
        G.q = b;
        rbgs_tile(G.nx, G.ny, H, tu, G.tw, G.th);
        G.tiles_x = (int)ceil_div(G.nx, G.tw);
        G.tile0 = tiles;
        G.aoff = goff[a * (qc + 1) + b];
        G.aoff_x = G.aoff_y = -1;
        tiles += G.tiles_x * (int)ceil_div(G.ny, G.th);
        K.lds = std::max(K.lds, rbgs_lds(G.nx, G.ny, H, G.tw, G.th));
        area = std::max(area, G.tw * G.th);
    }
    K.ntiles = tiles;
    K.bs = area <= 256 ? 64 : kBlock;     // small tiles: more, smaller workgroups per CU
    return K;
}

// The restricting pre-smoothing pass of level lev (halo H + 1 = 5): tiles of
// grids with q >= 1 get an even height so that row pairs stay in one tile;
// aoff_x / aoff_y point at the children (p-1,q) and (p,q-1), and rflags says
// which child has a second parent.
KLevel level_rbgs_restrict(int c, int pc, int qc, int lev, const std::vector<int64_t>& goff, int H, const Tuning& tu)
{
    KLevel K = level_rbgs(c, pc, qc, lev, goff, H + 1, tu);
    int tiles = 0, lds = 0, area = 0;
    for (int g = 0; g < K.ngrids; ++g) {
        KGrid& G = K.g[g];
        if (G.q >= 1 && (G.th & 1)) G.th = std::max(2, G.th - 1);
        G.tile0 = tiles;
        tiles += G.tiles_x * (int)ceil_div(G.ny, G.th);
        lds = std::max(lds, rbgs_lds(G.nx, G.ny, H + 1, G.tw, G.th));
        area = std::max(area, G.tw * G.th);
        G.aoff_x = G.p > 0 ? goff[(G.p - 1) * (qc + 1) + G.q] : -1;
        G.aoff_y = G.q > 0 ? goff[G.p * (qc + 1) + G.q - 1] : -1;
        G.rflags = (G.q + 1 <= qc ? 1 : 0) | (G.p + 1 <= pc ? 2 : 0);
    }
    K.ntiles = tiles;
    K.lds = lds;
    K.bs = area <= 256 ? 64 : kBlock;
    return K;
}

// LDS layout of the tail of class (pc,qc) with top level m (see KTail);
// returns its bytes, or 0 if it does not fit the descriptor
template <typename T>
size_t tail_layout(int c, int pc, int qc, int m, const std::vector<int64_t>& goff, KTail& TL)
{
    std::memset(&TL, 0, sizeof TL);
    if (m >= kMaxTailLevels) return 0;
    TL.top = m;
    TL.pc = pc;
    TL.qc = qc;
    TL.c = c;
    TL.lc = (c & (c - 1)) == 0 ? __builtin_ctz(c) : -1;
    // the face conductances of every level first (the image prepared per
    // stage), then the iterates and right-hand sides
    int64_t off = 0;
    for (int lev = 0; lev <= m; ++lev) {
        KTailLevel& L = TL.lvl[lev];
        const int pmin = std::max(0, lev - qc), pmax = std::min(pc, lev);
        L.pmin = pmin;
        L.ng = pmax - pmin + 1;
        const int64_t cells = grid_cells(c, 0, lev);
        L.cells = (int)cells;
        L.csh = (cells & (cells - 1)) == 0 ? __builtin_ctzll(cells) : -1;
        L.x0 = (int)off;
        for (int g = 0; g < L.ng; ++g) off += cells + ((int64_t)c << (lev - pmin - g));      // (nx+1) ny
        L.y0 = (int)off;
        for (int g = 0; g < L.ng; ++g) off += cells + ((int64_t)c << (pmin + g));            // nx (ny+1)
        if (lev == m)
            for (int g = 0; g < L.ng; ++g) TL.top_aoff[g] = goff[(pmin + g) * (qc + 1) + (lev - pmin - g)];
    }
    off = (off + 3) / 4 * 4;
    TL.nstat = (int)off;
    for (int lev = 0; lev <= m; ++lev) {
        KTailLevel& L = TL.lvl[lev];
        L.v0 = (int)off; off += (int64_t)L.cells * L.ng;
        L.b0 = (int)off; off += (int64_t)L.cells * L.ng;
    }
    TL.zero = (int)off;
    off += 1;
    if (off > (int64_t)1 << 30) return 0;
    // red-black slot table entries (pairs of cells: grids with an even width)
    int32_t ns = 0;
    for (int lev = 0; lev <= m; ++lev) {
        TL.slot_off[lev] = ns;
        ns += (TL.lvl[lev].cells / 2) * TL.lvl[lev].ng;
    }
    TL.nslots = (c & 1) ? 0 : ns;
    // levels whose slots fit one per lane of a wavefront keep their slot
    // state in registers (the small levels that a W-cycle visits most)
    TL.reg_levels = 0;
    if (TL.nslots > 0)
        for (int lev = 1; lev <= std::min(m, g_tail_reg_levels); ++lev) {
            if ((TL.lvl[lev].cells / 2) * TL.lvl[lev].ng > 64) break;
            TL.reg_levels = lev;
        }
    TL.lds_elems = (int)off;
    TL.chol_off = (int)(((size_t)off * sizeof(T) + 15) / 16 * 16);
    return (size_t)TL.chol_off + sizeof(double) * (size_t)c * c * c * c;
}

// faces of every tail grid plus the top level's cells (bytes of type T per problem)
double tail_bytes(const KTail& TL, size_t elem)
{
    double per = 0.0;
    for (int lev = 0; lev <= TL.top; ++lev) {
        const KTailLevel& L = TL.lvl[lev];
        for (int g = 0; g < L.ng; ++g) {
            const int p = L.pmin + g, q = lev - p;
            per += 2.0 * L.cells + (double)(TL.c << p) + (double)(TL.c << q);   // (nx+1) ny + nx (ny+1)
        }
        if (lev == TL.top) per += 3.0 * L.cells * L.ng;
    }
    return per * elem;
}

// deepest tail whose LDS image fits the budget: the phases of the tail are
// latency-bound, so several problems per CU must be resident to hide it
// (measured at 256x256 x 4096: 20 KB, levels 0..4 and eight problems per CU,
// beat 8, 28, 40 and 45 KB)
template <typename T>
int choose_tail(int c, int pc, int qc, int L, int req, size_t budget, const std::vector<int64_t>& goff)
{
    KTail TL;
    if (req >= 0) return std::min(req, L);
    int best = 0;
    for (int m = 0; m <= std::min(L, kMaxTailLevels - 1); ++m) {
        const size_t bytes = tail_layout<T>(c, pc, qc, m, goff, TL);
        if (bytes == 0 || bytes > budget) break;
        best = m;
    }
    return best;
}

// The plan of class (pc,qc) on stage L = pc + qc for the problems of
// `samples`: arena layout of its grids, tail, smoother tiles and transfer
// launches per level.  Stage tables (first problem, arena, partial sums, tail
// images) are set by the caller.  With `host_cycles` the class never runs
// its whole solve in one kernel.
ClassPlan plan_class(int c, int pc, int qc, std::vector<int> samples, const msg_solve_opts& o, const Tuning& tu,
                     bool host_cycles)
{
    const int L = pc + qc;
    const int H = 2 * g_fuse;
    ClassPlan C;
    C.pc = pc;
    C.qc = qc;
    C.L = L;
    C.samples = std::move(samples);
    C.K = (int)C.samples.size();
    C.goff.assign((size_t)(pc + 1) * (qc + 1), 0);
    int64_t off = 0;
    for (int a = 0; a <= pc; ++a)
        for (int b = 0; b <= qc; ++b) {
            C.goff[a * (qc + 1) + b] = off;
            off += grid_cells(c, a, b);
        }
    C.stride = off;
    // The default LDS budget per problem is set for thousands of resident
    // problems.  A caller solving few large problems (the request loop's
    // large-request lane) passes a larger one: the tail then holds more
    // levels (each level on chip halves the host level visits of a cycle),
    // runs on four wavefronts, and rectangles up to that budget are solved
    // whole in one kernel.  The plan depends on the options and the class
    // rectangle only, never on how many problems share the class, so a
    // sample's result does not depend on its batch.
    const size_t tail_budget = (size_t)tu.tail_budget;
    const size_t solve_budget = std::max((size_t)g_solve_lds, tail_budget);
    // classes whose whole rectangle fits in LDS run their adaptive
    // cycles inside one FP64 kernel; the others cycle on the host
    // down to a tail of levels 0..tail_top < L
    const size_t b64 = L < kMaxTailLevels ? tail_layout<double>(c, pc, qc, L, C.goff, C.tail64) : 0;
    C.tail64_lds = b64;
    if (o.tail_levels >= 0) C.solve_in_tail = L <= o.tail_levels && b64 > 0;
    else C.solve_in_tail = b64 > 0 && b64 <= solve_budget;
    if (L == 0) C.solve_in_tail = b64 > 0;
    if (host_cycles) C.solve_in_tail = false;
    const int mcap = std::max(0, L - 1);
    C.tail_top = o.precision == MSG_MIXED ? choose_tail<float>(c, pc, qc, mcap, o.tail_levels, tail_budget, C.goff)
                                           : choose_tail<double>(c, pc, qc, mcap, o.tail_levels, tail_budget, C.goff);
    C.tail_lds = o.precision == MSG_MIXED ? tail_layout<float>(c, pc, qc, C.tail_top, C.goff, C.tail)
                                           : tail_layout<double>(c, pc, qc, C.tail_top, C.goff, C.tail);
    C.tail_threads = C.tail_lds > kWideTailLds ? 256 : 64;
    C.top1d = level_1d(c, pc, qc, L, C.goff, 1, qc);
    C.rb.resize(L + 1);
    C.rbc.resize(L + 1);
    C.pro.resize(L + 1);
    C.res.resize(L + 1);
    C.rbr.resize(L + 1);
    // the fused pair of passes has a halo of 2 (2 + 2) + 1 cells: tiles twice
    // as wide and twice as large as the plain passes' keep its halo share
    // moderate (128 x 16 cells and 39 KB of LDS at the default plan)
    Tuning tu2 = tu;
    tu2.tile_w = g_cr_tw > 0 ? g_cr_tw : std::min(256, 2 * tu.tile_w);
    tu2.tile_cells = g_cr_cells > 0 ? g_cr_cells : std::min(4096, 2 * tu.tile_cells);
    tu2.tile_lds = std::min(kRbgsLdsMax, g_cr_lds > 0 ? g_cr_lds : std::max(4 * tu.tile_lds, 4096));
    if (g_fuse == 2) C.rbcr.resize(L + 1);
    for (int lev = 1; lev <= L; ++lev) {
        C.rb[lev] = level_rbgs(c, pc, qc, lev, C.goff, H, tu);
        C.rbr[lev] = level_rbgs_restrict(c, pc, qc, lev, C.goff, H, tu);
        C.rbc[lev] = C.rb[lev];
        for (int g = 0; g < C.rbc[lev].ngrids; ++g) {
            KGrid& G = C.rbc[lev].g[g];
            G.aoff_x = G.p > 0 ? C.goff[(G.p - 1) * (qc + 1) + G.q] : -1;
            G.aoff_y = G.q > 0 ? C.goff[G.p * (qc + 1) + G.q - 1] : -1;
        }
        C.pro[lev] = level_1d(c, pc, qc, lev, C.goff, 1, qc, -1);
        C.res[lev] = level_1d(c, pc, qc, lev - 1, C.goff, 2, qc, -1);
        if (g_fuse == 2) C.rbcr[lev] = level_rbgs_restrict(c, pc, qc, lev, C.goff, 2 * H, tu2);
    }
    return C;
}

std::vector<StagePlan> make_plans(const BatchLayout& BL, const msg_solve_opts& o)
{
    const Tuning tu = tuning_of(o);
    std::vector<StagePlan> plans(BL.maxL + 1);
    const int c = BL.c;
    for (int L = 0; L <= BL.maxL; ++L) {
        StagePlan& SP = plans[L];
        SP.L = L;
        for (int pc = 0; pc <= L; ++pc) {
            const int qc = L - pc;
            if (pc > kMaxIndex || qc > kMaxIndex) continue;
            std::vector<int> samples;
            for (int s = 0; s < BL.S; ++s)
                if (BL.P[s] >= pc && BL.Q[s] >= qc) samples.push_back(s);
            if (samples.empty()) continue;
            ClassPlan C = plan_class(c, pc, qc, std::move(samples), o, tu, false);
            C.first = SP.K;
            C.arena = SP.arena_cells;
            SP.K += C.K;
            SP.arena_cells += C.stride * C.K;
            C.part0 = SP.part_slots;
            SP.part_slots += (int64_t)C.top1d.ntiles * C.K;
            if (!C.solve_in_tail && C.tail_lds > 0) {
                C.tpack = SP.tpack_elems;
                SP.tpack_elems += (int64_t)C.tail.nstat * C.K;
            }
            SP.slot_entries += C.tail.nslots + C.tail64.nslots;
            C.ci = (int)SP.classes.size();
            SP.classes.push_back(std::move(C));
        }
    }
    return plans;
}

// ---------------------------------------------------------------- workspace
struct Ws {
    size_t gcls;
    size_t bpyr, chol, a64v, a64v2, a64b, a32v, a32v2, a32b, part, active, pcycles, dead, nactive, sbase, gbase, rbase, probs,
        pyrprobs, tails, cls, tpack, slots, total;
};

Ws ws_layout(const BatchLayout& BL, const std::vector<StagePlan>& plans, bool mixed)
{
    int64_t arena = 0, parts = 0, probs = 0, tpack = 0, slots = 0;
    for (const StagePlan& SP : plans) {
        tpack = std::max(tpack, SP.tpack_elems);
        slots = std::max(slots, SP.slot_entries);
        arena = std::max(arena, SP.arena_cells);
        parts = std::max(parts, SP.part_slots);
        probs = std::max<int64_t>(probs, SP.K);
    }
    const int n0 = BL.c * BL.c;
    Ws w;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
    w.bpyr = take(sizeof(double) * BL.cell[BL.S]);
    w.chol = take(sizeof(double) * (size_t)BL.S * n0 * n0);
    w.a64v = take(sizeof(double) * arena);
    w.a64v2 = take(sizeof(double) * arena);
    w.a64b = take(sizeof(double) * arena);
    w.a32v = take(mixed ? sizeof(float) * arena : 0);
    w.a32v2 = take(mixed ? sizeof(float) * arena : 0);
    w.a32b = take(mixed ? sizeof(float) * arena : 0);
    w.part = take(sizeof(double) * 2 * std::max<int64_t>(parts, 1));
    w.active = take(sizeof(int32_t) * std::max<int64_t>(probs, 1));
    w.pcycles = take(sizeof(int32_t) * std::max<int64_t>(probs, 1));
    w.dead = take(sizeof(int32_t) * BL.S);
    w.nactive = take(sizeof(int32_t) * (kMaxIndex + 1));
    w.sbase = take(sizeof(SampleBase) * BL.S);
    w.gbase = take(sizeof(int64_t) * BL.S);
    w.rbase = take(sizeof(int64_t) * BL.S);
    w.probs = take(sizeof(KProb) * std::max<int64_t>(probs, 1));
    w.pyrprobs = take(sizeof(KProb) * BL.S);
    w.tails = take(sizeof(KTail) * 2 * (kMaxIndex + 1));
    w.cls = take(sizeof(int32_t) * std::max<int64_t>(probs, 1));
    w.gcls = take(sizeof(int32_t) * kMaxGroups * std::max<int64_t>(probs, 1));
    w.tpack = take((mixed ? sizeof(float) : sizeof(double)) * std::max<int64_t>(tpack, 1));
    w.slots = take(sizeof(int4) * std::max<int64_t>(slots, 1));
    w.total = off;
    return w;
}

std::vector<SampleBase> sample_bases(const BatchLayout& BL)
{
    std::vector<SampleBase> v(BL.S);
    for (int s = 0; s < BL.S; ++s) {
        v[s].fx = BL.xf[s];
        v[s].fy = BL.yf[s];
        v[s].P = BL.P[s];
        v[s].Q = BL.Q[s];
    }
    return v;
}

// launch a per-problem kernel over problems [0, K) in chunks that keep the
// block count below 2^31
template <typename F>
msg_status chunked(const KLevel& L, int K, F&& f)
{
    const int64_t per = std::max<int64_t>(1, ((int64_t)1 << 30) / std::max(1, L.ntiles));
    for (int64_t k0 = 0; k0 < K; k0 += per) {
        const int kn = (int)std::min<int64_t>(per, K - k0);
        hipError_t e = f((int)k0, kn);
        if (e != hipSuccess) return fail(MSG_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    }
    return MSG_OK;
}

}  // namespace

// Per-kernel-kind event timing while profiling is on: a pair of events
// around each timed launch, resolved at the next synchronisation point.
// With every = n > 1 one launch in n is timed, picked by a hash of a running
// launch counter (a fixed stride could alias with the regular pattern of
// launches in a cycle); every launch is counted.  The few long launches
// that solve whole classes are always timed and kept apart from the sampled
// population, which alone is scaled.
struct Profiler {
    bool on = false;
    int every = 1;
    uint64_t draw = 0;
    int64_t seen[MSG_KERNEL_KINDS] = {};
    msg_kernel_stats fixed[MSG_KERNEL_KINDS] = {};
    struct Rec {
        hipEvent_t a, b;
        int kind;
        double bytes;
        double model;      // bytes of the per-step model (msg_kernel_stats.model_bytes)
        int also;          // a second kind the launch counts towards (a subset kind), or -1
        bool always;       // outside the sampled population
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> pending;
    msg_kernel_stats tot[MSG_KERNEL_KINDS] = {};

    hipEvent_t get()
    {
        if (pool.empty()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    // resolve every pending pair (the stream has been synchronised)
    void resolve()
    {
        for (Rec& r : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                for (int k : {r.kind, r.also}) {
                    if (k < 0) continue;
                    msg_kernel_stats& t = r.always ? fixed[k] : tot[k];
                    t.launches += 1;
                    t.milliseconds += ms;
                    t.bytes += r.bytes;
                    t.model_bytes += r.model;
                }
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
    void reset()
    {
        pending.clear();
        for (auto& t : tot) t = msg_kernel_stats{0, 0.0, 0.0, 0.0};
        for (auto& t : fixed) t = msg_kernel_stats{0, 0.0, 0.0, 0.0};
        for (auto& n : seen) n = 0;
        draw = 0;
    }
    // count a launch of `kind` (and `also`); true when it is to be timed
    bool pick(int kind, int also, bool always)
    {
        if (always) return true;
        seen[kind] += 1;
        if (also >= 0) seen[also] += 1;
        if (every <= 1) return true;
        uint64_t z = (draw++) + 0x9E3779B97F4A7C15ull;          // splitmix64 finaliser
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return z % (uint64_t)every == 0;
    }
    ~Profiler()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        for (Rec& r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    }
};


// What one concurrently solved part of a batch owns: its stream, the side
// streams its classes alternate over, their fork/join events, and its
// kernel timing.
struct Lane {
    Profiler prof;
    hipStream_t own = nullptr;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr, join[kSideStreams] = {}, done = nullptr;
    ~Lane()
    {
        for (int k = 0; k < kSideStreams; ++k) {
            if (side[k]) (void)hipStreamDestroy(side[k]);
            if (join[k]) (void)hipEventDestroy(join[k]);
        }
        if (own) (void)hipStreamDestroy(own);
        if (fork) (void)hipEventDestroy(fork);
        if (done) (void)hipEventDestroy(done);
    }
    // default-priority streams and their events, created on first use; the
    // side streams only for solves that use them (an idle stream still takes
    // a share of the device's hardware queues)
    hipError_t streams(bool with_side)
    {
        hipError_t e = hipSuccess;
        if (!fork) {
            e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&own, hipStreamNonBlocking);
        }
        for (int k = 0; with_side && k < g_side && e == hipSuccess; ++k) {
            if (side[k]) continue;
            e = hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&join[k], hipEventDisableTiming);
        }
        return e;
    }
};

constexpr int kMaxParts = 8;       // most concurrent parts a large batch is split into
// parts used (2..kMaxParts, MSG_PARTS); 256x256 x 4096 FP64: 233 samples/s
// with 2, 253 with 3, 210 with 4 while each part also created two idle side
// streams.  With the side streams made only when used: 313 with 3, 260 with
// 4, and with GPU_MAX_HW_QUEUES = 8: 312 with 4, 296 with 6, 302 with 8
// (16 queues); three parts already keep the device busy.
int g_parts = 3;
constexpr int kSplitMin = 1024;    // smallest batch split by the automatic overlap

struct msg_handle_s {
    int device;
    Lane lane[kMaxParts];
};

// Bytes of workspace of a part, and the split of a batch into parts.
namespace {

size_t part_ws_bytes(const msg_batch_desc* batch, const msg_solve_opts* opts)
{
    const BatchLayout BL = make_layout(batch);
    return ws_layout(BL, make_plans(BL, *opts), opts->precision == MSG_MIXED).total;
}

// overlap mode actually used: -1 picks 2 (concurrent parts) for large
// batches and 0 otherwise.  Extra streams pay only while the device has
// hardware queues to spare: with several callers solving concurrently (the
// request loop), class streams made every batch wait on the others (median
// latency 730 ms against 2.8 ms without them, 1000 requests at 400/s).
int overlap_mode(const msg_batch_desc* batch, const msg_solve_opts* opts)
{
    const int m = opts->overlap < 0 ? (batch->n_samples >= kSplitMin ? 2 : 0) : opts->overlap;
    return (m == 2 && batch->n_samples < g_parts) ? 1 : m;
}

struct Split {
    int n;
    msg_batch_desc part[kMaxParts];
    int first[kMaxParts];
    size_t ws_off[kMaxParts], ws_bytes[kMaxParts], total;
};

Split split_batch(const msg_batch_desc* batch, const msg_solve_opts* opts)
{
    Split sp;
    size_t off = 0;
    sp.n = g_parts;
    for (int k = 0; k < sp.n; ++k) {
        const int a = (int)((int64_t)batch->n_samples * k / sp.n);
        const int b = (int)((int64_t)batch->n_samples * (k + 1) / sp.n);
        sp.first[k] = a;
        sp.part[k] = msg_batch_desc{b - a, batch->c, batch->P + a, batch->Q + a};
        sp.ws_off[k] = off;
        sp.ws_bytes[k] = part_ws_bytes(&sp.part[k], opts);
        off = align_up(off + sp.ws_bytes[k]);
    }
    sp.total = off;
    return sp;
}

}  // namespace

namespace {

// Debug switch read at every solve: MSG_DEBUG_SPLIT_SWEEPS=1 runs each
// smoothing pass as its separate steps (correction, copy, one launch per
// colour of every half-sweep) and restricts with k_restrict instead of the
// fused restricting pass, so a test can compare the fused kernels with
// their unfused definition bit for bit.  The on-chip tail is unchanged.
bool split_sweeps()
{
    const char* t = std::getenv("MSG_DEBUG_SPLIT_SWEEPS");
    return t && std::atoi(t) != 0;
}

// tuning overrides from the environment, read once per process (handles may
// be created from several threads; sizes may be asked for before any handle)
void read_env()
{
    static std::once_flag env_once;
    std::call_once(env_once, [] {
        if (const char* f = std::getenv("MSG_RBGS_FUSE")) g_fuse = std::atoi(f) == 1 ? 1 : 2;
        if (const char* t = std::getenv("MSG_TAIL_LDS")) g_tail_lds = std::max(1024, std::atoi(t));
        if (const char* t = std::getenv("MSG_SPLIT_INNER")) g_split_inner = std::atoi(t) > 0 ? 1 : 0;
        if (const char* t = std::getenv("MSG_SOLVE_LDS")) g_solve_lds = std::max(0, std::atoi(t));
        if (const char* t = std::getenv("MSG_DEBUG_STAGES")) g_debug_stages = std::atoi(t) != 0;
        if (const char* t = std::getenv("MSG_HANDOFF")) g_handoff = std::max(0, std::atoi(t));
        if (const char* t = std::getenv("MSG_TAIL_REG")) g_tail_reg_levels = std::max(0, std::min(kTailRegLevels, std::atoi(t)));
        if (const char* t = std::getenv("MSG_SIDE_STREAMS")) g_side = std::max(1, std::min(kSideStreams, std::atoi(t)));
        if (const char* t = std::getenv("MSG_RBGS_TW")) g_rbgs_tw = std::max(4, std::min(256, std::atoi(t)));
        if (const char* t = std::getenv("MSG_RBGS_CELLS")) g_rbgs_cells = std::max(64, std::min(4096, std::atoi(t)));
        if (const char* t = std::getenv("MSG_RBGS_LDS")) g_rbgs_lds = std::max(1024, std::min(kRbgsLdsMax, std::atoi(t)));
        if (const char* t = std::getenv("MSG_PARTS")) g_parts = std::max(2, std::min(kMaxParts, std::atoi(t)));
        if (const char* t = std::getenv("MSG_TAIL_TABLE")) g_tail_table = std::atoi(t) != 0;
        if (const char* t = std::getenv("MSG_FUSE_RESTRICT")) g_fuse_restrict = std::atoi(t) != 0;
        if (const char* t = std::getenv("MSG_FUSE_VISITS")) g_fuse_visits = std::atoi(t) != 0;
        if (const char* t = std::getenv("MSG_CR_TW")) g_cr_tw = std::max(4, std::min(256, std::atoi(t)));
        if (const char* t = std::getenv("MSG_CR_CELLS")) g_cr_cells = std::max(64, std::min(4096, std::atoi(t)));
        if (const char* t = std::getenv("MSG_CR_LDS")) g_cr_lds = std::max(1024, std::min(kRbgsLdsMax, std::atoi(t)));
    });
}

}  // namespace

// ======================================================================
// C-ABI
// ======================================================================
extern "C" {

void msg_default_opts(msg_solve_opts* o)
{
    if (!o) return;
    o->mu = 2;
    o->nu1 = 2;
    o->nu2 = 2;
    o->max_cycles = 50;
    o->tol = 1e-10;
    o->omega = 1.0;
    o->precision = MSG_FP64;
    o->tail_levels = -1;
    o->handoff = -1;
    o->overlap = -1;
    o->tail_budget = 0;
    o->tile_width = 0;
    o->tile_cells = 0;
    o->tile_lds = 0;
    o->graphs = 0;
}

const char* msg_last_error(void) { return g_err.c_str(); }

msg_status msg_create(msg_handle* h, int device)
{
    if (!h) return fail(MSG_ERR_ARG, "handle pointer is NULL");
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(MSG_ERR_ARG, "device %d not present (%d devices)", device, n);
    HIPCHK(hipSetDevice(device));
    read_env();
    // this device's copy of the no-allocation scratch (noalloc.hip)
    msg_status st = msg::noalloc_setup(device);
    if (st != MSG_OK) return st;
    *h = new msg_handle_s{device};
    return MSG_OK;
}

void msg_destroy(msg_handle h) { delete h; }

msg_status msg_layout(const msg_batch_desc* batch, int64_t* cell_off_out, int64_t* xface_off_out,
                      int64_t* yface_off_out, int64_t* grid_off_out)
{
    msg_status st = check_batch(batch);
    if (st != MSG_OK) return st;
    const BatchLayout BL = make_layout(batch);
    for (int s = 0; s <= BL.S; ++s) {
        if (cell_off_out) cell_off_out[s] = BL.cell[s];
        if (xface_off_out) xface_off_out[s] = BL.xf[s];
        if (yface_off_out) yface_off_out[s] = BL.yf[s];
        if (grid_off_out) grid_off_out[s] = BL.grid[s];
    }
    return MSG_OK;
}

msg_status msg_workspace_size(msg_handle, const msg_batch_desc* batch, const msg_solve_opts* opts, size_t* bytes)
{
    msg_status st = check_batch(batch);
    if (st != MSG_OK) return st;
    if ((st = check_opts(opts)) != MSG_OK) return st;
    if (!bytes) return fail(MSG_ERR_ARG, "bytes is NULL");
    read_env();
    *bytes = overlap_mode(batch, opts) == 2 ? split_batch(batch, opts).total : part_ws_bytes(batch, opts);
    return MSG_OK;
}

}  // extern "C"

// msg_sample_field with its device staging (the per-sample tables and, without
// d_xi, the drawn normals) in `staging` of `cap` bytes, or, when staging is
// null, in memory allocated on the stream for the call.
msg_status msg::sample_field_impl(msg_handle h, const msg_field_spec* spec, const msg_batch_desc* batch,
                                  const double* d_xi, double* d_kx, double* d_ky, float* d_kx32, float* d_ky32,
                                  msg_stream stream, void* staging, size_t cap)
{
    if (!h) return fail(MSG_ERR_ARG, "handle is NULL");
    msg_status st = check_batch(batch);
    if (st != MSG_OK) return st;
    if (!spec || !d_kx || !d_ky) return fail(MSG_ERR_ARG, "spec, kx and ky are required");
    if ((d_kx32 == nullptr) != (d_ky32 == nullptr)) return fail(MSG_ERR_ARG, "give both FP32 copies or neither");
    if (spec->face_rule != MSG_FACE_POINT && spec->face_rule != MSG_FACE_MEAN)
        return fail(MSG_ERR_ARG, "unknown face rule %d", spec->face_rule);
    hipStream_t s = (hipStream_t)stream;
    FieldArgs A;
    std::memset(&A, 0, sizeof A);
    A.c = batch->c;
    if (spec->kind == MSG_FIELD_COS_TABLE) {
        if (spec->n_terms < 1 || spec->n_terms > kMaxCosTerms || !spec->a || !spec->b || !spec->amp)
            return fail(MSG_ERR_ARG, "cosine table needs 1..%d terms with a, b, amp", kMaxCosTerms);
        A.kind = 0;
        A.n_terms = spec->n_terms;
        A.cos.n = spec->n_terms;
        int mx = 0, my = 0;
        for (int t = 0; t < spec->n_terms; ++t) {
            if (spec->a[t] < 0 || spec->b[t] < 0 || spec->a[t] >= kMaxModes || spec->b[t] >= kMaxModes)
                return fail(MSG_ERR_ARG, "term %d: frequencies must be in 0..%d", t, kMaxModes - 1);
            if (!std::isfinite(spec->amp[t])) return fail(MSG_ERR_ARG, "term %d: amplitude not finite", t);
            A.cos.a[t] = spec->a[t];
            A.cos.b[t] = spec->b[t];
            A.cos.amp[t] = spec->amp[t];
            mx = std::max(mx, spec->a[t] + 1);
            my = std::max(my, spec->b[t] + 1);
        }
        A.Mx = mx;
        A.My = my;
    } else if (spec->kind == MSG_FIELD_SEPARABLE_SE) {
        if (spec->mx < 1 || spec->my < 1 || spec->mx > kMaxModes || spec->my > kMaxModes)
            return fail(MSG_ERR_ARG, "separable field needs 1..%d modes per direction", kMaxModes);
        if (spec->n_terms != spec->mx * spec->my) return fail(MSG_ERR_ARG, "n_terms must equal mx*my");
        if (!(spec->sigma2 >= 0.0) || !(spec->lx > 0.0) || !(spec->ly > 0.0))
            return fail(MSG_ERR_ARG, "need sigma2 >= 0 and positive correlation lengths");
        A.kind = 1;
        A.n_terms = spec->n_terms;
        A.Mx = spec->mx;
        A.My = spec->my;
        A.sigma = std::sqrt(spec->sigma2);
        // per-direction eigenvalues exp(-pi^2 l^2 k^2 / 2), normalised to sum one
        auto eig = [](int m, double l, double* lam) {
            double sum = 0.0;
            for (int k = 0; k < m; ++k) sum += (lam[k] = std::exp(-M_PI * M_PI * l * l * k * k / 2.0));
            for (int k = 0; k < m; ++k) lam[k] /= sum;
        };
        eig(spec->mx, spec->lx, A.lamx);
        eig(spec->my, spec->ly, A.lamy);
    } else {
        return fail(MSG_ERR_ARG, "unknown field kind %d", spec->kind);
    }
    const BatchLayout BL = make_layout(batch);
    const std::vector<SampleBase> bases = sample_bases(BL);
    const bool mean = spec->face_rule == MSG_FACE_MEAN;
    // samples grouped by grid index: one launch per (grid, face kind).  The
    // synthesis covers every grid (MSG_FACE_POINT) or each sample's finest
    // grid only (MSG_FACE_MEAN), whose coarser grids then take face means.
    std::map<std::pair<int, int>, std::vector<int32_t>> bygrid, coarse;
    for (int s = 0; s < BL.S; ++s)
        for (int p = 0; p <= BL.P[s]; ++p)
            for (int q = 0; q <= BL.Q[s]; ++q) {
                if (!mean || (p == BL.P[s] && q == BL.Q[s])) bygrid[{p, q}].push_back(s);
                if (mean && !(p == BL.P[s] && q == BL.Q[s])) coarse[{p, q}].push_back(s);
            }
    size_t nlist = 0;
    for (auto& kv : bygrid) nlist += kv.second.size();
    for (auto& kv : coarse) nlist += kv.second.size();
    std::vector<int64_t> ids;
    if (!d_xi) {
        ids.resize(BL.S);
        for (int k = 0; k < BL.S; ++k) ids[k] = spec->sample_id ? spec->sample_id[k] : k;
    }
    HIPCHK(hipSetDevice(h->device));
    void* dmem = nullptr;
    const size_t o_lists = align_up(sizeof(SampleBase) * BL.S);
    const size_t o_ids = o_lists + align_up(sizeof(int32_t) * nlist);
    const size_t o_xi = o_ids + align_up(sizeof(int64_t) * ids.size());
    const size_t bytes = o_xi + (d_xi ? 0 : sizeof(double) * (size_t)BL.S * A.n_terms);
    if (staging) {
        if (bytes > cap)
            return fail(MSG_ERR_WORKSPACE,
                        "the batch needs %zu bytes of device staging, the no-allocation scratch holds %zu; "
                        "pass d_xi or split the batch", bytes, cap);
        dmem = staging;
    } else {
        HIPCHK(hipMallocAsync(&dmem, bytes, s));
    }
    SampleBase* d_bases = (SampleBase*)dmem;
    int32_t* d_lists = (int32_t*)((char*)dmem + o_lists);
    std::vector<int32_t> lists;
    lists.reserve(nlist);
    for (auto& kv : bygrid) lists.insert(lists.end(), kv.second.begin(), kv.second.end());
    for (auto& kv : coarse) lists.insert(lists.end(), kv.second.begin(), kv.second.end());
    HIPCHK(hipMemcpyAsync(d_bases, bases.data(), sizeof(SampleBase) * BL.S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_lists, lists.data(), sizeof(int32_t) * nlist, hipMemcpyHostToDevice, s));
    const double* xi = d_xi;
    if (!d_xi) {
        int64_t* d_ids = (int64_t*)((char*)dmem + o_ids);
        double* d_draw = (double*)((char*)dmem + o_xi);
        HIPCHK(hipMemcpyAsync(d_ids, ids.data(), sizeof(int64_t) * BL.S, hipMemcpyHostToDevice, s));
        hipError_t e = launch_kl_xi(BL.S, A.n_terms, spec->seed, d_ids, d_draw, s);
        if (e != hipSuccess) return fail(MSG_ERR_HIP, "normals launch: %s", hipGetErrorString(e));
        xi = d_draw;
    }
    size_t at = 0;
    for (auto& kv : bygrid) {
        A.p = kv.first.first;
        A.q = kv.first.second;
        A.nx = batch->c << A.p;
        A.ny = batch->c << A.q;
        const int n = (int)kv.second.size();
        for (int kind = 0; kind < 2; ++kind) {
            A.kind_faces = kind;
            for (int s0 = 0; s0 < n; s0 += 65535) {
                hipError_t e = launch_field(A, std::min(65535, n - s0), d_lists + at + s0, d_bases, xi, d_kx, d_ky,
                                            d_kx32, d_ky32, s);
                if (e != hipSuccess) return fail(MSG_ERR_HIP, "field launch: %s", hipGetErrorString(e));
            }
        }
        at += n;
    }
    for (auto& kv : coarse) {
        const int n = (int)kv.second.size();
        for (int kind = 0; kind < 2; ++kind)
            for (int s0 = 0; s0 < n; s0 += 65535) {
                hipError_t e = launch_face_mean(batch->c, kv.first.first, kv.first.second, kind, std::min(65535, n - s0),
                                                d_lists + at + s0, d_bases, d_kx, d_ky, d_kx32, d_ky32, s);
                if (e != hipSuccess) return fail(MSG_ERR_HIP, "face mean launch: %s", hipGetErrorString(e));
            }
        at += n;
    }
    if (!staging) HIPCHK(hipFreeAsync(dmem, s));
    HIPCHK(hipStreamSynchronize(s));   // the host staging vectors die with this call
    return MSG_OK;
}

int msg::handle_device(msg_handle h) { return h->device; }

msg_status msg::report(msg_status st, const char* text) { return fail(st, "%s", text); }

extern "C" {

msg_status msg_sample_field(msg_handle h, const msg_field_spec* spec, const msg_batch_desc* batch,
                            const double* d_xi, double* d_kx, double* d_ky, float* d_kx32, float* d_ky32,
                            msg_stream stream)
{
    return msg::sample_field_impl(h, spec, batch, d_xi, d_kx, d_ky, d_kx32, d_ky32, stream, nullptr, 0);
}

static_assert(MSG_QOI_MEAN == QOI_MEAN && MSG_QOI_POINT == QOI_POINT && MSG_QOI_SUBDOMAIN == QOI_SUBDOMAIN &&
                  MSG_QOI_FLUX == QOI_FLUX,
              "quantity kinds of the C-ABI and the kernels agree");

msg_status msg_quantity(const msg_batch_desc* batch, int kind, const double* d_kx, const double* d_u, double* d_q,
                        msg_stream stream)
{
    msg_status st = check_batch(batch);
    if (st != MSG_OK) return st;
    if (kind < MSG_QOI_MEAN || kind > MSG_QOI_FLUX) return fail(MSG_ERR_ARG, "unknown quantity kind %d", kind);
    if (!d_u || !d_q) return fail(MSG_ERR_ARG, "u and q are required");
    if (kind == MSG_QOI_FLUX && !d_kx) return fail(MSG_ERR_ARG, "the flux needs kx");
    hipStream_t s = (hipStream_t)stream;
    const BatchLayout BL = make_layout(batch);
    std::vector<int32_t> pq(2 * BL.S);
    int maxg = 1;
    for (int k = 0; k < BL.S; ++k) {
        pq[2 * k] = BL.P[k];
        pq[2 * k + 1] = BL.Q[k];
        maxg = std::max(maxg, (BL.P[k] + 1) * (BL.Q[k] + 1));
    }
    void* dmem = nullptr;
    const size_t a = align_up(sizeof(int32_t) * 2 * BL.S), b = align_up(sizeof(int64_t) * BL.S);
    HIPCHK(hipMallocAsync(&dmem, a + 3 * b, s));
    char* m = (char*)dmem;
    HIPCHK(hipMemcpyAsync(m, pq.data(), sizeof(int32_t) * 2 * BL.S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(m + a, BL.cell.data(), sizeof(int64_t) * BL.S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(m + a + b, BL.xf.data(), sizeof(int64_t) * BL.S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(m + a + 2 * b, BL.grid.data(), sizeof(int64_t) * BL.S, hipMemcpyHostToDevice, s));
    for (int s0 = 0; s0 < BL.S; s0 += 65535) {
        const int n = std::min(65535, BL.S - s0);
        hipError_t e = launch_qoi(n, maxg, kind, BL.c, (int32_t*)m + 2 * s0, (int64_t*)(m + a) + s0,
                                  (int64_t*)(m + a + b) + s0, (int64_t*)(m + a + 2 * b) + s0, d_kx, d_u, d_q, s);
        if (e != hipSuccess) return fail(MSG_ERR_HIP, "quantity launch: %s", hipGetErrorString(e));
    }
    HIPCHK(hipFreeAsync(dmem, s));
    HIPCHK(hipStreamSynchronize(s));   // the host staging vectors die with this call
    return MSG_OK;
}

msg_status mimc_delta_q(const msg_batch_desc* batch, const double* d_q, double* d_dq, msg_stream stream)
{
    msg_status st = check_batch(batch);
    if (st != MSG_OK) return st;
    if (!d_q || !d_dq) return fail(MSG_ERR_ARG, "q and dq are required");
    hipStream_t s = (hipStream_t)stream;
    const BatchLayout BL = make_layout(batch);
    std::vector<int32_t> pq(2 * BL.S);
    int maxg = 1;
    for (int k = 0; k < BL.S; ++k) {
        pq[2 * k] = BL.P[k];
        pq[2 * k + 1] = BL.Q[k];
        maxg = std::max(maxg, (BL.P[k] + 1) * (BL.Q[k] + 1));
    }
    void* dmem = nullptr;
    const size_t a = align_up(sizeof(int32_t) * 2 * BL.S);
    HIPCHK(hipMallocAsync(&dmem, a + sizeof(int64_t) * BL.S, s));
    HIPCHK(hipMemcpyAsync(dmem, pq.data(), sizeof(int32_t) * 2 * BL.S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync((char*)dmem + a, BL.grid.data(), sizeof(int64_t) * BL.S, hipMemcpyHostToDevice, s));
    for (int s0 = 0; s0 < BL.S; s0 += 65535) {
        const int n = std::min(65535, BL.S - s0);
        hipError_t e = launch_delta_q(n, maxg, (int32_t*)dmem + 2 * s0, (int64_t*)((char*)dmem + a) + s0, d_q, d_dq, s);
        if (e != hipSuccess) return fail(MSG_ERR_HIP, "delta_q launch: %s", hipGetErrorString(e));
    }
    HIPCHK(hipFreeAsync(dmem, s));
    HIPCHK(hipStreamSynchronize(s));
    return MSG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- the solve
namespace {

struct Ctx {
    const BatchLayout* BL;
    const msg_solve_opts* o;
    hipStream_t s;
    int c;
    const double* chol;
    KProb* probs;       // device, current stage
    int32_t* active;
    Profiler* prof;
    int64_t kact;       // problems of the current class still cycling
    const KTail* tails; // device: per class of the level, [2 ci] cycle tail, [2 ci + 1] whole-class tail
    void* tpack;        // device: tail conductance images of the stage (type of the cycles)
    bool split = false; // debug: smoothing passes as one launch per colour, no fused transfers
};

// algorithmic bytes: data a kernel must touch at least once per active problem
template <typename T>
double level_bytes(const KLevel& L, int kind_rel /*0 smooth, 1 restrict, 2 prolong, 3 correction children, 4 copy,
                                                   5 restricted outputs of a pass, 6 combination*/,
                   int64_t K)
{
    double per = 0.0;
    for (int g = 0; g < L.ngrids; ++g) {
        const KGrid& G = L.g[g];
        const double cells = (double)G.nx * G.ny;
        const double faces = (double)(G.nx + 1) * G.ny + (double)G.nx * (G.ny + 1);
        if (kind_rel == 0) {
            per += 3 * cells + faces;                         // v, b, kx, ky read; v written
        } else if (kind_rel == 1) {
            per += 2 * cells;                                 // coarse b and v written
            if (G.aoff_x >= 0) per += 2 * (2 * cells) + ((2 * G.nx + 1.0) * G.ny + 2.0 * G.nx * (G.ny + 1));
            if (G.aoff_y >= 0) per += 2 * (2 * cells) + ((G.nx + 1.0) * 2 * G.ny + G.nx * (2.0 * G.ny + 1));
        } else if (kind_rel == 2) {
            per += 2 * cells + faces;                         // fine v read and written, faces read
            if (G.aoff_x >= 0) per += cells / 2;
            if (G.aoff_y >= 0) per += cells / 2;
        } else if (kind_rel == 3) {
            if (G.aoff_x >= 0) per += cells / 2;              // coarse iterates of the children
            if (G.aoff_y >= 0) per += cells / 2;
        } else if (kind_rel == 5) {
            if (G.aoff_x >= 0) per += cells / 2;              // restricted residual into each child
            if (G.aoff_y >= 0) per += cells / 2;
        } else if (kind_rel == 6) {
            if (G.aoff_x >= 0 && G.aoff_y >= 0) per += 4 * cells;   // two halves combined, iterate zeroed
        } else {
            per += 2 * cells;                                 // iterate read and written
        }
    }
    return per * sizeof(T) * (double)K;
}

// bytes of the per-step model on a level: `values` values of type T per cell
// (5 per red-black sweep, 5 for a residual with its restriction or for a
// correction, 2 for a copy)
template <typename T>
double model_bytes(const KLevel& L, double values, int64_t K)
{
    double cells = 0.0;
    for (int g = 0; g < L.ngrids; ++g) cells += (double)L.g[g].nx * L.g[g].ny;
    return cells * values * sizeof(T) * (double)K;
}

// model < 0: the per-step model's bytes equal the algorithmic bytes
template <typename F>
msg_status timed(const Ctx& X, int kind, double bytes, F&& f, int also = -1, bool always = false, double model = -1.0)
{
    Profiler* P = X.prof;
    if (!P || !P->on || !P->pick(kind, also, always)) return f();
    Profiler::Rec r{P->get(), P->get(), kind, bytes, model < 0.0 ? bytes : model, also, always};
    if (!r.a || !r.b) return fail(MSG_ERR_HIP, "event creation failed");
    HIPCHK(hipEventRecord(r.a, X.s));
    msg_status st = f();
    HIPCHK(hipEventRecord(r.b, X.s));
    P->pending.push_back(r);
    return st;
}

// The iterates of a class live in two buffers: the smoother reads one and
// writes the other.  cur[l] says which buffer holds the current iterate of
// the grids on level l (all grids of a level of a class move together).
template <typename T>
struct Iter {
    T* v[2];
    int cur[2 * kMaxIndex + 2];
    T* now(int l) const { return v[cur[l]]; }
};

// the state a W-cycle on level L depends on: the buffers and which holds
// level L (every coarser level's is set by the restriction before use)
template <typename T>
bool same_start(const Iter<T>& a, const Iter<T>& b, int L)
{
    return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.cur[L] == b.cur[L];
}

// A class's captured W-cycle and the buffer states before and after it.
struct ClassGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Iter<double> before64{}, after64{};
    Iter<float> before32{}, after32{};
    ClassGraph() = default;
    ClassGraph(const ClassGraph&) = delete;
    ClassGraph& operator=(const ClassGraph&) = delete;
    ClassGraph(ClassGraph&& o) noexcept { *this = std::move(o); }
    ClassGraph& operator=(ClassGraph&& o) noexcept
    {
        std::swap(graph, o.graph);
        std::swap(exec, o.exec);
        before64 = o.before64; after64 = o.after64; before32 = o.before32; after32 = o.after32;
        return *this;
    }
    ~ClassGraph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Algorithm MSG mu-cycle on level lev of class C, recursion on the host down
// to the tail level, whose cycles run inside one workgroup per problem.
// problems [k0, k0 + kn) of a class
struct Span {
    int k0, kn;
};



// One class of a lockstep group: its plan, the problems [k0, k0 + kn) of the
// class it cycles, and how many of them still cycle (byte counts).
struct Member {
    const ClassPlan* C;
    Span sp;
    int64_t kact;
};

// Classes of one F-cycle stage that share the tail level and the tail's
// workgroup size issue the same sequence of passes in their W-cycles, so
// they recurse in lockstep: each pass is launched per class, but every visit
// of the on-chip tail is one launch for all of them (block b is stage problem
// gfirst + b, with its class's tail descriptor from the table gcls), so that
// the latency-bound tails of the classes run side by side on the chip.  The
// buffer states of their iterates move together (one Iter for the group).
// gcls null: a single class, launched as before.
struct Group {
    std::vector<Member> m;
    int tail_top = 0, tail_threads = 64;
    size_t tail_lds = 0;
    const int32_t* gcls = nullptr;
    int gfirst = 0, gend = 0;
};

Group single_group(const ClassPlan& C, const Span& sp, int64_t kact)
{
    Group G;
    G.m.push_back(Member{&C, sp, kact});
    G.tail_top = C.tail_top;
    G.tail_threads = C.tail_threads;
    G.tail_lds = C.tail_lds;
    return G;
}

// Flags of one W-cycle visit of a level (mu_cycle below).  In a W-cycle the
// post-smoothing pass of one visit of a level and the pre-smoothing pass of
// the next visit follow each other with nothing in between (the parent level
// calls its coarse cycle mu times in a row); such a pair runs as one pass.
constexpr int kLeavePost = 1;   // end without the correction and post-smoothing (the next visit applies them)
constexpr int kFusedPre = 2;    // start with the previous visit's correction and post-smoothing, fused
                                // with this visit's pre-smoothing and restriction

template <typename T>
msg_status mu_cycle(const Ctx& X, const Group& G, int lev, Iter<T>& it, T* B, const T* KX, const T* KY,
                    int flags = 0)
{
    msg_status st;
    const int M = G.tail_top, Lstage = G.m[0].C->L;
    auto tail = [&](int count, int combine) -> msg_status {
        T* V = it.now(M);
        double bytes = 0.0;
        for (const Member& e : G.m) bytes += tail_bytes(e.C->tail, sizeof(T)) * (double)e.kact;
        if (!G.gcls) {
            const Member& e = G.m[0];
            const ClassPlan& C = *e.C;
            const T* pack = C.tpack >= 0 ? (const T*)X.tpack : nullptr;
            return timed(X, MSG_KERNEL_TAIL, bytes, [&] {
                return chunked(C.top1d, e.sp.kn, [&](int k0, int kn) {
                    const int kb = C.first + e.sp.k0 + k0;
                    return launch_tail<T>(X.tails, nullptr, 2 * C.ci, kb, C.tail_threads, C.tail_lds, kn,
                                          X.probs + kb, X.active + kb, X.c, X.o->mu, X.o->nu1, X.o->nu2,
                                          (T)X.o->omega, count, combine, V, B, KX, KY, pack, X.chol, TailSolve{},
                                          X.s);
                });
            });
        }
        return timed(X, MSG_KERNEL_TAIL, bytes, [&]() -> msg_status {
            hipError_t e = launch_tail<T>(X.tails, G.gcls + G.gfirst, 0, G.gfirst, G.tail_threads, G.tail_lds,
                                          G.gend - G.gfirst, X.probs + G.gfirst, X.active + G.gfirst, X.c, X.o->mu,
                                          X.o->nu1, X.o->nu2, (T)X.o->omega, count, combine, V, B, KX, KY,
                                          (const T*)X.tpack, X.chol, TailSolve{}, X.s);
            if (e != hipSuccess) return fail(MSG_ERR_HIP, "tail launch: %s", hipGetErrorString(e));
            return MSG_OK;
        });
    };
    if (lev <= M) return tail(1, 0);
    // sweeps red-black sweeps on level lev, two fused per pass; with `corr`
    // the first pass also applies the coarse-grid correction (eq. interpolation).
    // ns = 0 is a copy pass (no sweep).
    int flips = 0;
    int combine_in_tail = 0;        // the restriction into the tail's top level left two halves to average
    // split-sweep debug mode: the correction (k_prolong) on the input
    // buffer, a copy into the output buffer, then each half-sweep as one
    // in-place launch per colour over whole grids
    auto split_pass = [&](int ns, bool corr) -> msg_status {
        T* vin = it.v[it.cur[lev]];
        T* vout = it.v[1 - it.cur[lev]];
        const T* vc = corr ? it.now(lev - 1) : nullptr;
        for (const Member& e : G.m) {
            const ClassPlan& C = *e.C;
            const KLevel& P1 = C.pro[lev];
            const KProb* pr = X.probs + C.first + e.sp.k0;
            const int32_t* act = X.active + C.first + e.sp.k0;
            msg_status r = timed(X, MSG_KERNEL_SMOOTH, level_bytes<T>(P1, 0, e.kact) * ns, [&] {
                return chunked(P1, e.sp.kn, [&](int k0, int kn) -> hipError_t {
                    hipError_t h = hipSuccess;
                    if (corr)
                        h = launch_prolong<T>(P1, kn, pr + k0, act + k0, X.c, (T)X.o->omega, vc, vin, KX, KY, X.s);
                    if (h == hipSuccess)
                        h = launch_rbgs<T>(0, C.rb[lev], kn, pr + k0, act + k0, X.c, vin, vout, B, KX, KY, nullptr,
                                           (T)X.o->omega, X.s);
                    for (int sw = 0; sw < 2 * ns && h == hipSuccess; ++sw)
                        h = launch_rb_colour<T>(P1, kn, pr + k0, act + k0, X.c, sw & 1, vout, B, KX, KY, X.s);
                    return h;
                });
            });
            if (r != MSG_OK) return r;
        }
        it.cur[lev] ^= 1;
        ++flips;
        return MSG_OK;
    };
    auto pass = [&](int ns, bool corr) -> msg_status {
        if (X.split && ns > 0) return split_pass(ns, corr);
        const T* vin = it.now(lev);
        T* vout = it.v[1 - it.cur[lev]];
        const T* vc = corr ? it.now(lev - 1) : nullptr;
        for (const Member& e : G.m) {
            const ClassPlan& C = *e.C;
            const KLevel& L = corr ? C.rbc[lev] : C.rb[lev];
            const KProb* pr = X.probs + C.first + e.sp.k0;
            const int32_t* act = X.active + C.first + e.sp.k0;
            // smoother bytes (a copy: read and write the iterate), plus the coarse
            // iterates the correction reads
            const double bytes = ns == 0 ? level_bytes<T>(L, 4, e.kact)
                                         : level_bytes<T>(L, 0, e.kact) + (corr ? level_bytes<T>(L, 3, e.kact) : 0.0);
            const double model = model_bytes<T>(L, ns == 0 ? 2.0 : 5.0 * ns + (corr ? 5.0 : 0.0), e.kact);
            msg_status r = timed(
                X, MSG_KERNEL_SMOOTH, bytes,
                [&] {
                    return chunked(L, e.sp.kn, [&](int k0, int kn) {
                        return launch_rbgs<T>(ns, L, kn, pr + k0, act + k0, X.c, vin, vout, B, KX, KY, vc,
                                              (T)X.o->omega, X.s);
                    });
                },
                lev == Lstage ? MSG_KERNEL_SMOOTH_STAGE : -1, false, model);
            if (r != MSG_OK) return r;
        }
        it.cur[lev] ^= 1;
        ++flips;
        return MSG_OK;
    };
    auto smooth = [&](int sweeps, bool corr) -> msg_status {
        while (sweeps > 0) {
            // tiles are planned for the configured fusion; one sweep fits the same tile
            const int ns = (sweeps >= 2 && g_fuse == 2) ? 2 : 1;
            msg_status r = pass(ns, corr);
            if (r != MSG_OK) return r;
            sweeps -= ns;
            corr = false;
        }
        return MSG_OK;
    };
    const bool fused_pre = (flags & kFusedPre) != 0;
    if (g_fuse_restrict && g_fuse == 2 && X.o->nu1 == 2 && !X.split) {
        // pre-smoothing and the restriction of its residual in one pass, then
        // the coarse grids with two parents combine their halves.  Fused with
        // the previous visit's correction and post-smoothing, the restricted
        // values go to the coarse buffer that does not hold the correction
        // being read (other tiles of the same launch still read it).
        const int tb = fused_pre ? 1 - it.cur[lev - 1] : 0;
        {
            const T* vin = it.now(lev);
            T* vout = it.v[1 - it.cur[lev]];
            T* vco = it.v[tb];
            const T* ve = fused_pre ? it.now(lev - 1) : nullptr;
            for (const Member& e : G.m) {
                const ClassPlan& C = *e.C;
                const KLevel& L = fused_pre ? C.rbcr[lev] : C.rbr[lev];
                const KProb* pr = X.probs + C.first + e.sp.k0;
                const int32_t* act = X.active + C.first + e.sp.k0;
                const double bytes = level_bytes<T>(L, 0, e.kact) + level_bytes<T>(L, 5, e.kact) +
                                     (fused_pre ? level_bytes<T>(L, 3, e.kact) : 0.0);
                st = timed(
                    X, MSG_KERNEL_SMOOTH, bytes,
                    [&] {
                        return chunked(L, e.sp.kn, [&](int k0, int kn) {
                            if (fused_pre)
                                return launch_rbgs_corr_restrict<T>(L, kn, pr + k0, act + k0, X.c, vin, vout, B, KX,
                                                                    KY, ve, (T)X.o->omega, vco, X.s);
                            return launch_rbgs_restrict<T>(L, kn, pr + k0, act + k0, X.c, vin, vout, B, KX, KY, vco,
                                                           X.s);
                        });
                    },
                    lev == Lstage ? MSG_KERNEL_SMOOTH_STAGE : -1, false,
                    model_bytes<T>(L, fused_pre ? 30.0 : 15.0, e.kact));
                if (st != MSG_OK) return st;
            }
            it.cur[lev] ^= 1;
            ++flips;
        }
        // into the tail's top level, the tail's load averages the two
        // halves instead
        if (lev - 1 <= M) {
            combine_in_tail = 1;
            it.cur[lev - 1] = tb;
        } else {
            T* vc = it.v[tb];
            for (const Member& e : G.m) {
                const ClassPlan& C = *e.C;
                const KLevel& R = C.res[lev];
                const KProb* pr = X.probs + C.first + e.sp.k0;
                const int32_t* act = X.active + C.first + e.sp.k0;
                st = timed(
                    X, MSG_KERNEL_RESTRICT, level_bytes<T>(R, 6, e.kact),
                    [&] {
                        return chunked(R, e.sp.kn, [&](int k0, int kn) {
                            return launch_restrict_combine<T>(R, kn, pr + k0, act + k0, vc, B, X.s);
                        });
                    },
                    lev == Lstage ? MSG_KERNEL_RESTRICT_STAGE : -1);
                if (st != MSG_OK) return st;
            }
            it.cur[lev - 1] = tb;
        }
    } else {
        if ((st = smooth(X.o->nu1, false)) != MSG_OK) return st;
        const T* vf = it.now(lev);
        T* vc = it.v[0];
        for (const Member& e : G.m) {
            const ClassPlan& C = *e.C;
            const KLevel& L = C.res[lev];
            const KProb* pr = X.probs + C.first + e.sp.k0;
            const int32_t* act = X.active + C.first + e.sp.k0;
            st = timed(
                X, MSG_KERNEL_RESTRICT, level_bytes<T>(L, 1, e.kact),
                [&] {
                    return chunked(L, e.sp.kn, [&](int k0, int kn) {
                        return launch_restrict<T>(false, L, kn, pr + k0, act + k0, X.c, vf, vc, B, KX, KY, X.s);
                    });
                },
                lev == Lstage ? MSG_KERNEL_RESTRICT_STAGE : -1);
            if (st != MSG_OK) return st;
        }
        it.cur[lev - 1] = 0;
    }
    if (lev - 1 <= M) {
        if ((st = tail(X.o->mu, combine_in_tail)) != MSG_OK) return st;
    } else {
        // consecutive visits of level lev-1 share their boundary pass when
        // it is a two-sweep post-smoothing followed by a two-sweep restricting
        // pre-smoothing and every member planned the fused tiles
        bool pair = g_fuse_visits && g_fuse_restrict && g_fuse == 2 && X.o->nu1 == 2 && X.o->nu2 == 2 && !X.split;
        for (const Member& e : G.m)
            pair = pair && (int)e.C->rbcr.size() > lev - 1 && e.C->rbcr[lev - 1].ngrids > 0;
        for (int m = 0; m < X.o->mu; ++m) {
            const int f = pair ? ((m > 0 ? kFusedPre : 0) | (m + 1 < X.o->mu ? kLeavePost : 0)) : 0;
            if ((st = mu_cycle<T>(X, G, lev - 1, it, B, KX, KY, f)) != MSG_OK) return st;
        }
    }
    if (flags & kLeavePost) return MSG_OK;         // the next visit applies them, fused
    if (X.o->nu2 > 0) {
        if ((st = smooth(X.o->nu2, true)) != MSG_OK) return st;      // correction fused into the first pass
    } else {
        const T* vc = it.now(lev - 1);
        T* vf = it.now(lev);
        for (const Member& e : G.m) {
            const ClassPlan& C = *e.C;
            const KLevel& L = C.pro[lev];
            const KProb* pr = X.probs + C.first + e.sp.k0;
            const int32_t* act = X.active + C.first + e.sp.k0;
            st = timed(X, MSG_KERNEL_PROLONG, level_bytes<T>(L, 2, e.kact), [&] {
                return chunked(L, e.sp.kn, [&](int k0, int kn) {
                    return launch_prolong<T>(L, kn, pr + k0, act + k0, X.c, (T)X.o->omega, vc, vf, KX, KY, X.s);
                });
            });
            if (st != MSG_OK) return st;
        }
    }
    // The stage's own level keeps its iterate across cycles, and problems that
    // have stopped are skipped by every pass: an odd number of buffer swaps
    // per cycle would leave theirs behind, so a copy pass evens it out.
    if (lev == Lstage && (flips & 1)) return pass(0, false);
    return MSG_OK;
}

}  // namespace

namespace {

// One part of a batch (the whole batch, or one of the parts solved
// concurrently) on stream s with lane ln; ov > 0 lets the classes of a level
// alternate over the lane's side streams.  Arguments are validated by
// the caller; the part's arrays start at its first sample.
msg_status solve_part(msg_handle h, Lane& ln, int ov, const msg_batch_desc* batch, const msg_solve_opts* opts,
                      const double* d_kx, const double* d_ky, const float* d_kx32, const float* d_ky32,
                      const double* d_rhs, double* d_u_out, double* d_q_out, int32_t* d_status, int32_t* d_cycles,
                      void* d_ws, size_t ws_bytes, hipStream_t s)
{
    msg_status st = MSG_OK;
    const bool mixed = opts->precision == MSG_MIXED;
    const BatchLayout BL = make_layout(batch);
    const std::vector<StagePlan> plans = make_plans(BL, *opts);
    const Ws W = ws_layout(BL, plans, mixed);
    if (ws_bytes < W.total) return fail(MSG_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, W.total);
    if ((uintptr_t)d_ws % kAlign) return fail(MSG_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
    for (const StagePlan& SP : plans)
        for (const ClassPlan& C : SP.classes) {
            if (!C.solve_in_tail && (C.tail_lds == 0 || C.tail_lds > 160 * 1024))
                return fail(MSG_ERR_UNSUPPORTED, "tail of class (%d,%d) does not fit LDS; lower tail_levels", C.pc, C.qc);
            if (C.solve_in_tail && C.tail64_lds > 160 * 1024)
                return fail(MSG_ERR_UNSUPPORTED, "class (%d,%d) does not fit LDS; lower tail_levels", C.pc, C.qc);
        }
    HIPCHK(hipSetDevice(h->device));
    if (ov > 0 || opts->graphs > 0) HIPCHK(ln.streams(true));
    char* ws = (char*)d_ws;
    const int c = BL.c, S = BL.S;

    // host tables, alive until the final synchronisation
    const std::vector<SampleBase> bases = sample_bases(BL);
    std::vector<int64_t> gbase(BL.grid.begin(), BL.grid.begin() + S), rbase(BL.top.begin(), BL.top.begin() + S);
    HIPCHK(hipMemcpyAsync(ws + W.sbase, bases.data(), sizeof(SampleBase) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws + W.gbase, gbase.data(), sizeof(int64_t) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws + W.rbase, rbase.data(), sizeof(int64_t) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(d_status, 0, sizeof(int32_t) * S, s));
    HIPCHK(hipMemsetAsync(ws + W.dead, 0x7f, sizeof(int32_t) * S, s));

    double* bpyr = (double*)(ws + W.bpyr);
    double* chol = (double*)(ws + W.chol);
    SampleBase* d_bases = (SampleBase*)(ws + W.sbase);
    int32_t* dead = (int32_t*)(ws + W.dead);
    int32_t* nact = (int32_t*)(ws + W.nactive);
    double* part = (double*)(ws + W.part);

    // coarsest-grid inverses, one per sample (from the Cholesky factor)
    {
        hipError_t e = launch_chol(S, c, d_bases, d_kx, d_ky, chol, s);
        if (e != hipSuccess) return fail(MSG_ERR_HIP, "cholesky launch: %s", hipGetErrorString(e));
    }

    // right-hand side pyramid (Algorithm MSG F-cycle, restriction of b by
    // eq. restriction), per class of samples sharing a rectangle
    std::map<std::pair<int, int>, std::vector<int>> rects;
    for (int k = 0; k < S; ++k) rects[{BL.P[k], BL.Q[k]}].push_back(k);
    std::vector<KProb> pyr;
    pyr.reserve(S);
    for (auto& kv : rects)
        for (int k : kv.second) {
            KProb p;
            std::memset(&p, 0, sizeof p);
            p.sample = k;
            p.Qs = BL.Q[k];
            p.cell_base = BL.cell[k];
            p.fx_base = BL.xf[k];
            p.fy_base = BL.yf[k];
            p.arena_base = BL.cell[k];
            pyr.push_back(p);
        }
    HIPCHK(hipMemcpyAsync(ws + W.pyrprobs, pyr.data(), sizeof(KProb) * S, hipMemcpyHostToDevice, s));
    {
        const KProb* dp = (const KProb*)(ws + W.pyrprobs);
        int first = 0;
        for (auto& kv : rects) {
            const int P = kv.first.first, Q = kv.first.second, K = (int)kv.second.size();
            std::vector<int64_t> goff((size_t)(P + 1) * (Q + 1));
            for (int a = 0; a <= P; ++a)
                for (int b = 0; b <= Q; ++b) goff[a * (Q + 1) + b] = cell_off(c, Q, a, b);
            const KLevel top = level_1d(c, P, Q, P + Q, goff, 0, Q);
            st = chunked(top, K, [&](int k0, int kn) {
                return launch_rhs_top(top, kn, dp + first + k0, bpyr, d_rhs, (const int64_t*)(ws + W.rbase), s);
            });
            if (st != MSG_OK) return st;
            for (int lev = P + Q - 1; lev >= 0; --lev) {
                const KLevel L = level_1d(c, P, Q, lev, goff, 2, Q);
                st = chunked(L, K, [&](int k0, int kn) {
                    return launch_restrict<double>(true, L, kn, dp + first + k0, nullptr, c, nullptr, nullptr, bpyr,
                                                   d_kx, d_ky, s);
                });
                if (st != MSG_OK) return st;
            }
            first += K;
        }
    }

    Ctx X;
    X.BL = &BL;
    X.o = opts;
    X.s = s;
    X.c = c;
    X.chol = chol;
    X.prof = &ln.prof;
    X.kact = 0;
    X.split = split_sweeps();
    double* a64b = (double*)(ws + W.a64b);
    float* a32b = mixed ? (float*)(ws + W.a32b) : nullptr;
    Iter<double> it64;
    Iter<float> it32;
    it64.v[0] = (double*)(ws + W.a64v);
    it64.v[1] = (double*)(ws + W.a64v2);
    it32.v[0] = mixed ? (float*)(ws + W.a32v) : nullptr;
    it32.v[1] = mixed ? (float*)(ws + W.a32v2) : nullptr;
    X.probs = (KProb*)(ws + W.probs);
    X.active = (int32_t*)(ws + W.active);
    int32_t* pcycles = (int32_t*)(ws + W.pcycles);

    // host staging of the per-level tables; they live until the stream has
    // consumed them (every level synchronises before the next reuses them)
    std::vector<KProb> probs;
    std::vector<KTail> tails;
    std::vector<int32_t> cls;
    std::vector<std::vector<int32_t>> gcls_host;     // per lockstep group: class descriptor per stage problem
    std::vector<std::vector<int32_t>> gcls_sent;     // what the device holds for each group slot this stage
    X.tails = (const KTail*)(ws + W.tails);
    X.tpack = ws + W.tpack;
    for (const StagePlan& SP : plans) {
        const auto t_stage = std::chrono::steady_clock::now();
        gcls_sent.clear();
        // problems of this F-cycle level (the previous level's table copy has
        // completed: the stream was synchronised at its last convergence check)
        HIPCHK(hipStreamSynchronize(s));
        probs.assign(SP.K, KProb{});
        for (const ClassPlan& C : SP.classes)
            for (int k = 0; k < C.K; ++k) {
                const int smp = C.samples[k];
                KProb& p = probs[C.first + k];
                p.sample = smp;
                p.Qs = BL.Q[smp];
                p.cell_base = BL.cell[smp];
                p.fx_base = BL.xf[smp];
                p.fy_base = BL.yf[smp];
                p.arena_base = C.arena + (int64_t)k * C.stride;
                p.part_base = C.part0 + (int64_t)k * C.top1d.ntiles;
                p.grid_index = C.pc * (BL.Q[smp] + 1) + C.qc;
            }
        HIPCHK(hipMemcpyAsync(X.probs, probs.data(), sizeof(KProb) * SP.K, hipMemcpyHostToDevice, s));
        tails.assign(2 * SP.classes.size(), KTail{});
        {
            int4* d_slots = (int4*)(ws + W.slots);
            int64_t so = 0;
            for (const ClassPlan& C : SP.classes) {
                tails[2 * C.ci] = C.tail;
                tails[2 * C.ci].first = C.first;
                tails[2 * C.ci].pack_off = std::max<int64_t>(C.tpack, 0);
                tails[2 * C.ci + 1] = C.tail64;
                for (int t = 0; t < 2; ++t) {
                    KTail& TL = tails[2 * C.ci + t];
                    if (TL.nslots > 0 && g_tail_table) {
                        TL.slots = d_slots + so;
                        so += TL.nslots;
                    }
                }
            }
        }
        HIPCHK(hipMemcpyAsync(ws + W.tails, tails.data(), sizeof(KTail) * tails.size(), hipMemcpyHostToDevice, s));
        // the red-black slot table of every tail of the stage
        for (size_t t = 0; t < tails.size(); ++t) {
            if (!tails[t].slots) continue;
            hipError_t e = launch_tail_slots(X.tails + t, const_cast<int4*>(tails[t].slots), s);
            if (e != hipSuccess) return fail(MSG_ERR_HIP, "slot table: %s", hipGetErrorString(e));
        }
        {
            hipError_t e = launch_activate(SP.K, X.probs, dead, SP.L, X.active, pcycles, s);
            if (e != hipSuccess) return fail(MSG_ERR_HIP, "activate: %s", hipGetErrorString(e));
        }
        // the conductance images of the tails the host cycles will visit
        for (const ClassPlan& C : SP.classes) {
            if (C.tpack < 0) continue;
            const KTail* tab = X.tails + 2 * C.ci;
            const KProb* pr = X.probs + C.first;
            hipError_t e = mixed ? launch_tail_pack<float>(tab, C.K, pr, c, d_kx32, d_ky32, (float*)X.tpack + C.tpack, s)
                                 : launch_tail_pack<double>(tab, C.K, pr, c, d_kx, d_ky, (double*)X.tpack + C.tpack, s);
            if (e != hipSuccess) return fail(MSG_ERR_HIP, "tail image: %s", hipGetErrorString(e));
        }
        // which buffer holds each level's current iterate, per class
        const int ncls = (int)SP.classes.size();
        std::vector<Iter<double>> i64(ncls, it64);
        std::vector<Iter<float>> i32(ncls, it32);
        for (int ci = 0; ci < ncls; ++ci) {
            std::fill(std::begin(i64[ci].cur), std::end(i64[ci].cur), 0);
            std::fill(std::begin(i32[ci].cur), std::end(i32[ci].cur), 0);
            const ClassPlan& C = SP.classes[ci];
            st = chunked(C.top1d, C.K, [&](int k0, int kn) {
                return launch_fmg(C.top1d, kn, X.probs + C.first + k0, X.active + C.first + k0, c, it64.v[0], a64b,
                                  d_u_out, bpyr, d_kx, d_ky, s);
            });
            if (st != MSG_OK) return st;
        }
        // classes that fit in LDS: the whole adaptive loop in one kernel, all
        // such classes of the level in one launch so that their slowest
        // problems overlap
        {
            cls.assign(SP.K, -1);
            size_t lds = 0;
            double bytes = 0.0;
            int64_t nsolve = 0;
            for (const ClassPlan& C : SP.classes) {
                if (!C.solve_in_tail) continue;
                for (int k = 0; k < C.K; ++k) cls[C.first + k] = 2 * C.ci + 1;
                lds = std::max(lds, C.tail64_lds);
                bytes += tail_bytes(C.tail64, sizeof(double)) * C.K;
                nsolve += C.K;
            }
            if (nsolve > 0) {
                HIPCHK(hipMemcpyAsync(ws + W.cls, cls.data(), sizeof(int32_t) * SP.K, hipMemcpyHostToDevice, s));
                const int threads = lds >= 24576 ? 256 : 64;
                st = timed(X, MSG_KERNEL_TAIL, bytes, [&]() -> msg_status {
                    const int64_t per = (int64_t)1 << 30;
                    for (int64_t k0 = 0; k0 < SP.K; k0 += per) {
                        const int kn = (int)std::min<int64_t>(per, SP.K - k0);
                        TailSolve ad{opts->tol, opts->max_cycles, SP.L, pcycles + k0, d_status, dead};
                        hipError_t e = launch_tail<double>(X.tails, (const int32_t*)(ws + W.cls) + k0, 0, (int)k0, threads, lds,
                                                           kn, X.probs + k0, X.active + k0, c, opts->mu, opts->nu1,
                                                           opts->nu2, opts->omega, -1, 0, it64.v[0], a64b, d_kx, d_ky,
                                                           nullptr, chol, ad, s);
                        if (e != hipSuccess) return fail(MSG_ERR_HIP, "tail launch: %s", hipGetErrorString(e));
                    }
                    return MSG_OK;
                }, -1, true);
                if (st != MSG_OK) return st;
            }
        }
        // captured W-cycles of this stage's classes (not while timing kernels:
        // the per-launch events would be captured too)
        const bool use_graphs = opts->graphs > 0 && !ln.prof.on;
        std::vector<ClassGraph> graphs(ncls);
        // adaptive number of cycles per problem (Section 2): check, then cycle
        std::vector<int32_t> host_active(ncls, 0);
        std::vector<char> handed(ncls, 0);
        int iters = 0;
        for (int it = 0; it <= opts->max_cycles + 1; ++it) {
            // classes down to a few slow problems whose rectangle fits in LDS:
            // the rest of their adaptive loop runs in one kernel (all such
            // classes together), continuing from their current iterates
            const int handoff = opts->handoff >= 0 ? opts->handoff : g_handoff;
            if (it > 0 && handoff > 0) {
                // one launch per iterate buffer the handed classes are on
                for (int buf = 0; buf < 2; ++buf) {
                    size_t lds = 0;
                    int64_t n = 0;
                    for (int ci = 0; ci < ncls; ++ci) {
                        const ClassPlan& C = SP.classes[ci];
                        if (C.solve_in_tail || handed[ci] || host_active[ci] == 0 || host_active[ci] > handoff)
                            continue;
                        if (C.tail64_lds == 0 || C.tail64_lds > 160 * 1024 || i64[ci].cur[SP.L] != buf) continue;
                        if (n == 0) cls.assign(SP.K, -1);
                        for (int k = 0; k < C.K; ++k) cls[C.first + k] = 2 * C.ci + 1;
                        lds = std::max(lds, C.tail64_lds);
                        n += host_active[ci];
                        handed[ci] = 1;
                        host_active[ci] = 0;
                    }
                    if (n == 0) continue;
                    HIPCHK(hipMemcpyAsync(ws + W.cls, cls.data(), sizeof(int32_t) * SP.K, hipMemcpyHostToDevice, s));
                    TailSolve ad{opts->tol, opts->max_cycles, SP.L, pcycles, d_status, dead};
                    st = timed(X, MSG_KERNEL_TAIL, 0.0, [&]() -> msg_status {
                        hipError_t e = launch_tail<double>(X.tails, (const int32_t*)(ws + W.cls), 0, 0,
                                                           lds >= 24576 ? 256 : 64, lds, SP.K, X.probs, X.active, c,
                                                           opts->mu, opts->nu1, opts->nu2, opts->omega, -1, 0,
                                                           it64.v[buf], a64b, d_kx, d_ky, nullptr, chol, ad, s);
                        if (e != hipSuccess) return fail(MSG_ERR_HIP, "handoff launch: %s", hipGetErrorString(e));
                        return MSG_OK;
                    }, -1, true);
                    if (st != MSG_OK) return st;
                    // the device copy of cls must be consumed before the host vector is rebuilt
                    HIPCHK(hipStreamSynchronize(s));
                }
            }
            HIPCHK(hipMemsetAsync(nact, 0, sizeof(int32_t) * ncls, s));
            iters = it;
            for (int ci = 0; ci < ncls; ++ci) {
                const ClassPlan& C = SP.classes[ci];
                if (C.solve_in_tail || handed[ci]) continue;   // solved in one kernel
                if (it > 0 && host_active[ci] == 0) continue;   // this class has stopped
                if (mixed) i32[ci].cur[SP.L] = 0;          // the check writes the FP32 top iterate (zero)
                const double nb = (3.0 * grid_cells(c, C.pc, C.qc) + (double)((c << C.pc) + 1) * (c << C.qc) +
                                   (double)(c << C.pc) * ((c << C.qc) + 1)) * sizeof(double) *
                                  (it == 0 ? C.K : host_active[ci]);
                const double* vtop = i64[ci].now(SP.L);
                st = timed(X, MSG_KERNEL_RESIDUAL_NORM, nb, [&] {
                    return chunked(C.top1d, C.K, [&](int k0, int kn) {
                        return launch_resnorm(C.top1d, kn, X.probs + C.first + k0, X.active + C.first + k0, c,
                                              vtop, a64b, d_kx, d_ky, part, it32.v[0], a32b, s);
                    });
                });
                if (st != MSG_OK) return st;
                hipError_t e = launch_converge(C.K, C.top1d.ntiles, X.probs + C.first, X.active + C.first,
                                               pcycles + C.first, dead, d_status, part, opts->tol, opts->max_cycles,
                                               SP.L, nact + ci, s);
                if (e != hipSuccess) return fail(MSG_ERR_HIP, "converge: %s", hipGetErrorString(e));
            }
            HIPCHK(hipMemcpyAsync(host_active.data(), nact, sizeof(int32_t) * ncls, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (ln.prof.on) ln.prof.resolve();
            int64_t any = 0;
            for (int32_t a : host_active) any += a;
            if (any == 0) break;
            // one W-cycle per class still cycling.  With overlap the classes
            // alternate over two streams forked from this part's stream, so
            // that one's on-chip, latency-bound tail runs beside another's
            // bandwidth-bound sweeps.  They touch disjoint problems.
            // Graphs are captured on library streams only (the caller's may
            // be the null stream, which cannot be captured): without overlap
            // the classes then run on the lane's own stream, forked from and
            // joined back to the part's stream.
            const bool fork = ov > 0 || use_graphs;
            int rr = 0;
            if (!use_graphs) {
                // the classes still cycling, in lockstep groups of equal tail
                // level and tail workgroup: one tail launch per group visit
                std::vector<Group> groups;
                std::vector<std::vector<int>> gci;
                for (int ci = 0; ci < ncls; ++ci) {
                    const ClassPlan& C = SP.classes[ci];
                    if (host_active[ci] == 0) continue;
                    size_t g = 0;
                    while (g < groups.size() &&
                           (groups[g].tail_top != C.tail_top || groups[g].tail_threads != C.tail_threads))
                        ++g;
                    if (g == groups.size()) {
                        groups.push_back(single_group(C, Span{0, C.K}, host_active[ci]));
                        gci.push_back({ci});
                        continue;
                    }
                    groups[g].m.push_back(Member{&C, Span{0, C.K}, host_active[ci]});
                    groups[g].tail_lds = std::max(groups[g].tail_lds, C.tail_lds);
                    gci[g].push_back(ci);
                }
                gcls_host.resize(groups.size());
                for (size_t g = 0; g < groups.size(); ++g) {
                    Group& G = groups[g];
                    if (G.m.size() < 2) continue;
                    G.gfirst = INT_MAX;
                    G.gend = 0;
                    gcls_host[g].assign(SP.K, -1);
                    for (const Member& e : G.m) {
                        G.gfirst = std::min(G.gfirst, e.C->first);
                        G.gend = std::max(G.gend, e.C->first + e.C->K);
                        for (int k = 0; k < e.C->K; ++k) gcls_host[g][e.C->first + k] = 2 * e.C->ci;
                    }
                    // uploaded only when the group's membership changed since the
                    // last cycle of this stage (a class stopped)
                    int32_t* d = (int32_t*)(ws + W.gcls) + (int64_t)g * SP.K;
                    if (gcls_sent.size() <= g) gcls_sent.resize(g + 1);
                    if (gcls_sent[g] != gcls_host[g]) {
                        HIPCHK(hipMemcpyAsync(d, gcls_host[g].data(), sizeof(int32_t) * SP.K, hipMemcpyHostToDevice, s));
                        gcls_sent[g] = gcls_host[g];
                    }
                    G.gcls = d;
                }
                if (fork) {
                    HIPCHK(hipEventRecord(ln.fork, s));
                    for (int k = 0; k < g_side; ++k) HIPCHK(hipStreamWaitEvent(ln.side[k], ln.fork, 0));
                }
                for (size_t g = 0; g < groups.size(); ++g) {
                    const Group& G = groups[g];
                    Ctx Y = X;
                    Y.s = ov > 0 ? ln.side[rr++ % g_side] : s;
                    // the members' buffer states are equal: they have cycled together
                    // since the stage began
                    const int c0 = gci[g][0];
                    if (!mixed) {
                        Iter<double> it = i64[c0];
                        if ((st = mu_cycle<double>(Y, G, SP.L, it, a64b, d_kx, d_ky)) != MSG_OK) return st;
                        for (int ci : gci[g]) i64[ci] = it;
                        continue;
                    }
                    Iter<float> it = i32[c0];
                    if ((st = mu_cycle<float>(Y, G, SP.L, it, a32b, d_kx32, d_ky32)) != MSG_OK) return st;
                    for (int ci : gci[g]) i32[ci] = it;
                    for (int ci : gci[g]) {
                        const ClassPlan& C = SP.classes[ci];
                        const float* e32 = i32[ci].now(SP.L);
                        st = chunked(C.top1d, C.K, [&](int k0, int kn) {
                            const int a = C.first + k0;
                            return launch_ir_update(C.top1d, kn, X.probs + a, X.active + a, it64.v[0], e32, Y.s);
                        });
                        if (st != MSG_OK) return st;
                    }
                }
            } else {
            if (fork) {
                HIPCHK(hipEventRecord(ln.fork, s));
                for (int k = 0; k < g_side; ++k) HIPCHK(hipStreamWaitEvent(ln.side[k], ln.fork, 0));
            }
            int rr = 0;
            for (int ci = 0; ci < ncls; ++ci) {
                const ClassPlan& C = SP.classes[ci];
                if (host_active[ci] == 0) continue;        // every problem of this class has stopped
                Ctx Y = X;
                Y.kact = host_active[ci];
                Y.s = ov > 0 ? ln.side[rr++ % g_side] : (use_graphs ? ln.side[0] : s);
                const Span span{0, C.K};
                // one W-cycle of the class (and its refinement update)
                auto cycle = [&]() -> msg_status {
                    const Group G1 = single_group(C, span, Y.kact);
                    if (!mixed) return mu_cycle<double>(Y, G1, SP.L, i64[ci], a64b, d_kx, d_ky);
                    msg_status r = mu_cycle<float>(Y, G1, SP.L, i32[ci], a32b, d_kx32, d_ky32);
                    if (r != MSG_OK) return r;
                    const float* e32 = i32[ci].now(SP.L);
                    return chunked(C.top1d, C.K, [&](int k0, int kn) {
                        const int a = C.first + k0;
                        return launch_ir_update(C.top1d, kn, X.probs + a, X.active + a, it64.v[0], e32, Y.s);
                    });
                };
                if (!use_graphs) {
                    if ((st = cycle()) != MSG_OK) return st;
                    continue;
                }
                // The launch sequence of a class's W-cycle is the same every
                // cycle of the stage (stopped problems are masked on the
                // device), so it is captured once and replayed.
                ClassGraph& G = graphs[ci];
                if (!G.exec) {
                    G.before64 = i64[ci];
                    G.before32 = i32[ci];
                    HIPCHK(hipStreamBeginCapture(Y.s, hipStreamCaptureModeThreadLocal));
                    const msg_status r = cycle();
                    hipGraph_t g = nullptr;
                    const hipError_t e = hipStreamEndCapture(Y.s, &g);
                    if (r != MSG_OK) {
                        if (g) (void)hipGraphDestroy(g);
                        return r;
                    }
                    if (e != hipSuccess) return fail(MSG_ERR_HIP, "W-cycle capture: %s", hipGetErrorString(e));
                    G.graph = g;
                    HIPCHK(hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0));
                    G.after64 = i64[ci];
                    G.after32 = i32[ci];
                } else {
                    // replays assume the buffer state the capture started from
                    if (!same_start(i64[ci], G.before64, SP.L) || !same_start(i32[ci], G.before32, SP.L))
                        return fail(MSG_ERR_HIP, "W-cycle graph replay from a different buffer state");
                    i64[ci] = G.after64;
                    i32[ci] = G.after32;
                }
                HIPCHK(hipGraphLaunch(G.exec, Y.s));
            }
            }
            for (int k = 0; fork && k < g_side; ++k) {
                HIPCHK(hipEventRecord(ln.join[k], ln.side[k]));
                HIPCHK(hipStreamWaitEvent(s, ln.join[k], 0));
            }
        }
        // returned solutions of this level and their means
        for (int ci = 0; ci < ncls; ++ci) {
            const ClassPlan& C = SP.classes[ci];
            const double* vtop = i64[ci].now(SP.L);
            st = chunked(C.top1d, C.K, [&](int k0, int kn) {
                return launch_snapshot(C.top1d, kn, X.probs + C.first + k0, dead, SP.L, c, vtop, d_u_out, part, s);
            });
            if (st != MSG_OK) return st;
            const int64_t cells = grid_cells(c, C.pc, C.qc);
            hipError_t e = launch_qreduce(C.K, C.top1d.ntiles, cells, X.probs + C.first, pcycles + C.first,
                                          (const int64_t*)(ws + W.gbase), part, d_q_out, d_cycles, s);
            if (e != hipSuccess) return fail(MSG_ERR_HIP, "qreduce: %s", hipGetErrorString(e));
        }
        if (g_debug_stages) {
            HIPCHK(hipStreamSynchronize(s));
            int in_tail = 0;
            for (const ClassPlan& C : SP.classes) in_tail += C.solve_in_tail;
            const double ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_stage).count();
            std::fprintf(stderr, "[msg] level %2d: %2d classes (%d in one kernel, tail top %d), %6d problems, "
                                 "%4d host iterations, %9.2f ms\n",
                         SP.L, ncls, in_tail, SP.classes.back().tail_top, SP.K, iters, ms);
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    if (ln.prof.on) ln.prof.resolve();
    return MSG_OK;
}

}  // namespace

extern "C" msg_status msg_solve_batch(msg_handle h, const msg_batch_desc* batch, const msg_solve_opts* opts,
                                      const double* d_kx, const double* d_ky, const float* d_kx32,
                                      const float* d_ky32, const double* d_rhs, double* d_u_out, double* d_q_out,
                                      int32_t* d_status, int32_t* d_cycles, void* d_ws, size_t ws_bytes,
                                      msg_stream stream)
{
    if (!h) return fail(MSG_ERR_ARG, "handle is NULL");
    msg_status st = check_batch(batch);
    if (st != MSG_OK) return st;
    if ((st = check_opts(opts)) != MSG_OK) return st;
    if (!d_kx || !d_ky || !d_u_out || !d_q_out || !d_status || !d_ws)
        return fail(MSG_ERR_ARG, "kx, ky, u_out, q_out, status and workspace are required");
    const bool mixed = opts->precision == MSG_MIXED;
    if (mixed && (!d_kx32 || !d_ky32)) return fail(MSG_ERR_ARG, "mixed precision needs the FP32 coefficient copies");
    if ((uintptr_t)d_ws % kAlign) return fail(MSG_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
    hipStream_t s = (hipStream_t)stream;
    const int mode = overlap_mode(batch, opts);
    if (mode < 2)
        return solve_part(h, h->lane[0], mode, batch, opts, d_kx, d_ky, d_kx32, d_ky32, d_rhs, d_u_out, d_q_out,
                          d_status, d_cycles, d_ws, ws_bytes, s);

    // parts of the batch, each a whole F-cycle of its own on one stream of
    // its own (forked from and joined back to the caller's), driven by one
    // host thread each: one part's long-running problems, latency-bound tails
    // and host round trips overlap the others' work.  Each part uses a single
    // stream: more streams than the device's hardware queues share queues and
    // serialise (measured: 244 samples/s against 210 with the classes of
    // each of two halves also on two streams, 256x256 x 4096)
    const Split sp = split_batch(batch, opts);
    if (ws_bytes < sp.total) return fail(MSG_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, sp.total);
    const BatchLayout BL = make_layout(batch);
    HIPCHK(hipSetDevice(h->device));
    for (int k = 0; k < sp.n; ++k) HIPCHK(h->lane[k].streams(g_split_inner > 0));
    HIPCHK(hipEventRecord(h->lane[0].done, s));
    for (int k = 0; k < sp.n; ++k) HIPCHK(hipStreamWaitEvent(h->lane[k].own, h->lane[0].done, 0));
    msg_status res[kMaxParts];
    std::string err[kMaxParts];
    auto part = [&](int k) {
        const int a = sp.first[k];
        if (hipSetDevice(h->device) != hipSuccess) {
            res[k] = MSG_ERR_HIP;
            err[k] = "hipSetDevice failed";
            return;
        }
        res[k] = solve_part(h, h->lane[k], g_split_inner, &sp.part[k], opts, d_kx + BL.xf[a], d_ky + BL.yf[a],
                            d_kx32 ? d_kx32 + BL.xf[a] : nullptr, d_ky32 ? d_ky32 + BL.yf[a] : nullptr,
                            d_rhs ? d_rhs + BL.top[a] : nullptr, d_u_out + BL.cell[a], d_q_out + BL.grid[a],
                            d_status + a, d_cycles ? d_cycles + BL.grid[a] : nullptr, (char*)d_ws + sp.ws_off[k],
                            sp.ws_bytes[k], h->lane[k].own);
        if (res[k] != MSG_OK) err[k] = msg_last_error();
    };
    std::vector<std::thread> threads;
    for (int k = 1; k < sp.n; ++k) threads.emplace_back(part, k);
    part(0);
    for (std::thread& t : threads) t.join();
    for (int k = 0; k < sp.n; ++k) {
        HIPCHK(hipEventRecord(h->lane[k].done, h->lane[k].own));
        HIPCHK(hipStreamWaitEvent(s, h->lane[k].done, 0));
    }
    for (int k = 0; k < sp.n; ++k)
        if (res[k] != MSG_OK) return fail(res[k], "part %d: %s", k, err[k].c_str());
    return MSG_OK;
}

// ---------------------------------------------------------------- plain cycles
namespace {

// Standard multigrid on the grids (P-k, Q-k), k = 0..m, of a sample: their
// arena offsets and the launches on each.
struct MgPlan {
    int m = 0;
    int64_t stride = 0;                 // arena cells per problem
    std::vector<int64_t> goff;          // arena offset of grid k
    std::vector<KLevel> rb;             // smoother tiles of grid k
    std::vector<KLevel> res;            // restriction into grid k (k >= 1) from grid k-1
    std::vector<KLevel> pro;            // prolongation onto grid k (k < m) from grid k+1
    KLevel top1d;                       // grid 0, 1-D tiles of kBlock cells
};

KLevel one_grid(KLevel L, int64_t aoff, int64_t aoff_x)
{
    L.g[0].aoff = aoff;
    L.g[0].aoff_x = aoff_x;
    L.g[0].aoff_y = -1;
    return L;
}

MgPlan plan_mg(int c, int P, int Q, const Tuning& tu)
{
    MgPlan M;
    M.m = std::min(P, Q);
    const int H = 2 * g_fuse;
    for (int k = 0; k <= M.m; ++k) {
        M.goff.push_back(M.stride);
        M.stride += grid_cells(c, P - k, Q - k);
    }
    M.rb.resize(M.m + 1);
    M.res.resize(M.m + 1);
    M.pro.resize(M.m + 1);
    for (int k = 0; k <= M.m; ++k) {
        // the class (a,b) on its own level a+b holds the single grid (a,b)
        const int a = P - k, b = Q - k;
        const std::vector<int64_t> zero((size_t)(a + 1) * (b + 1), 0);
        M.rb[k] = one_grid(level_rbgs(c, a, b, a + b, zero, H, tu), M.goff[k], -1);
        const KLevel l1 = level_1d(c, a, b, a + b, zero, 0, b);
        if (k > 0) M.res[k] = one_grid(l1, M.goff[k], M.goff[k - 1]);
        if (k < M.m) M.pro[k] = one_grid(l1, M.goff[k], M.goff[k + 1]);
        if (k == 0) M.top1d = one_grid(l1, M.goff[0], -1);
    }
    return M;
}

struct CycWs {
    size_t chol, v0, v1, b, part, active, probs, sbase, tails, tpack, total;
};

CycWs cycles_ws(const BatchLayout& BL, int64_t stride, int64_t top_tiles, int64_t nstat)
{
    const int64_t S = BL.S, n0 = (int64_t)BL.c * BL.c;
    CycWs w;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
    w.chol = take(sizeof(double) * S * n0 * n0);
    w.v0 = take(sizeof(double) * S * stride);
    w.v1 = take(sizeof(double) * S * stride);
    w.b = take(sizeof(double) * S * stride);
    w.part = take(sizeof(double) * 2 * S * top_tiles);
    w.active = take(sizeof(int32_t) * S);
    w.probs = take(sizeof(KProb) * S);
    w.sbase = take(sizeof(SampleBase) * S);
    w.tails = take(sizeof(KTail) * 2);
    w.tpack = take(sizeof(double) * std::max<int64_t>(1, nstat * S));
    w.total = off;
    return w;
}

msg_status check_cycles(const msg_batch_desc* batch, const msg_solve_opts* opts, int kind)
{
    msg_status st = check_batch(batch);
    if (st != MSG_OK) return st;
    if ((st = check_opts(opts)) != MSG_OK) return st;
    if (kind != MSG_CYCLES_MSG && kind != MSG_CYCLES_MG) return fail(MSG_ERR_ARG, "unknown cycle kind %d", kind);
    if (opts->precision != MSG_FP64) return fail(MSG_ERR_UNSUPPORTED, "plain cycles run in FP64 only");
    const int P = batch->P[0], Q = batch->Q[0];
    for (int s = 1; s < batch->n_samples; ++s)
        if (batch->P[s] != P || batch->Q[s] != Q)
            return fail(MSG_ERR_UNSUPPORTED, "plain cycles need the same (P,Q) for every sample (sample %d)", s);
    if (kind == MSG_CYCLES_MG && P != Q)
        return fail(MSG_ERR_UNSUPPORTED, "standard multigrid needs P == Q (got %d, %d)", P, Q);
    return MSG_OK;
}

// the MSG class (P,Q) cycled on the host down to its on-chip tail
ClassPlan cycles_class(const BatchLayout& BL, const msg_solve_opts& o)
{
    std::vector<int> samples(BL.S);
    for (int s = 0; s < BL.S; ++s) samples[s] = s;
    ClassPlan C = plan_class(BL.c, BL.P[0], BL.Q[0], std::move(samples), o, tuning_of(o), true);
    C.tpack = 0;
    return C;
}

size_t cycles_ws_bytes(const BatchLayout& BL, const msg_solve_opts& o, int kind)
{
    if (kind == MSG_CYCLES_MG) {
        const MgPlan M = plan_mg(BL.c, BL.P[0], BL.Q[0], tuning_of(o));
        return cycles_ws(BL, M.stride, M.top1d.ntiles, 0).total;
    }
    const ClassPlan C = cycles_class(BL, o);
    return cycles_ws(BL, C.stride, C.top1d.ntiles, C.tail.nstat).total;
}

// One standard-multigrid mu-cycle on grid k (the comparison method of
// Section 2): pre-smoothing, 2D restriction of the residual, mu cycles on the
// next coarser grid (the exact solve on grid m), bilinear correction,
// post-smoothing.
msg_status mg_cycle(const Ctx& X, const MgPlan& M, int k, Iter<double>& it, double* B, const double* KX,
                    const double* KY)
{
    const int K = (int)X.kact;
    msg_status st;
    if (k == M.m) {
        double* v = it.now(k);
        return timed(X, MSG_KERNEL_TAIL, 0.0, [&]() -> msg_status {
            hipError_t e = launch_dense_apply(K, X.probs, X.active, X.c * X.c, M.goff[k], X.chol, v, B, X.s);
            if (e != hipSuccess) return fail(MSG_ERR_HIP, "coarsest solve: %s", hipGetErrorString(e));
            return MSG_OK;
        });
    }
    auto smooth = [&](int sweeps) -> msg_status {
        const KLevel& L = M.rb[k];
        while (sweeps > 0) {
            const int ns = (sweeps >= 2 && g_fuse == 2) ? 2 : 1;
            const double* vin = it.now(k);
            double* vout = it.v[1 - it.cur[k]];
            msg_status r = timed(
                X, MSG_KERNEL_SMOOTH, level_bytes<double>(L, 0, K),
                [&] {
                    return chunked(L, K, [&](int k0, int kn) {
                        return launch_rbgs<double>(ns, L, kn, X.probs + k0, X.active + k0, X.c, vin, vout, B, KX,
                                                   KY, nullptr, X.o->omega, X.s);
                    });
                },
                -1, false, model_bytes<double>(L, 5.0 * ns, K));
            if (r != MSG_OK) return r;
            it.cur[k] ^= 1;
            sweeps -= ns;
        }
        return MSG_OK;
    };
    if ((st = smooth(X.o->nu1)) != MSG_OK) return st;
    {
        const KLevel& L = M.res[k + 1];
        const double* vf = it.now(k);
        double* vc = it.v[0];
        const KGrid& G = L.g[0];
        // fine v, b and faces read; coarse b and v written
        const double fine = 4.0 * G.nx * G.ny;
        const double bytes = (2.0 * fine + (2.0 * G.nx + 1) * 2 * G.ny + 2.0 * G.nx * (2 * G.ny + 1) +
                              2.0 * G.nx * G.ny) * sizeof(double) * K;
        st = timed(X, MSG_KERNEL_RESTRICT, bytes, [&] {
            return chunked(L, K, [&](int k0, int kn) {
                return launch_restrict2d(L, kn, X.probs + k0, X.active + k0, X.c, vf, vc, B, KX, KY, X.s);
            });
        });
        if (st != MSG_OK) return st;
        it.cur[k + 1] = 0;
    }
    for (int t = 0; t < X.o->mu; ++t)
        if ((st = mg_cycle(X, M, k + 1, it, B, KX, KY)) != MSG_OK) return st;
    {
        const KLevel& L = M.pro[k];
        const double* vc = it.now(k + 1);
        double* vf = it.now(k);
        const KGrid& G = L.g[0];
        const double bytes = (2.0 * G.nx * G.ny + G.nx * G.ny / 4.0) * sizeof(double) * K;
        st = timed(X, MSG_KERNEL_PROLONG, bytes, [&] {
            return chunked(L, K, [&](int k0, int kn) {
                return launch_prolong2d(L, kn, X.probs + k0, X.active + k0, X.o->omega, vc, vf, X.s);
            });
        });
        if (st != MSG_OK) return st;
    }
    return smooth(X.o->nu2);
}

}  // namespace

extern "C" msg_status msg_cycles_workspace_size(msg_handle, const msg_batch_desc* batch, const msg_solve_opts* opts,
                                                int kind, size_t* bytes)
{
    if (!bytes) return fail(MSG_ERR_ARG, "output is required");
    msg_status st = check_cycles(batch, opts, kind);
    if (st != MSG_OK) return st;
    read_env();
    *bytes = cycles_ws_bytes(make_layout(batch), *opts, kind);
    return MSG_OK;
}

extern "C" msg_status msg_cycles(msg_handle h, const msg_batch_desc* batch, const msg_solve_opts* opts, int kind,
                                 int ncycles, const double* d_kx, const double* d_ky, const double* d_rhs,
                                 double* d_u_top, double* d_ratios, void* d_ws, size_t ws_bytes, msg_stream stream)
{
    if (!h) return fail(MSG_ERR_ARG, "handle is NULL");
    msg_status st = check_cycles(batch, opts, kind);
    if (st != MSG_OK) return st;
    if (ncycles < 0 || ncycles > 10000) return fail(MSG_ERR_ARG, "ncycles must be 0..10000 (got %d)", ncycles);
    if (!d_kx || !d_ky || !d_u_top || !d_ratios || !d_ws)
        return fail(MSG_ERR_ARG, "kx, ky, u_top, ratios and the workspace are required");
    if ((uintptr_t)d_ws % kAlign) return fail(MSG_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
    const BatchLayout BL = make_layout(batch);
    const int c = BL.c, S = BL.S, P = BL.P[0], Q = BL.Q[0];
    const bool mg = kind == MSG_CYCLES_MG;
    const Tuning tu = tuning_of(*opts);
    MgPlan M;
    ClassPlan C;
    if (mg) {
        M = plan_mg(c, P, Q, tu);
    } else {
        C = cycles_class(BL, *opts);
        if (C.tail_lds == 0 || C.tail_lds > 160 * 1024)
            return fail(MSG_ERR_UNSUPPORTED, "tail of class (%d,%d) does not fit LDS; lower tail_levels", P, Q);
    }
    const int64_t stride = mg ? M.stride : C.stride;
    const KLevel top1d = mg ? M.top1d : C.top1d;
    const int64_t top_off = mg ? M.goff[0] : C.goff[P * (Q + 1) + Q];
    const CycWs W = cycles_ws(BL, stride, top1d.ntiles, mg ? 0 : C.tail.nstat);
    if (ws_bytes < W.total) return fail(MSG_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, W.total);
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    Lane& ln = h->lane[0];

    // host tables, alive until the final synchronisation
    const std::vector<SampleBase> bases = sample_bases(BL);
    std::vector<KProb> probs(S);
    for (int k = 0; k < S; ++k) {
        KProb& p = probs[k];
        std::memset(&p, 0, sizeof p);
        p.sample = k;
        p.Qs = Q;
        p.cell_base = BL.cell[k];
        p.fx_base = BL.xf[k];
        p.fy_base = BL.yf[k];
        p.arena_base = (int64_t)k * stride;
        p.part_base = (int64_t)k * top1d.ntiles;
        p.grid_index = P * (Q + 1) + Q;
    }
    const std::vector<int32_t> ones(S, 1);
    KTail tails[2] = {C.tail, C.tail64};
    HIPCHK(hipMemcpyAsync(ws + W.sbase, bases.data(), sizeof(SampleBase) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws + W.probs, probs.data(), sizeof(KProb) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws + W.active, ones.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, s));
    if (!mg) HIPCHK(hipMemcpyAsync(ws + W.tails, tails, sizeof tails, hipMemcpyHostToDevice, s));

    Ctx X;
    X.BL = &BL;
    X.o = opts;
    X.s = s;
    X.c = c;
    X.chol = (const double*)(ws + W.chol);
    X.probs = (KProb*)(ws + W.probs);
    X.active = (int32_t*)(ws + W.active);
    X.prof = &ln.prof;
    X.kact = S;
    X.tails = (const KTail*)(ws + W.tails);
    X.tpack = ws + W.tpack;
    double* B = (double*)(ws + W.b);
    double* part = (double*)(ws + W.part);
    Iter<double> it;
    it.v[0] = (double*)(ws + W.v0);
    it.v[1] = (double*)(ws + W.v1);
    std::fill(std::begin(it.cur), std::end(it.cur), 0);

    {
        hipError_t e = launch_chol(S, c, (const SampleBase*)(ws + W.sbase), d_kx, d_ky, (double*)(ws + W.chol), s);
        if (e != hipSuccess) return fail(MSG_ERR_HIP, "cholesky launch: %s", hipGetErrorString(e));
    }
    if (!mg) {
        hipError_t e = launch_tail_pack<double>(X.tails, S, X.probs, c, d_kx, d_ky, (double*)X.tpack, s);
        if (e != hipSuccess) return fail(MSG_ERR_HIP, "tail image: %s", hipGetErrorString(e));
    }
    // the finest grid: v = 0, b = h
    KLevel top = top1d;
    top.g[0].aoff = top_off;
    st = chunked(top, S, [&](int k0, int kn) { return launch_plain_init(top, kn, X.probs + k0, d_rhs, it.v[0], B, s); });
    if (st != MSG_OK) return st;
    const int lev_top = mg ? 0 : P + Q;
    for (int k = 0; k <= ncycles; ++k) {
        const double* v = it.now(lev_top);
        st = chunked(top, S, [&](int k0, int kn) {
            return launch_resnorm(top, kn, X.probs + k0, X.active + k0, c, v, B, d_kx, d_ky, part, nullptr, nullptr,
                                  s);
        });
        if (st != MSG_OK) return st;
        hipError_t e = launch_ratio(S, top.ntiles, X.probs, part, d_ratios, k, ncycles + 1, s);
        if (e != hipSuccess) return fail(MSG_ERR_HIP, "ratio: %s", hipGetErrorString(e));
        if (k == ncycles) break;
        st = mg ? mg_cycle(X, M, 0, it, B, d_kx, d_ky)
                : mu_cycle<double>(X, single_group(C, Span{0, S}, S), P + Q, it, B, d_kx, d_ky);
        if (st != MSG_OK) return st;
    }
    const int64_t ntop = grid_cells(c, P, Q);
    HIPCHK(hipMemcpy2DAsync(d_u_top, sizeof(double) * ntop, it.now(lev_top) + top_off, sizeof(double) * stride,
                            sizeof(double) * ntop, S, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ln.prof.on) ln.prof.resolve();
    return MSG_OK;
}

// ---------------------------------------------------------------- Matern fields
namespace {

constexpr uint64_t kMaternKey1 = 0x6D617465726Eull;
constexpr int kMaternRowLog = 13;        // rows of up to 8192 points in one workgroup (128 KB of LDS)
constexpr int kMaternMaxLog = 15;        // longer rows (up to 32768 points) by the four-step FFT
constexpr int kMaternChunk = 8;          // samples per chunk at the suggested workspace size
constexpr int kMaternBlocks = 256;       // partial min/max blocks per sample

int log2_ceil(int64_t x)
{
    int l = 0;
    while (((int64_t)1 << l) < x) ++l;
    return l;
}

// log2 of the embedding lattice per direction for a sample of rectangle (P,Q)
void matern_shape(int c, int P, int Q, double nu, int pad, int& lx, int& ly)
{
    const int64_t Nx = (int64_t)c << P, Ny = (int64_t)c << Q;
    int m = pad > 0 ? pad : 1 + 2 * (int)std::ceil(std::sqrt(nu) * std::log2((double)std::max(Nx, Ny)));
    m = std::max(m, 2);                  // at least the minimal embedding
    lx = log2_ceil(m * 2 * Nx);
    ly = log2_ceil(m * 2 * Ny);
}

msg_status check_matern(const msg_batch_desc* batch, const msg_matern_spec* sp)
{
    msg_status st = check_batch(batch);
    if (st != MSG_OK) return st;
    if (!sp || !sp->eta || !sp->theta) return fail(MSG_ERR_ARG, "spec with eta and theta arrays is required");
    if (!(sp->lambda > 0.0) || !std::isfinite(sp->lambda)) return fail(MSG_ERR_ARG, "lambda must be positive");
    if (!(sp->nu > 0.0) || sp->nu > 8.0) return fail(MSG_ERR_ARG, "nu must be in (0, 8]");
    if (sp->pad < 0 || sp->pad > 64) return fail(MSG_ERR_ARG, "pad must be 0..64");
    for (int s = 0; s < batch->n_samples; ++s) {
        if (!(sp->eta[s] > 0.0) || !std::isfinite(sp->eta[s]) || !std::isfinite(sp->theta[s]))
            return fail(MSG_ERR_ARG, "sample %d: eta must be positive and theta finite", s);
        int lx, ly;
        matern_shape(batch->c, batch->P[s], batch->Q[s], sp->nu, sp->pad, lx, ly);
        if (lx > kMaternMaxLog || ly > kMaternMaxLog)
            return fail(MSG_ERR_UNSUPPORTED, "sample %d: embedding of 2^%d x 2^%d points exceeds 32768 per direction",
                        s, lx, ly);
    }
    return MSG_OK;
}

struct MatWs {
    size_t tw, smp, idx, part, a, b, total;
    int chunk;
};

// workspace with room for `chunk` samples of the largest embedding
MatWs matern_ws(const msg_batch_desc* batch, const msg_matern_spec* sp, int chunk)
{
    int64_t mmax = 1;
    int lmax = 1;
    for (int s = 0; s < batch->n_samples; ++s) {
        int lx, ly;
        matern_shape(batch->c, batch->P[s], batch->Q[s], sp->nu, sp->pad, lx, ly);
        mmax = std::max<int64_t>(mmax, (int64_t)1 << (lx + ly));
        lmax = std::max(lmax, std::max(lx, ly));
    }
    MatWs w;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
    w.tw = take(sizeof(double2) * ((size_t)1 << (lmax - 1)));
    w.smp = take(sizeof(MaternSample) * batch->n_samples);
    w.idx = take(sizeof(int32_t) * batch->n_samples);
    w.part = take(sizeof(double2) * kMaternBlocks * chunk);
    w.a = take(sizeof(double2) * mmax * chunk);
    w.b = take(sizeof(double2) * mmax * chunk);
    w.total = off;
    w.chunk = chunk;
    return w;
}

}  // namespace

extern "C" msg_status msg_matern_workspace_size(const msg_batch_desc* batch, const msg_matern_spec* spec,
                                                size_t* bytes)
{
    if (!bytes) return fail(MSG_ERR_ARG, "output is required");
    msg_status st = check_matern(batch, spec);
    if (st != MSG_OK) return st;
    *bytes = matern_ws(batch, spec, std::min(batch->n_samples, kMaternChunk)).total;
    return MSG_OK;
}

extern "C" msg_status msg_sample_matern(msg_handle h, const msg_matern_spec* sp, const msg_batch_desc* batch,
                                        double* d_kx, double* d_ky, float* d_kx32, float* d_ky32, double* d_ratio,
                                        void* d_ws, size_t ws_bytes, msg_stream stream)
{
    if (!h) return fail(MSG_ERR_ARG, "handle is NULL");
    msg_status st = check_matern(batch, sp);
    if (st != MSG_OK) return st;
    if (!d_kx || !d_ky || !d_ws) return fail(MSG_ERR_ARG, "kx, ky and the workspace are required");
    if ((d_kx32 == nullptr) != (d_ky32 == nullptr)) return fail(MSG_ERR_ARG, "give both FP32 copies or neither");
    if ((uintptr_t)d_ws % kAlign) return fail(MSG_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
    // as many samples per chunk as the workspace holds
    int chunk = 0;
    for (int k = std::min(batch->n_samples, 1 << 16); k >= 1; k = k > 64 ? k / 2 : k - 1)
        if (matern_ws(batch, sp, k).total <= ws_bytes) {
            chunk = k;
            break;
        }
    if (chunk == 0)
        return fail(MSG_ERR_WORKSPACE, "workspace of %zu bytes holds no sample; need %zu", ws_bytes,
                    matern_ws(batch, sp, 1).total);
    const MatWs W = matern_ws(batch, sp, chunk);
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    const int c = batch->c, S = batch->n_samples;
    const BatchLayout BL = make_layout(batch);

    // samples grouped by rectangle; per-sample table in group order
    std::map<std::pair<int, int>, std::vector<int>> rects;
    for (int k = 0; k < S; ++k) rects[{BL.P[k], BL.Q[k]}].push_back(k);
    std::vector<MaternSample> tab;
    std::vector<int32_t> idx;
    tab.reserve(S);
    idx.reserve(S);
    for (auto& kv : rects)
        for (int k : kv.second) {
            MaternSample m;
            const double a = 1.0 / std::sqrt(sp->eta[k] * sp->lambda), b = 1.0 / std::sqrt(sp->lambda);
            const double cs = std::cos(sp->theta[k]), sn = std::sin(sp->theta[k]);
            m.t00 = a * cs;
            m.t01 = -a * sn;
            m.t10 = b * sn;
            m.t11 = b * cs;
            m.id = sp->sample_id ? sp->sample_id[k] : k;
            m.fx_base = BL.xf[k];
            m.fy_base = BL.yf[k];
            tab.push_back(m);
            idx.push_back(k);
        }
    MaternSample* d_tab = (MaternSample*)(ws + W.smp);
    int32_t* d_idx = (int32_t*)(ws + W.idx);
    double2* tw = (double2*)(ws + W.tw);
    double2* part = (double2*)(ws + W.part);
    double2* A = (double2*)(ws + W.a);
    double2* B = (double2*)(ws + W.b);
    HIPCHK(hipMemcpyAsync(d_tab, tab.data(), sizeof(MaternSample) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_idx, idx.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, s));
    int lmax = 1;
    for (auto& kv : rects) {
        int lx, ly;
        matern_shape(c, kv.first.first, kv.first.second, sp->nu, sp->pad, lx, ly);
        lmax = std::max(lmax, std::max(lx, ly));
    }
    auto chk = [&](hipError_t e, const char* what) -> msg_status {
        return e == hipSuccess ? MSG_OK : fail(MSG_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    };
    // rows longer than one workgroup holds run as the four-step FFT
    // (MSG_MATERN_ROW_LOG lowers that length, for tests of the long-row path)
    int row_log = kMaternRowLog;
    // (at least half the longest row's log, so that both factors fit one workgroup)
    if (const char* t = std::getenv("MSG_MATERN_ROW_LOG"))
        row_log = std::max((kMaternMaxLog + 1) / 2, std::min(kMaternRowLog, std::atoi(t)));
    const int tw_log = std::min(lmax, row_log);
    auto fft = [&](int64_t rows, int logn, double2* X, double2* scratch) -> hipError_t {
        if (logn <= row_log) return launch_fft_rows(rows, logn, (1 << tw_log) >> logn, tw, X, s);
        return launch_fft_rows_long(rows, logn, (logn + 1) / 2, tw_log, tw, X, scratch, s);
    };
    if ((st = chk(launch_mat_twiddles(1 << tw_log, tw, s), "twiddles")) != MSG_OK) return st;
    const double coef = std::pow(2.0, 1.0 - sp->nu) / std::tgamma(sp->nu);
    int first = 0;
    for (auto& kv : rects) {
        const int P = kv.first.first, Q = kv.first.second, n = (int)kv.second.size();
        int lx, ly;
        matern_shape(c, P, Q, sp->nu, sp->pad, lx, ly);
        const int Mx = 1 << lx, My = 1 << ly;
        const int64_t M = (int64_t)Mx * My;
        const double hx = 1.0 / (2.0 * (double)((int64_t)c << P)), hy = 1.0 / (2.0 * (double)((int64_t)c << Q));
        for (int k0 = 0; k0 < n; k0 += chunk) {
            const int K = std::min(chunk, n - k0);
            const MaternSample* t = d_tab + first + k0;
            if ((st = chk(launch_mat_row(K, Mx, My, hx, hy, sp->nu, coef, t, A, s), "embedding row")) != MSG_OK ||
                (st = chk(fft((int64_t)K * My, lx, A, B), "fft")) != MSG_OK ||
                (st = chk(launch_transpose(K, My, Mx, A, B, s), "transpose")) != MSG_OK ||
                (st = chk(fft((int64_t)K * Mx, ly, B, A), "fft")) != MSG_OK)
                return st;
            if (d_ratio &&
                (st = chk(launch_eig_ratio(K, M, kMaternBlocks, B, part, d_idx + first + k0, d_ratio, s),
                          "eigenvalue check")) != MSG_OK)
                return st;
            if ((st = chk(launch_mat_xi(K, Mx, My, sp->seed, kMaternKey1, t, B, s), "normals")) != MSG_OK ||
                (st = chk(fft((int64_t)K * Mx, ly, B, A), "fft")) != MSG_OK ||
                (st = chk(launch_transpose(K, Mx, My, B, A, s), "transpose")) != MSG_OK ||
                (st = chk(fft((int64_t)K * My, lx, A, B), "fft")) != MSG_OK ||
                (st = chk(launch_mat_faces(K, c, P, Q, Mx, My, t, A, d_kx, d_ky, d_kx32, d_ky32, s), "faces")) !=
                    MSG_OK)
                return st;
        }
        first += n;
    }
    // the host tables above are read by the copies on the stream
    HIPCHK(hipStreamSynchronize(s));
    return MSG_OK;
}

extern "C" msg_status msg_set_profiling(msg_handle h, int enable)
{
    if (!h) return fail(MSG_ERR_ARG, "handle is NULL");
    if (enable < 0) return fail(MSG_ERR_ARG, "profiling rate %d is negative", enable);
    for (Lane& ln : h->lane) {
        ln.prof.on = enable != 0;
        ln.prof.every = std::max(1, enable);
        ln.prof.reset();
    }
    return MSG_OK;
}

extern "C" msg_status msg_get_profile(msg_handle h, int kind, msg_kernel_stats* out)
{
    if (!h || !out) return fail(MSG_ERR_ARG, "handle and output are required");
    if (kind < 0 || kind >= MSG_KERNEL_KINDS) return fail(MSG_ERR_ARG, "unknown kernel kind %d", kind);
    *out = msg_kernel_stats{0, 0.0, 0.0, 0.0};
    int64_t all = 0;
    msg_kernel_stats fx{0, 0.0, 0.0, 0.0};
    for (const Lane& ln : h->lane) {
        out->launches += ln.prof.tot[kind].launches;
        out->milliseconds += ln.prof.tot[kind].milliseconds;
        out->bytes += ln.prof.tot[kind].bytes;
        out->model_bytes += ln.prof.tot[kind].model_bytes;
        all += ln.prof.seen[kind];
        fx.launches += ln.prof.fixed[kind].launches;
        fx.milliseconds += ln.prof.fixed[kind].milliseconds;
        fx.bytes += ln.prof.fixed[kind].bytes;
        fx.model_bytes += ln.prof.fixed[kind].model_bytes;
    }
    // sampled timing: totals over the sampled population estimated from its
    // timed launches (zero when none was timed), plus the always-timed ones
    if (all > out->launches) {
        const double f = out->launches > 0 ? (double)all / (double)out->launches : 0.0;
        out->milliseconds *= f;
        out->bytes *= f;
        out->model_bytes *= f;
        out->launches = all;
    }
    out->launches += fx.launches;
    out->milliseconds += fx.milliseconds;
    out->bytes += fx.bytes;
    out->model_bytes += fx.model_bytes;
    return MSG_OK;
}
