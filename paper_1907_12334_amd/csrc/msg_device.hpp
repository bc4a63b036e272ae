// msg_device.hpp -- structures passed from the host scheduler to the HIP
// kernels of the batched MSG solver, and the closed-form offsets of the packed
// grid layout (grids of a sample packed p-major then q-minor, each grid
// row-major with x fastest; see include/msg.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msg {

constexpr int kMaxIndex = 14;          // largest p or q of a grid
constexpr int kMaxLevelGrids = kMaxIndex + 1;
constexpr int kMaxCosTerms = 64;
constexpr int kMaxModes = 64;
constexpr int kBlock = 256;            // threads per block of the level kernels
constexpr int kRbgsLds = 2048;         // LDS elements of a smoother tile (iterate with halo)
constexpr int kRbgsLdsMax = 8192;      // upper bound of a tuned tile (64 KB in FP64)

// ---- offsets of grid (p,q) inside a sample with finest index (P,Qs) ------
// cells of the grids before (p,q): sum over a < p, b <= Qs of c2^a c2^b,
// plus sum over b < q of c2^p c2^b.
__host__ __device__ inline int64_t cell_off(int c, int Qs, int p, int q)
{
    const int64_t c2 = (int64_t)c * c;
    return c2 * (((int64_t)1 << p) - 1) * (((int64_t)2 << Qs) - 1) + c2 * ((int64_t)1 << p) * (((int64_t)1 << q) - 1);
}
// x-faces: grid (a,b) holds (c2^a + 1) c2^b of them
__host__ __device__ inline int64_t xface_off(int c, int Qs, int p, int q)
{
    const int64_t rows = (int64_t)c * (((int64_t)2 << Qs) - 1);
    return rows * ((int64_t)c * (((int64_t)1 << p) - 1) + p) + ((int64_t)c * ((int64_t)1 << p) + 1) * (int64_t)c * (((int64_t)1 << q) - 1);
}
// y-faces: grid (a,b) holds c2^a (c2^b + 1) of them
__host__ __device__ inline int64_t yface_off(int c, int Qs, int p, int q)
{
    const int64_t cols = (int64_t)c * (((int64_t)2 << Qs) - 1) + (Qs + 1);
    return (int64_t)c * (((int64_t)1 << p) - 1) * cols + (int64_t)c * ((int64_t)1 << p) * ((int64_t)c * (((int64_t)1 << q) - 1) + q);
}
__host__ __device__ inline int64_t sample_cells(int c, int P, int Q) { return cell_off(c, Q, P + 1, 0); }
__host__ __device__ inline int64_t sample_xfaces(int c, int P, int Q) { return xface_off(c, Q, P + 1, 0); }
__host__ __device__ inline int64_t sample_yfaces(int c, int P, int Q) { return yface_off(c, Q, P + 1, 0); }

// One problem of an F-cycle level: grid (p,q) of one sample, iterated over
// its own rectangle [0..p] x [0..q].  Its iterates and right-hand sides live
// in the stage arena; its coefficients are the sample's.
struct KProb {
    int32_t sample;
    int32_t Qs;            // sample's finest y index (layout of its arrays)
    int64_t cell_base;     // sample's first cell in u_out / b_pyr
    int64_t fx_base;       // sample's first x-face
    int64_t fy_base;       // sample's first y-face
    int64_t arena_base;    // problem's first cell in the arena
    int64_t part_base;     // problem's first partial-sum slot
    int32_t grid_index;    // (p,q) as p*(Qs+1)+q inside the sample's per-grid arrays
    int32_t pad;
};

// One grid of a problem class at the level a kernel works on.
struct KGrid {
    int32_t nx, ny;        // cells
    int32_t p, q;          // grid index
    int32_t tw, th;        // tile of the smoother (cells)
    int32_t tiles_x;       // tiles per row of tiles
    int32_t tile0;         // first block of this grid inside the launch
    int64_t aoff;          // arena offset of the grid inside a problem
    int64_t aoff_x;        // arena offset of the x-related grid ((p+1,q) or (p-1,q)), -1 if none
    int64_t aoff_y;        // arena offset of the y-related grid ((p,q+1) or (p,q-1)), -1 if none
    int32_t rflags;        // restricting pass: bit 0, grid (p-1,q) has a second parent (p-1,q+1);
                           // bit 1, grid (p,q-1) has a second parent (p+1,q-1)
    int32_t pad;
};

struct KLevel {
    int32_t ngrids;
    int32_t ntiles;        // blocks per problem
    int32_t nblocks;       // real blocks of the launch (ntiles * problems); set by the launcher
    int32_t bs;            // threads per block (0: kBlock); a 1-D tile is bs consecutive cells
    int32_t lds;           // smoother: LDS elements of the largest tile with its halo
    int32_t pad;
    KGrid g[kMaxLevelGrids];
};

// The grids of levels 0..top of a problem class held in LDS by the tail
// kernel.  Every grid of level l of a class has c^2 2^l cells and grid index
// p = pmin + g (q = l - p), so a level is described by a handful of numbers:
// its grids' iterates and right-hand sides sit in blocks of `cells` elements;
// its x-face conductances follow each other (grid g starts at
// x0 + g*cells + c*(2^(qmax+1) - 2^(qmax+1-g)), qmax = l - pmin) and so do its
// y-face conductances (y0 + g*cells + c*2^pmin*(2^g - 1)).  The conductance
// runs of all levels come first, so that they form one image that can be
// prepared once per F-cycle stage and copied in whole.
struct KTailLevel {
    int32_t pmin, ng;          // grids p = pmin .. pmin+ng-1
    int32_t cells, csh;        // cells per grid and its log2 (or -1)
    int32_t v0, b0;            // LDS element offsets: iterates, right-hand sides
    int32_t x0, y0;            // LDS element offsets of the face conductance runs
};

constexpr int kMaxTailLevels = 9;        // levels 0..8
constexpr int kTailRegLevels = 3;        // tail levels that can keep their slot state in registers

struct KTail {
    int32_t top;               // level the cycles start on
    int32_t pc, qc;            // the class rectangle
    int32_t c, lc;             // coarsest cells per direction and its log2 (or -1)
    int32_t lds_elems;         // LDS elements of type T (the coarsest inverse in doubles follows)
    int32_t chol_off;          // byte offset of the coarsest-grid inverse in LDS
    int32_t nstat;             // elements [0, nstat): every face conductance run (a multiple of 4)
    KTailLevel lvl[kMaxTailLevels];
    int64_t top_aoff[kMaxLevelGrids];    // arena offsets of the top level's grids
    // Red-black slot table (grids with an even number of columns): per level,
    // one entry per pair of cells (2k, j), (2k+1, j) of every grid, holding the
    // LDS offsets of cell (2k, j), of its west x-face and of its south y-face,
    // and bits: nx (0-15), j odd (16), k first pair (17), k last pair (18),
    // j first row (19), j last row (20).  Built once per stage on the device;
    // null: the smoother decodes each slot itself.
    const int4* slots;
    int32_t slot_off[kMaxTailLevels];    // first entry of each level
    int32_t nslots;                      // entries of all levels 0..top
    int32_t zero;                        // LDS element holding 0: what a neighbour beyond a wall reads
    int32_t reg_levels;                  // levels 1..reg_levels keep their slot entries and reciprocal
                                         // diagonals in registers for the whole launch (0: none)
    int32_t first;                       // the class's first problem in the stage's problem table
    int64_t pack_off;                    // element offset of the class's conductance images in the
                                         // stage's image buffer (K * nstat elements, problem order)
};

struct KCosTable {
    int32_t n;
    int32_t a[kMaxCosTerms];
    int32_t b[kMaxCosTerms];
    double amp[kMaxCosTerms];
};

}  // namespace msg
