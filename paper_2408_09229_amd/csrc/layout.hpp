// Launch arguments and workspace records shared by the host library and the
// kernels.  Plain structs only (passed by value to kernels).
#pragma once
#include <stdint.h>

namespace vg {

constexpr int kMaxDim = 16;
constexpr int kFillThreads = 1024;     // one persistent workgroup per CU
constexpr int kLanesPerTile = kFillThreads;
// largest tile: the fill keeps the tile's cube starts in LDS as 16-bit
// offsets from the tile's first sample (plus one, clamped to tile + 2)
constexpr int kMaxTile = 32768;

// Partial moments of one hypercube's weights over a contiguous run of its
// samples: count, mean and sum of squared deviations (Chan et al. 1983 form,
// so that runs merge without cancellation).
struct Partial {
    uint32_t h;
    uint32_t n;
    double mean;
    double m2;
};

// Per-tile side record for cubes that cross tile boundaries.
enum : uint32_t { kHasHead = 1u, kHasTail = 2u, kSpan = 4u };
struct TileSide {
    Partial head;   // the tile's first cube, when it began in an earlier tile
    Partial tail;   // the tile's last cube, when it continues into a later tile
    uint32_t flags;
    uint32_t pad;
};

// Problem constants used by the per-sample path.
struct SampleConst {
    int32_t D;
    uint32_t ng;
    uint32_t nst;
    uint32_t nst_magic;
    int32_t nst_shift;         // -1: N_st = 1 (magic 2^31)
    uint32_t n_eval;
    uint32_t n_cubes;
    uint32_t key0, key1;       // Philox key = seed
    uint32_t ctr3;             // instance << 8 (counter word 3 high bits)
    int32_t family;
    int32_t n_params;
    const double* prm;         // raw parameters (device)
    const double* aux_d;       // derived constants, FP64 (device)
    const float* aux_f;        // derived constants, FP32 (device)
    int32_t n_aux;             // entries of aux_d / aux_f
};

struct FillArgs {
    SampleConst sc;
    uint32_t t;                 // iteration index (counter word 2)
    int32_t tile;               // samples per tile = kLanesPerTile * per_lane
    int32_t per_lane;
    int32_t n_tiles;
    int32_t lds_hist;           // 1: LDS histograms, 0: global FP64 atomics
    int32_t accum;              // VEGAS_ACC_*
    const void* grid;           // [D][N_g+1], FP64 or FP32 per precision
    const uint32_t* start;      // [N_c+1] first sample of each cube
    const uint32_t* tile_first; // [n_tiles+1] cube holding each tile's first sample
    double* v_out;              // [N_c] unbiased per-cube variance
    double* wg_part;            // [n_wg][2]: sum of cube means, sum of v/n
    TileSide* side;             // [n_tiles]
    double* hist_H;             // LDS mode or hist_slots: [n_wg][D*N_g]; else [D*N_g]
    uint32_t* hist_C;           // same layout
    double* hist_Cw;            // warped fill (global mode): [D*N_g] FP64 sums of J_F
    unsigned long long* vmax;   // max v_h as FP64 bits (v >= 0)
    unsigned long long* nonfinite;
    int32_t hist_slots;         // global mode: 1 = each workgroup adds into its own slot [n_wg][D*N_g]
};

struct FixupArgs {
    int32_t n_tiles;
    const TileSide* side;
    double* v_out;
    double* fix_part;           // [n_tiles][2]
    unsigned long long* vmax;
};

struct FinalArgs {
    int32_t n_wg;
    int32_t n_tiles;
    double n_cubes;
    const double* wg_part;
    const double* fix_part;
    double* iter_out;           // (I_t, sigma_t^2)
};

struct AllocArgs {
    uint32_t n_cubes;
    uint32_t n_min;
    uint64_t R;                 // N_ev - n_min N_c
    uint32_t n_eval;
    double beta;
    int32_t uniform;            // 1: Q_h = 1
    int32_t tile;
    int32_t tile_shift;         // tile = 2^tile_shift
    int32_t n_tiles;
    int32_t per_block;          // cubes per block
    const double* v;
    const unsigned long long* vmax;   // max v (monotone beta)
    double* qmax_buf;           // [n_blocks] block maxima of q (general beta)
    unsigned long long* bsum;   // [n_blocks] block sums of Q
    unsigned long long* boff;   // [n_blocks] exclusive offsets; boff[n_blocks] = T
    uint32_t* start;            // [N_c+1] out
    uint32_t* tile_first;       // [n_tiles+1] out
    uint32_t* qbuf;             // [N_c] Q_h saturated at 2^32-1 (null: recompute)
};

constexpr int kHistParts = 8;          // first-level slot groups of the histogram reduce

struct HistReduceArgs {
    int32_t nbins;              // D * N_g
    int32_t n_slots;
    int32_t parts;              // 1 .. kHistParts
    const double* hist_H;       // [n_slots][nbins]
    const uint32_t* hist_C;
    double* part_H;             // [parts][nbins]
    uint32_t* part_C;
};

struct MapArgs {
    int32_t D;
    int32_t ng;
    int32_t n_slots;            // partial histograms to add, in order
    int32_t parts;              // 0: add the slots in order; > 0: in `parts`
                                // consecutive groups, each in order, then the
                                // groups in order (what k_hist_reduce followed
                                // by a map over its groups adds)
    double alpha;
    const double* hist_H;       // [n_slots][D*N_g]
    const uint32_t* hist_C;
    const double* hist_Cw;      // non-null (one slot, parts 0): FP64 weights in place of hist_C
    double* grid64;             // [D][N_g+1] in/out
    float* grid32;              // [D][N_g+1] out (FP32 copy)
    double* Hsum;               // [D][N_g] reduced histogram (kept for inspection; may be null)
    double* Csum;
};

// The cube fix-up, the iteration estimate and the map refinement of a small
// problem (few tiles, few histogram slots) in one launch of D + 1
// workgroups: workgroup d < D refines axis d, workgroup D runs the fix-up and
// then the estimate.
struct UpdateArgs {
    FixupArgs fx;
    FinalArgs fin;
    MapArgs map;
};

// ---------------------------------------------------------------------------
// batched problems: many independent integrals advanced together
// ---------------------------------------------------------------------------
// Per-problem record (device), built by the host at create.
struct BatchInst {
    SampleConst sc;             // prm / aux point into the workspace
    double alpha, beta;
    uint64_t R;                 // N_ev - n_min N_c
    uint32_t n_min;
    int32_t adapt_strat;        // 0: the allocation stays uniform
    int32_t adapt_map;          // 0: the map stays as it is
    int32_t per_lane, tile, tile_shift, n_tiles;
    uint32_t tile0;             // first global tile
    uint32_t item0, n_items;    // its work items (consecutive)
    uint32_t blk0, n_blk;       // its allocation blocks (consecutive)
    const double* lo;           // [D] box
    const double* hi;
    double* grid64;             // [D][N_g+1]
    float* grid32;
    uint32_t* start[2];         // [N_c+1], double-buffered
    uint32_t* tfirst[2];        // [n_tiles+1]
    double* v;                  // [N_c]
    double* hist_H;             // [n_items][D*N_g]: one slot per work item
    uint32_t* hist_C;
    unsigned long long* bsum;   // [n_blk]
    unsigned long long* boff;   // [n_blk+1]
    unsigned long long* ctr;    // vmax[2], qmax[2] (FP64 bits, by iteration parity), non-finite count
    double* iter;               // [max_iter][2]: (I_t, sigma_t^2)
};

// A work item: consecutive tiles of one problem, the unit of the queue.
struct BatchItem {
    uint32_t inst;
    uint32_t tile0;             // first tile, local to the problem
    uint32_t n_tiles;
    uint32_t pad;
};

struct BatchArgs {
    int32_t n_inst;
    int32_t n_items;
    int32_t n_tiles;            // over all problems
    int32_t n_blk;
    int32_t n_axes;
    uint32_t t;                 // iteration (Philox counter word 2)
    int32_t cur;                // allocation buffer the fill reads
    int32_t force_uniform;      // 1: write the uniform allocation
    const BatchInst* inst;
    const BatchItem* items;     // problem order
    const uint32_t* order;      // queue order of the items (largest first)
    const uint32_t* tile_inst;  // [n_tiles] problem of each global tile
    const uint32_t* blk_inst;   // [n_blk] problem of each allocation block
    const uint32_t* axis_inst;  // [n_axes] problem << 4 | axis
    unsigned int* next;         // queue head
    double* item_part;          // [n_items][2]: sum of cube means, sum of v/n
    TileSide* side;             // [n_tiles]
    double* fix_part;           // [n_tiles][2]
    unsigned long long* nonfinite;
};

}  // namespace vg
