// Batched persistent launches: the system table, per-launch operands and
// the batch object shared by batch.hip (launches) and solver.hip (batched
// CG).
#pragma once

#include <vector>

#include "common.h"

namespace tomo {

constexpr int kMaxSys = 32;   // systems per batch
constexpr int kQueues = 8;    // one work queue per XCD

struct SysDev {
    GridDev grid;
    const ViewDev *views;
    const int32_t *frame_views;
    const int32_t *frame_voff;
    const uint8_t *map_mask;
    const uint8_t *data_mask;
    float *part;          // owner partials [splits][ntot] (splits > 1)
    uint16_t *kept_pre;   // kept-pixel rows of the data mask (row intervals only), or null
    uint16_t *kept_cols;
    float *bricked;       // P's bricked copy of M x (the system's tuning asks for bricks), or null
    RayTable tab;         // the system's ray table (tab.d null: P^T sets its rays up)
    BrickDev bk;
    BlockDev bd;
    int32_t nviews;
    int32_t p_log2_bw;
    int32_t maxit;
    int32_t view_begin;   // first row of this system in the max|y| table
    int64_t tile_begin;   // first P item
    int64_t item_begin;   // first P^T item
    int64_t ntot;         // voxels over all frames
};

// Per-launch operands, passed by value (no upload, graph-capture safe).
struct Operands {
    const float *src[kMaxSys];
    float *dst[kMaxSys];
    const int *done[kMaxSys];
    int32_t map;          // apply the map mask (P M x / M P^T y)
    int32_t acc;          // P^T: add into dst
};

int batch_project_ops(tomo_batch b, const Operands &ops, hipStream_t s);
int batch_backproject_ops(tomo_batch b, const Operands &ops, hipStream_t s);

}  // namespace tomo

struct tomo_batch_s {
    int device = 0;
    int32_t nsys = 0;
    std::vector<tomo::PlanRef> plans;
    std::vector<tomo_tuning> tunings;  // each system's tuning at creation (its P launch shape and layout)
    std::vector<tomo_geometry> geoms;  // headers (views and obstacle unused after planning)
    std::vector<tomo::SysDev> sys_h;
    tomo::SysDev *sys_d = nullptr;
    int64_t ntiles = 0, nitems = 0;
    int32_t nviews = 0;
    unsigned long long *q = nullptr;   // [kQueues + 1]: P^T work queues, then the leave counter
    uint32_t *ymax = nullptr;
    float *part = nullptr;
    unsigned *spill = nullptr;
    size_t lds_bytes = 0;
    unsigned grid_p = 0, grid_b = 0;
    bool rows = false;  // P^T walks footprint row intervals (most systems' plans ask for them)
    int32_t nt = 256;   // lanes per workgroup of the persistent P^T (the dominant system's tuning)
    uint16_t *kept = nullptr;  // kept-pixel rows of the systems' data masks
    float *bricks = nullptr;   // bricked copies of the cubes of the systems that walk bricks in P
    char *tables = nullptr;    // ray tables of the systems whose tuning asks for one
    ~tomo_batch_s();
};
