// Host-side context of a level, shared by the library's host sources.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <memory>
#include <set>
#include <string>
#include <vector>

#include "ppm.h"
#include "ppm_internal.h"

namespace ppm {
// The ghost-fill plan of a layout: copy descriptors grouped by destination
// box, with the exclusive prefix of their zone counts.
struct Plan {
  std::vector<FillDesc> desc;
  std::vector<long long> start;   // ndesc + 1
  std::vector<int> box_desc;      // nbox + 1: descriptor range of each destination box
};
// Rows per strip of the default tile order.
constexpr int STRIP_ROWS = 32;
}  // namespace ppm

using namespace ppm;

// ============================================================ context =====
// A level: box metadata, fill plan, tile lists and their device copies.
struct ppm_ctx {
  std::vector<ppm_box> boxes;
  ppm_layout layout{};
  std::vector<int64_t> off, foff[3];
  std::shared_ptr<const Plan> plan;
  bool plan_hit = false;
  std::vector<Tile> tilesS, tilesE;
  std::vector<int> tS_begin, tE_begin;  // nbox + 1
  std::vector<Tile> tilesX;             // front forms 2, 3: traced-grid runs of XF_OWNED zones
  std::vector<Tile> tilesXA;            // adjoint along x: traced-grid runs of XF_OWNED - 1 zones
  std::vector<int> tX_begin;            // nbox + 1
  std::vector<Tile> tilesY, tilesZ;     // front form 3: 8 x 8 wavefront patches (x-d planes) along y, z
  std::vector<int> tY_begin, tZ_begin;  // nbox + 1
  std::vector<Brick> bricks;
  std::vector<int> tB_begin;            // nbox + 1
  int fused = 0;                        // 1: final fluxes + update in one brick kernel; 2: streamed
  int stream_e[3] = {16, 8, 32};        // tile extents of the streamed final stage
  // front end: 0 trace and stage-1 solves as two staged kernels; 1 one
  // kernel streamed along z over x-y tiles of the traced grids (fbricks,
  // at most front_e zones per axis, balanced per box); 2 the x axis's trace
  // and solves in one kernel (tilesX), y and z staged; 3 each axis's trace
  // and solves in one kernel (tilesX, tilesY, tilesZ)
  int front = 2;
  int front_e[3] = {16, 8, 32};
  std::vector<Brick> fbricks;
  std::vector<int> tF_begin;            // nbox + 1
  int front_m[2] = {1, 1};              // largest x, y extents of the front tiles
  int device = -1;                      // HIP device current at ppm_ctx_create
  // Generation of the device state a captured graph bakes in (workspace,
  // tile lists, step form, inflow states): bumped whenever one changes; a
  // graph captured under another generation is refused at launch.
  unsigned long long gen = 1;
  std::set<ppm_graph*> graphs;          // live graphs captured on this context
  int tile = TILE, strip_rows = STRIP_ROWS;
  long long LS = 0, LE = 0;
  // device copies
  DevBox* d_boxes = nullptr;
  Tile* d_tilesS = nullptr;
  Tile* d_tilesE = nullptr;
  Tile* d_tilesX = nullptr;
  Tile* d_tilesXA = nullptr;
  Tile* d_tilesY = nullptr;
  Tile* d_tilesZ = nullptr;
  Brick* d_bricks = nullptr;
  Brick* d_fbricks = nullptr;
  FillDesc* d_desc = nullptr;
  long long* d_start = nullptr;
  int* d_inv_start = nullptr;
  int* d_inv_idx = nullptr;
  void* awork = nullptr;
  size_t awork_bytes = 0;
  void* swork = nullptr;
  size_t swork_bytes = 0;
  const double* inflow[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // ppm_set_inflow
  StepConsts* d_consts = nullptr;
  int* d_flags = nullptr;
  void* work = nullptr;
  size_t work_bytes = 0;
  std::string err;
  // stage timing with HIP events (ppm_profile_enable / ppm_profile_read)
  struct ProfRec {
    int tag0, n;
    std::array<hipEvent_t, STEP_EVENTS> ev;
  };
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<std::array<hipEvent_t, STEP_EVENTS>> pool;

  // An event set for a record of n events starting at stage tag tag0.
  ProfRec* begin_rec(int tag0, int n) {
    std::array<hipEvent_t, STEP_EVENTS> ev{};
    if (!pool.empty()) {
      ev = pool.back();
      pool.pop_back();
    } else {
      for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
    }
    recs.push_back(ProfRec{tag0, n, ev});
    return &recs.back();
  }

  DevLevel level() const {
    DevLevel L;
    L.boxes = d_boxes;
    L.tilesS = d_tilesS;
    L.tilesE = d_tilesE;
    L.tilesX = d_tilesX;
    L.tilesXA = d_tilesXA;
    L.tilesY = d_tilesY;
    L.tilesZ = d_tilesZ;
    L.desc = d_desc;
    L.desc_start = d_start;
    L.consts = d_consts;
    L.flags = d_flags;
    L.inv_start = d_inv_start;
    L.inv_idx = d_inv_idx;
    L.LS = LS;
    L.LE = LE;
    L.tile = tile;
    for (int f = 0; f < 6; ++f) L.inflow.p[f] = inflow[f];
    for (int d = 0; d < 3; ++d) L.inflow.ext[d] = layout.domain.hi[d] - layout.domain.lo[d] + 1;
    L.bricks = d_bricks;
    L.fused = fused;
    for (int d = 0; d < 3; ++d) L.stream_e[d] = stream_e[d];
    L.fbricks = d_fbricks;
    L.front = front;
    L.front_m[0] = front_m[0];
    L.front_m[1] = front_m[1];
    return L;
  }
  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return PPM_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return PPM_EHIP;
  }
};

