// Host side of the library: level context, ghost-fill plan (hash-sorted box
// intersections with a plan cache), tile lists, the C ABI of ppm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <list>
#include <map>
#include <mutex>
#include <sstream>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ppm_ctx.h"

using namespace ppm;

namespace {

struct IBox {
  int lo[3], hi[3];
};


struct LayoutKey {
  std::vector<int> v;  // nbox, boxes, domain, bc, ngrow
  size_t hash = 0;
  bool operator==(const LayoutKey& o) const { return hash == o.hash && v == o.v; }
};

LayoutKey make_key(const ppm_layout& L) {
  LayoutKey k;
  k.v.push_back(L.nbox);
  for (int b = 0; b < L.nbox; ++b)
    for (int d = 0; d < 3; ++d) { k.v.push_back(L.boxes[b].lo[d]); k.v.push_back(L.boxes[b].hi[d]); }
  for (int d = 0; d < 3; ++d) { k.v.push_back(L.domain.lo[d]); k.v.push_back(L.domain.hi[d]); }
  for (int f = 0; f < 6; ++f) k.v.push_back(L.bc[f]);
  k.v.push_back(L.ngrow);
  size_t h = 1469598103934665603ull;  // FNV-1a over the words
  for (int x : k.v) { h ^= (size_t)(unsigned)x; h *= 1099511628211ull; }
  k.hash = h;
  return k;
}

// -------------------------------------------------------- validation -------
std::string validate_layout(const ppm_layout& L) {
  if (L.nbox < 1 || !L.boxes) return "layout: no boxes";
  if (L.ngrow != NG) return "layout: ngrow must be 4";
  long long dvol = 1;
  int ext[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = L.domain.hi[d] - L.domain.lo[d] + 1;
    if (ext[d] < NG) return "layout: domain extent below the ghost width";
    dvol *= ext[d];
    const bool pl = L.bc[2 * d] == PPM_BC_PERIODIC, ph = L.bc[2 * d + 1] == PPM_BC_PERIODIC;
    if (pl != ph) return "layout: a periodic axis needs both faces periodic";
    for (int s = 0; s < 2; ++s)
      if (L.bc[2 * d + s] < 0 || L.bc[2 * d + s] > PPM_BC_INFLOW) return "layout: unknown boundary code";
  }
  int ninflow = 0;
  for (int f = 0; f < 6; ++f) ninflow += L.bc[f] == PPM_BC_INFLOW;
  if (ninflow > 1) return "layout: at most one inflow face";
  long long vol = 0;
  for (int b = 0; b < L.nbox; ++b) {
    long long v = 1;
    for (int d = 0; d < 3; ++d) {
      const int n = L.boxes[b].hi[d] - L.boxes[b].lo[d] + 1;
      if (n < 1) return "layout: empty box";
      if (L.boxes[b].lo[d] < L.domain.lo[d] || L.boxes[b].hi[d] > L.domain.hi[d])
        return "layout: box outside the domain";
      v *= n;
    }
    // zone indices within a box (ghost layers included) are decoded in
    // 32 bits by multiply-and-shift, exact below 2^31
    long long stored = 1;
    for (int d = 0; d < 3; ++d) stored *= (long long)(L.boxes[b].hi[d] - L.boxes[b].lo[d] + 1 + 2 * NG);
    if (stored >= (1ll << 31)) return "layout: a box holds 2^31 zones or more with its ghost layers";
    vol += v;
  }
  if (vol != dvol) return "layout: boxes do not tile the domain (volume mismatch)";
  // disjointness through a painted ownership map of the domain
  std::vector<int> own((size_t)dvol, -1);
  for (int b = 0; b < L.nbox; ++b) {
    const ppm_box& B = L.boxes[b];
    for (int z = B.lo[2]; z <= B.hi[2]; ++z)
      for (int y = B.lo[1]; y <= B.hi[1]; ++y)
        for (int x = B.lo[0]; x <= B.hi[0]; ++x) {
          const size_t i = ((size_t)(z - L.domain.lo[2]) * ext[1] + (y - L.domain.lo[1])) * ext[0] +
                           (x - L.domain.lo[0]);
          if (own[i] >= 0) return "layout: boxes overlap";
          own[i] = b;
        }
  }
  return "";
}

// ---------------------------------------------------- plan construction ----
// Intersections of ghost regions with boxes (paper Sec. 2).  The domain is
// cut into M rectangular bins at least one box wide per axis; every box is
// sorted into the bin of its lowest corner, so a box extends no further than
// the next bin up.  A query region then only looks at the bins from one
// below its low corner to its high corner: O(N + N^2/M) for all queries
// instead of O(N^2) all-pairs.
struct Binner {
  int dlo[3], ext[3], bs[3], nb[3], maxext[3];
  std::vector<std::vector<int>> bins;
  const ppm_layout* L;
  bool brute;

  Binner(const ppm_layout& lay, bool brute_force) : L(&lay), brute(brute_force) {
    for (int d = 0; d < 3; ++d) {
      dlo[d] = lay.domain.lo[d];
      ext[d] = lay.domain.hi[d] - lay.domain.lo[d] + 1;
      maxext[d] = 1;
      for (int b = 0; b < lay.nbox; ++b)
        maxext[d] = std::max(maxext[d], lay.boxes[b].hi[d] - lay.boxes[b].lo[d] + 1);
      bs[d] = maxext[d];
      nb[d] = (ext[d] + bs[d] - 1) / bs[d];
    }
    bins.assign((size_t)nb[0] * nb[1] * nb[2], {});
    for (int b = 0; b < lay.nbox; ++b) {
      int k[3];
      for (int d = 0; d < 3; ++d) k[d] = (lay.boxes[b].lo[d] - dlo[d]) / bs[d];
      bins[((size_t)k[2] * nb[1] + k[1]) * nb[0] + k[0]].push_back(b);
    }
  }

  // Boxes intersecting the global region q (inside the domain), in box order.
  void query(const IBox& q, std::vector<int>& out) const {
    out.clear();
    auto hit = [&](int b) {
      const ppm_box& B = L->boxes[b];
      for (int d = 0; d < 3; ++d)
        if (B.hi[d] < q.lo[d] || B.lo[d] > q.hi[d]) return false;
      return true;
    };
    if (brute) {
      for (int b = 0; b < L->nbox; ++b)
        if (hit(b)) out.push_back(b);
      return;
    }
    int k0[3], k1[3];
    for (int d = 0; d < 3; ++d) {
      k0[d] = std::max(0, (std::max(q.lo[d] - maxext[d] + 1, dlo[d]) - dlo[d]) / bs[d]);
      k1[d] = std::min(nb[d] - 1, (q.hi[d] - dlo[d]) / bs[d]);
    }
    for (int z = k0[2]; z <= k1[2]; ++z)
      for (int y = k0[1]; y <= k1[1]; ++y)
        for (int x = k0[0]; x <= k1[0]; ++x)
          for (int b : bins[((size_t)z * nb[1] + y) * nb[0] + x])
            if (hit(b)) out.push_back(b);
    std::sort(out.begin(), out.end());
  }
};

Plan build_plan(const ppm_layout& L, bool brute) {
  Plan P;
  Binner bin(L, brute);
  int dlo[3], dhi[3], ext[3];
  for (int d = 0; d < 3; ++d) {
    dlo[d] = L.domain.lo[d];
    dhi[d] = L.domain.hi[d];
    ext[d] = dhi[d] - dlo[d] + 1;
  }
  std::vector<int> found;
  P.box_desc.push_back(0);
  for (int b = 0; b < L.nbox; ++b) {
    const ppm_box& B = L.boxes[b];
    int n[3];
    for (int d = 0; d < 3; ++d) n[d] = B.hi[d] - B.lo[d] + 1;
    // 26 ghost sub-regions of the grown box (box-local), each cut at the
    // domain faces into pieces wholly inside or wholly outside the domain.
    for (int sz = -1; sz <= 1; ++sz)
      for (int sy = -1; sy <= 1; ++sy)
        for (int sx = -1; sx <= 1; ++sx) {
          if (sx == 0 && sy == 0 && sz == 0) continue;
          const int s[3] = {sx, sy, sz};
          // per axis: up to 3 pieces [a, b] in global coordinates + their map
          struct Piece { int lo, hi, a, c, refl, inflow; };  // inflow: face index or -1
          std::vector<Piece> pcs[3];
          for (int d = 0; d < 3; ++d) {
            int l, h;
            if (s[d] < 0) { l = -NG; h = -1; }
            else if (s[d] == 0) { l = 0; h = n[d] - 1; }
            else { l = n[d]; h = n[d] + NG - 1; }
            l += B.lo[d];
            h += B.lo[d];
            const int cuts[4] = {l, std::max(l, dlo[d]), std::min(h, dhi[d]) + 1, h + 1};
            // below the domain (nothing beyond a coarse-fine face: the
            // two-level advance interpolates those ghost zones)
            if (cuts[0] < cuts[1] && L.bc[2 * d] != PPM_BC_COARSE_FINE) {
              const int bc = L.bc[2 * d];
              Piece pc{cuts[0], std::min(cuts[1] - 1, h), 1, 0, 0, -1};
              if (bc == PPM_BC_PERIODIC) { pc.a = 1; pc.c = ext[d]; }
              else if (bc == PPM_BC_OUTFLOW) { pc.a = 0; pc.c = dlo[d]; }
              else if (bc == PPM_BC_INFLOW) { pc.a = 0; pc.c = dlo[d]; pc.inflow = 2 * d; }
              else { pc.a = -1; pc.c = 2 * dlo[d] - 1; pc.refl = 1; }
              pcs[d].push_back(pc);
            }
            if (cuts[1] < cuts[2]) pcs[d].push_back(Piece{cuts[1], cuts[2] - 1, 1, 0, 0, -1});
            if (cuts[2] < cuts[3] && L.bc[2 * d + 1] != PPM_BC_COARSE_FINE) {
              const int bc = L.bc[2 * d + 1];
              Piece pc{std::max(cuts[2], l), cuts[3] - 1, 1, 0, 0, -1};
              if (bc == PPM_BC_PERIODIC) { pc.a = 1; pc.c = -ext[d]; }
              else if (bc == PPM_BC_OUTFLOW) { pc.a = 0; pc.c = dhi[d]; }
              else if (bc == PPM_BC_INFLOW) { pc.a = 0; pc.c = dhi[d]; pc.inflow = 2 * d + 1; }
              else { pc.a = -1; pc.c = 2 * dhi[d] + 1; pc.refl = 1; }
              pcs[d].push_back(pc);
            }
          }
          for (const Piece& px : pcs[0])
            for (const Piece& py : pcs[1])
              for (const Piece& pz : pcs[2]) {
                const Piece* pp[3] = {&px, &py, &pz};
                int inface = -1;
                for (int d = 0; d < 3; ++d)
                  if (pp[d]->inflow >= 0) inface = pp[d]->inflow;
                if (inface >= 0) {
                  // beyond the inflow face: the face's prescribed state at the
                  // domain-relative image of the transverse coordinates
                  FillDesc D;
                  D.dst = b;
                  D.src = -1 - inface;
                  D.sign = 0;
                  long long cnt = 1;
                  for (int d = 0; d < 3; ++d) {
                    const Piece& q = *pp[d];
                    D.lo[d] = q.lo - B.lo[d];
                    D.hi[d] = q.hi - B.lo[d];
                    if (d == inface / 2) {
                      D.a[d] = 0;
                      D.c[d] = 0;
                    } else {
                      D.a[d] = q.a;
                      D.c[d] = q.a * B.lo[d] + q.c - dlo[d];
                      if (q.refl) D.sign |= 1 << d;
                    }
                    cnt *= (q.hi - q.lo + 1);
                  }
                  D.count = (int)cnt;
                  P.desc.push_back(D);
                  continue;
                }
                IBox img;
                for (int d = 0; d < 3; ++d) {
                  const Piece& q = *pp[d];
                  if (q.a == 1) { img.lo[d] = q.lo + q.c; img.hi[d] = q.hi + q.c; }
                  else if (q.a == -1) { img.lo[d] = q.c - q.hi; img.hi[d] = q.c - q.lo; }
                  else { img.lo[d] = q.c; img.hi[d] = q.c; }
                }
                bin.query(img, found);
                for (int sb : found) {
                  const ppm_box& S = L.boxes[sb];
                  FillDesc D;
                  D.dst = b;
                  D.src = sb;
                  D.sign = 0;
                  long long cnt = 1;
                  for (int d = 0; d < 3; ++d) {
                    const Piece& q = *pp[d];
                    const int jl = std::max(img.lo[d], S.lo[d]), jh = std::min(img.hi[d], S.hi[d]);
                    int gl, gh;
                    if (q.a == 1) { gl = jl - q.c; gh = jh - q.c; }
                    else if (q.a == -1) { gl = q.c - jh; gh = q.c - jl; }
                    else { gl = q.lo; gh = q.hi; }
                    D.lo[d] = gl - B.lo[d];
                    D.hi[d] = gh - B.lo[d];
                    D.a[d] = q.a;
                    // src_local = a * dst_local + (a * lo_dst + c - lo_src)
                    D.c[d] = q.a * B.lo[d] + q.c - S.lo[d];
                    if (q.refl) D.sign |= 1 << d;
                    cnt *= (gh - gl + 1);
                  }
                  D.count = (int)cnt;
                  P.desc.push_back(D);
                }
              }
        }
    P.box_desc.push_back((int)P.desc.size());
  }
  P.start.resize(P.desc.size() + 1);
  P.start[0] = 0;
  for (size_t k = 0; k < P.desc.size(); ++k) P.start[k + 1] = P.start[k] + P.desc[k].count;
  return P;
}

// Cache of fill plans keyed by the layout (paper Sec. 2: frequently used
// communication patterns are kept).  Least-recently-used eviction.
struct PlanCache {
  std::mutex mu;
  std::list<std::pair<LayoutKey, std::shared_ptr<const Plan>>> lru;
  size_t cap = 16;
  long long lookups = 0, hits = 0;

  std::shared_ptr<const Plan> get(const ppm_layout& L, bool& hit) {
    LayoutKey k = make_key(L);
    std::lock_guard<std::mutex> g(mu);
    ++lookups;
    for (auto it = lru.begin(); it != lru.end(); ++it)
      if (it->first == k) {
        ++hits;
        hit = true;
        lru.splice(lru.begin(), lru, it);
        return lru.front().second;
      }
    hit = false;
    auto p = std::make_shared<const Plan>(build_plan(L, false));
    lru.emplace_front(std::move(k), p);
    if (lru.size() > cap) lru.pop_back();
    return p;
  }
};
PlanCache& plan_cache() {
  static PlanCache c;
  return c;
}

long long round_up(long long x, long long m) { return (x + m - 1) / m * m; }

// Tiles of `tile` consecutive linear zones of one box's grid (extents
// e0 x e1 x e2, x fastest), appended in strip order: the planes are cut into
// strips of `strip_rows` rows and each strip is walked through all planes
// before the next, so the z-neighbours of a tile were visited a few tiles
// earlier and are still in the XCD's L2 (strip_rows = 0: plane by plane).
void add_tiles(std::vector<Tile>& out, int b, int e0, int e1, int e2, int tile, int strip_rows) {
  const long long plane = (long long)e0 * e1, tot = plane * e2;
  const long long strip = strip_rows > 0 ? (long long)strip_rows * e0 : plane;
  std::vector<std::pair<std::pair<long long, long long>, long long>> keyed;
  for (long long s = 0; s < tot; s += tile) {
    const long long k = s / plane, off = s % plane;
    keyed.push_back({{off / strip, k}, s});
  }
  std::stable_sort(keyed.begin(), keyed.end(),
                   [](const auto& a, const auto& c) { return a.first < c.first; });
  for (const auto& kv : keyed) {
    const long long s = kv.second;
    out.push_back(Tile{b, (int)s, (int)std::min(s + tile, tot)});
  }
}

}  // namespace

struct ppm_graph {
  ppm_ctx* ctx = nullptr;          // null once the context is destroyed
  unsigned long long gen = 0;      // the context's generation at capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double* dtv = nullptr;  // device [dt, max signal speed] of the step being replayed
};

namespace {
// Blocks of valid zones per box for the fused final stage, x fastest then y
// then z: bricks of at most BRICK_E zones (form 1) or the streamed form's
// tiles of stream_e (form 2).
void build_bricks(ppm_ctx& c) {
  c.bricks.clear();
  c.tB_begin.assign(1, 0);
  const int* E = c.fused == 2 ? c.stream_e : BRICK_E;
  for (int b = 0; b < c.layout.nbox; ++b) {
    int n[3];
    for (int d = 0; d < 3; ++d) n[d] = c.boxes[b].hi[d] - c.boxes[b].lo[d] + 1;
    for (int z = 0; z < n[2]; z += E[2])
      for (int y = 0; y < n[1]; y += E[1])
        for (int x = 0; x < n[0]; x += E[0]) {
          Brick K;
          K.box = b;
          const int o[3] = {x, y, z};
          for (int d = 0; d < 3; ++d) {
            K.o[d] = o[d];
            K.e[d] = std::min(E[d], n[d] - o[d]);
          }
          brick_divisors(K);
          c.bricks.push_back(K);
        }
    c.tB_begin.push_back((int)c.bricks.size());
  }
}


// Tiles of the streamed front end: per box, the traced grid (zones -1..n
// per axis) cut into x-y tiles of at most front_e[0] x front_e[1] zones and
// z runs of at most front_e[2] planes, the pieces along each axis as even
// as possible (so no tile is a thin remainder).
void build_front(ppm_ctx& c) {
  c.fbricks.clear();
  c.tF_begin.assign(1, 0);
  c.front_m[0] = c.front_m[1] = 1;
  for (int b = 0; b < c.layout.nbox; ++b) {
    std::vector<int> org[3], ext[3];
    for (int d = 0; d < 3; ++d) {
      const int E = c.boxes[b].hi[d] - c.boxes[b].lo[d] + 3;
      const int k = (E + c.front_e[d] - 1) / c.front_e[d];
      int o = -1;
      for (int p = 0; p < k; ++p) {
        const int e = E / k + (p < E % k ? 1 : 0);
        org[d].push_back(o);
        ext[d].push_back(e);
        o += e;
      }
    }
    for (size_t z = 0; z < org[2].size(); ++z)
      for (size_t y = 0; y < org[1].size(); ++y)
        for (size_t x = 0; x < org[0].size(); ++x) {
          Brick K;
          K.box = b;
          K.o[0] = org[0][x];
          K.o[1] = org[1][y];
          K.o[2] = org[2][z];
          K.e[0] = ext[0][x];
          K.e[1] = ext[1][y];
          K.e[2] = ext[2][z];
          c.front_m[0] = std::max(c.front_m[0], K.e[0]);
          c.front_m[1] = std::max(c.front_m[1], K.e[1]);
          brick_divisors(K);
          c.fbricks.push_back(K);
        }
    c.tF_begin.push_back((int)c.fbricks.size());
  }
}

// The whole level's ranges of the fused front end's work lists.
FrontRanges front_all(const ppm_ctx& c) {
  return FrontRanges{0, (int)c.tilesX.size(), 0, (int)c.tilesY.size(), 0, (int)c.tilesZ.size()};
}

void build_tiles(ppm_ctx& c) {
  c.tilesS.clear();
  c.tilesE.clear();
  c.tS_begin.assign(1, 0);
  c.tE_begin.assign(1, 0);
  c.tilesX.clear();
  c.tilesXA.clear();
  c.tX_begin.assign(1, 0);
  c.tilesY.clear();
  c.tY_begin.assign(1, 0);
  c.tilesZ.clear();
  c.tZ_begin.assign(1, 0);
  for (int b = 0; b < c.layout.nbox; ++b) {
    int n[3];
    for (int d = 0; d < 3; ++d) n[d] = c.boxes[b].hi[d] - c.boxes[b].lo[d] + 1;
    add_tiles(c.tilesS, b, n[0] + 2 * NG, n[1] + 2 * NG, n[2] + 2 * NG, c.tile, c.strip_rows);
    add_tiles(c.tilesE, b, n[0] + 2, n[1] + 2, n[2] + 2, c.tile, c.strip_rows);
    add_tiles(c.tilesX, b, n[0] + 2, n[1] + 2, n[2] + 2, XF_OWNED, c.strip_rows);
    add_tiles(c.tilesXA, b, n[0] + 2, n[1] + 2, n[2] + 2, XF_OWNED - 1, c.strip_rows);
    // front form 3: workgroup w of a box along y or z; the kernel decodes w
    for (long long w = 0; w < front_yz_groups(n[0] + 2, n[1] + 2, n[2] + 2); ++w)
      c.tilesY.push_back(Tile{b, (int)w, (int)w + 1});
    for (long long w = 0; w < front_yz_groups(n[0] + 2, n[2] + 2, n[1] + 2); ++w)
      c.tilesZ.push_back(Tile{b, (int)w, (int)w + 1});
    c.tS_begin.push_back((int)c.tilesS.size());
    c.tE_begin.push_back((int)c.tilesE.size());
    c.tX_begin.push_back((int)c.tilesX.size());
    c.tY_begin.push_back((int)c.tilesY.size());
    c.tZ_begin.push_back((int)c.tilesZ.size());
  }
}

template <class T> hipError_t upload(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  hipError_t e = hipMalloc((void**)dst, bytes);
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

// Rebuilds and uploads the block list of the current final-stage form.
hipError_t upload_front(ppm_ctx& c) {
  build_front(c);
  (void)hipFree(c.d_fbricks);
  c.d_fbricks = nullptr;
  return upload(&c.d_fbricks, c.fbricks);
}

hipError_t upload_bricks(ppm_ctx& c) {
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  build_bricks(c);
  (void)hipFree(c.d_bricks);
  c.d_bricks = nullptr;
  return upload(&c.d_bricks, c.bricks);
}

std::string validate_params(const ppm_params* p) {
  if (!p) return "params: null";
  if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return "params: gamma must be > 1";
  if (!(p->small_dens >= 0x1p-120 && p->small_dens <= 0x1p120) ||
      !(p->small_pres >= 0x1p-120 && p->small_pres <= 0x1p120))
    return "params: floors must lie in [2^-120, 2^120]";
  if (p->riemann_iters < 0 || p->riemann_iters > 16) return "params: riemann_iters must be in [0, 16]";
  if (p->precision != 0 && p->precision != 1) return "params: precision must be 0 or 1";
  if ((p->limiter != 0 && p->limiter != 1) || (p->flattening != 0 && p->flattening != 1))
    return "params: limiter/flattening must be 0 or 1";
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(p->grav[d])) return "params: gravity must be finite";
  return "";
}

std::string validate_dx(const double dx[3]) {
  if (!dx) return "dx: null";
  for (int d = 0; d < 3; ++d)
    if (!(dx[d] > 0.0) || !std::isfinite(dx[d])) return "dx: spacings must be positive and finite";
  return "";
}
// Step scratch of the allocation-free step (ppm_hydro_step_noalloc): a
// file-scope device array of PPM_NOALLOC_SCRATCH_BYTES, one copy per GPU
// for the life of the process.  In host code `scratch` only names the
// symbol; its device address on each GPU comes from hipGetSymbolAddress,
// taken once per device (with that device current) when the first context
// is created there, and only that address is passed to kernels.
__attribute__((used)) static __device__ __align__(256) unsigned char scratch[PPM_NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};

// Records the scratch address of device `dev` (the current device).
void scratch_setup(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) g_scratch_ptr[dev] = ptr;
  else g_scratch_err[dev] = (e == hipSuccess) ? hipErrorInvalidSymbol : e;
}

void* scratch_ptr(int dev, hipError_t* err) {
  if (dev < 0 || dev >= MAX_DEVICES) { *err = hipErrorInvalidDevice; return nullptr; }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

int ppm_ctx_create(const ppm_layout* layout, ppm_ctx** out) {
  if (!layout || !out) return PPM_EINVAL;
  *out = nullptr;
  std::string msg = validate_layout(*layout);
  if (!msg.empty()) {
    std::fprintf(stderr, "ppm_ctx_create: %s\n", msg.c_str());
    return PPM_EINVAL;
  }
  auto ctx = std::make_unique<ppm_ctx>();
  ctx->boxes.assign(layout->boxes, layout->boxes + layout->nbox);
  ctx->layout = *layout;
  ctx->layout.boxes = ctx->boxes.data();
  const int nb = layout->nbox;
  ctx->plan = plan_cache().get(ctx->layout, ctx->plan_hit);

  std::vector<DevBox> db(nb);
  ctx->off.assign(nb + 1, 0);
  for (int d = 0; d < 3; ++d) ctx->foff[d].assign(nb + 1, 0);
  long long ps = 0, pe = 0;
  for (int b = 0; b < nb; ++b) {
    int n[3];
    for (int d = 0; d < 3; ++d) n[d] = layout->boxes[b].hi[d] - layout->boxes[b].lo[d] + 1;
    const long long NS = (long long)(n[0] + 2 * NG) * (n[1] + 2 * NG) * (n[2] + 2 * NG);
    const long long NE = (long long)(n[0] + 2) * (n[1] + 2) * (n[2] + 2);
    for (int d = 0; d < 3; ++d) db[b].n[d] = n[d];
    for (int d = 0; d < 2; ++d) {
      db[b].de[d] = make_div31((unsigned)(n[d] + 2));
      db[b].ds[d] = make_div31((unsigned)(n[d] + 2 * NG));
    }
    db[b].wall = 0;
    for (int d = 0; d < 3; ++d) {
      if (layout->boxes[b].lo[d] == layout->domain.lo[d] && layout->bc[2 * d] == PPM_BC_REFLECT)
        db[b].wall |= 1 << (2 * d);
      if (layout->boxes[b].hi[d] == layout->domain.hi[d] && layout->bc[2 * d + 1] == PPM_BC_REFLECT)
        db[b].wall |= 1 << (2 * d + 1);
    }
    db[b].soff = ctx->off[b];
    db[b].poff = ps;
    db[b].eoff = pe;
    ctx->off[b + 1] = ctx->off[b] + 5 * NS;
    for (int d = 0; d < 3; ++d) {
      long long fe = 5;
      for (int e = 0; e < 3; ++e) fe *= n[e] + (e == d ? 1 : 0);
      db[b].foff[d] = ctx->foff[d][b];
      ctx->foff[d][b + 1] = ctx->foff[d][b] + fe;
    }
    ps += NS;
    pe += NE;
  }
  ctx->LS = round_up(ps, 64);
  ctx->LE = round_up(pe, 64);

  // inverse of the fill plan: for every source box and zone class (per axis:
  // within NG of the low face, of the high face, of both or of neither) the
  // descriptors that can copy a zone of that class, in plan order
  std::vector<int> inv_start((size_t)nb * INV_CLASSES + 1, 0), inv_idx;
  {
    const std::vector<FillDesc>& desc = ctx->plan->desc;
    std::vector<unsigned long long> cmask(desc.size(), 0);  // bit per class
    for (size_t k = 0; k < desc.size(); ++k) {
      const FillDesc& D = desc[k];
      if (D.src < 0) continue;  // prescribed inflow state: no adjoint flows back
      const int* ns = layout->boxes[D.src].lo;
      unsigned axm[3];
      for (int d = 0; d < 3; ++d) {
        const int n = layout->boxes[D.src].hi[d] - ns[d] + 1;
        int y0, y1;
        if (D.a[d] == 1) { y0 = D.lo[d] + D.c[d]; y1 = D.hi[d] + D.c[d]; }
        else if (D.a[d] == -1) { y0 = D.c[d] - D.hi[d]; y1 = D.c[d] - D.lo[d]; }
        else { y0 = y1 = D.c[d]; }
        axm[d] = 0;
        for (int y = std::max(y0, 0); y <= std::min(y1, n - 1); ++y) axm[d] |= 1u << inv_axis_class(y, n);
      }
      for (int c = 0; c < INV_CLASSES; ++c)
        if ((axm[0] >> (c & 3) & 1) && (axm[1] >> ((c >> 2) & 3) & 1) && (axm[2] >> (c >> 4) & 1))
          cmask[k] |= 1ull << c;
    }
    for (size_t k = 0; k < desc.size(); ++k)
      for (int c = 0; c < INV_CLASSES; ++c)
        if (cmask[k] >> c & 1) inv_start[(size_t)desc[k].src * INV_CLASSES + c + 1]++;
    for (size_t i = 0; i + 1 < inv_start.size(); ++i) inv_start[i + 1] += inv_start[i];
    inv_idx.assign(inv_start.back(), 0);
    std::vector<int> fillp(inv_start.begin(), inv_start.end() - 1);
    for (size_t k = 0; k < desc.size(); ++k)
      for (int c = 0; c < INV_CLASSES; ++c)
        if (cmask[k] >> c & 1) inv_idx[fillp[(size_t)desc[k].src * INV_CLASSES + c]++] = (int)k;
  }
  build_tiles(*ctx);
  build_bricks(*ctx);
  build_front(*ctx);
  hipError_t e;
  if ((e = upload(&ctx->d_bricks, ctx->bricks)) != hipSuccess ||
      (e = upload(&ctx->d_fbricks, ctx->fbricks)) != hipSuccess ||
      (e = upload(&ctx->d_inv_start, inv_start)) != hipSuccess ||
      (e = upload(&ctx->d_inv_idx, inv_idx)) != hipSuccess ||
      (e = upload(&ctx->d_boxes, db)) != hipSuccess ||
      (e = upload(&ctx->d_tilesS, ctx->tilesS)) != hipSuccess ||
      (e = upload(&ctx->d_tilesE, ctx->tilesE)) != hipSuccess ||
      (e = upload(&ctx->d_tilesX, ctx->tilesX)) != hipSuccess ||
      (e = upload(&ctx->d_tilesXA, ctx->tilesXA)) != hipSuccess ||
      (e = upload(&ctx->d_tilesY, ctx->tilesY)) != hipSuccess ||
      (e = upload(&ctx->d_tilesZ, ctx->tilesZ)) != hipSuccess ||
      (e = upload(&ctx->d_desc, ctx->plan->desc)) != hipSuccess ||
      (e = upload(&ctx->d_start, ctx->plan->start)) != hipSuccess ||
      (e = hipMalloc((void**)&ctx->d_consts, sizeof(StepConsts))) != hipSuccess ||
      (e = hipMalloc((void**)&ctx->d_flags, 256)) != hipSuccess ||
      (e = hipMemset(ctx->d_flags, 0, 256)) != hipSuccess ||
      (e = hipMemset(ctx->d_consts, 0, sizeof(StepConsts))) != hipSuccess ||
      (e = hipGetDevice(&ctx->device)) != hipSuccess) {
    std::fprintf(stderr, "ppm_ctx_create: %s\n", hipGetErrorString(e));
    ppm_ctx_destroy(ctx.release());
    return PPM_EHIP;
  }
  scratch_setup(ctx->device);
  *out = ctx.release();
  return PPM_OK;
}

int ppm_ctx_destroy(ppm_ctx* ctx) {
  if (!ctx) return PPM_OK;
  for (ppm_graph* g : ctx->graphs) g->ctx = nullptr;  // their launches are refused from now on
  for (auto& r : ctx->recs) ctx->pool.push_back(r.ev);
  for (auto& ev : ctx->pool)
    for (auto& e : ev) (void)hipEventDestroy(e);
  (void)hipFree(ctx->d_boxes);
  (void)hipFree(ctx->d_tilesS);
  (void)hipFree(ctx->d_tilesE);
  (void)hipFree(ctx->d_tilesX);
  (void)hipFree(ctx->d_tilesXA);
  (void)hipFree(ctx->d_tilesY);
  (void)hipFree(ctx->d_tilesZ);
  (void)hipFree(ctx->d_bricks);
  (void)hipFree(ctx->d_fbricks);
  (void)hipFree(ctx->d_desc);
  (void)hipFree(ctx->d_start);
  (void)hipFree(ctx->d_consts);
  (void)hipFree(ctx->d_flags);
  (void)hipFree(ctx->d_inv_start);
  (void)hipFree(ctx->d_inv_idx);
  delete ctx;
  return PPM_OK;
}

const char* ppm_last_error(const ppm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ppm_layout_offsets(const ppm_ctx* ctx, int64_t* off) {
  if (!ctx || !off) return PPM_EINVAL;
  std::copy(ctx->off.begin(), ctx->off.end(), off);
  return PPM_OK;
}

int ppm_flux_offsets(const ppm_ctx* ctx, int32_t d, int64_t* off) {
  if (!ctx || !off || d < 0 || d > 2) return PPM_EINVAL;
  std::copy(ctx->foff[d].begin(), ctx->foff[d].end(), off);
  return PPM_OK;
}

size_t ppm_workspace_bytes(const ppm_ctx* ctx, int32_t precision) {
  if (!ctx) return 0;
  const size_t s = precision == 1 ? sizeof(float) : sizeof(double);
  return s * (size_t)(P_PLANES * ctx->LS + E_PLANES * ctx->LE);
}

int ppm_set_workspace(ppm_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return PPM_EINVAL;
  if (((uintptr_t)dev_ptr) % 256 != 0) return ctx->fail(PPM_EINVAL, "workspace must be 256-byte aligned");
  if (dev_ptr != ctx->work || (dev_ptr ? bytes : 0) != ctx->work_bytes) ++ctx->gen;
  ctx->work = dev_ptr;
  ctx->work_bytes = dev_ptr ? bytes : 0;
  return PPM_OK;
}

int ppm_set_inflow(ppm_ctx* ctx, int32_t face, const double* state) {
  if (!ctx) return PPM_EINVAL;
  if (face < 0 || face > 5 || ctx->layout.bc[face] != PPM_BC_INFLOW)
    return ctx->fail(PPM_EINVAL, "set_inflow: the face is not an inflow face of the layout");
  if (ctx->inflow[face] != state) ++ctx->gen;
  ctx->inflow[face] = state;
  return PPM_OK;
}

int ppm_fill_boundary(ppm_ctx* ctx, double* U, int32_t mode, void* stream) {
  if (!ctx) return PPM_EINVAL;
  if (!U) return ctx->fail(PPM_EINVAL, "fill: null state");
  for (int f = 0; f < 6; ++f)
    if (ctx->layout.bc[f] == PPM_BC_INFLOW && !ctx->inflow[f])
      return ctx->fail(PPM_EINVAL, "fill: inflow face without its state (ppm_set_inflow)");
  if (mode != PPM_LAUNCH_BATCHED && mode != PPM_LAUNCH_PER_BOX) return ctx->fail(PPM_EINVAL, "fill: bad mode");
  hipStream_t s = (hipStream_t)stream;
  const DevLevel L = ctx->level();
  const Plan& P = *ctx->plan;
  if (mode == PPM_LAUNCH_BATCHED) {
    ppm_ctx::ProfRec* r = ctx->prof ? ctx->begin_rec(PROF_FILL, 2) : nullptr;
    if (r) (void)hipEventRecord(r->ev[0], s);
    const int rc = ctx->hip(launch_fill(L, U, 0, (int)P.desc.size(), 0, P.start.back(), s), "fill");
    if (r) (void)hipEventRecord(r->ev[1], s);
    return rc;
  }
  for (int b = 0; b < ctx->layout.nbox; ++b) {
    const int d0 = P.box_desc[b], d1 = P.box_desc[b + 1];
    const int rc = ctx->hip(launch_fill(L, U, d0, d1, P.start[d0], P.start[d1], s), "fill");
    if (rc) return rc;
  }
  return PPM_OK;
}

int ppm_compute_dt(ppm_ctx* ctx, const double* U, const double dx[3], const ppm_params* params,
                   double* dt_dev, void* stream) {
  if (!ctx) return PPM_EINVAL;
  std::string m = validate_params(params);
  if (m.empty()) m = validate_dx(dx);
  if (m.empty() && !(params->cfl > 0.0 && params->cfl < 1.0)) m = "params: cfl must be in (0, 1)";
  if (m.empty() && (!U || !dt_dev)) m = "compute_dt: null pointer";
  if (!m.empty()) return ctx->fail(PPM_EINVAL, m);
  ppm_ctx::ProfRec* r = ctx->prof ? ctx->begin_rec(PROF_DT, 2) : nullptr;
  if (r) (void)hipEventRecord(r->ev[0], (hipStream_t)stream);
  const int rc = ctx->hip(launch_compute_dt(ctx->level(), 0, (int)ctx->tilesE.size(), U, dx, params->gamma,
                                            params->small_pres, params->cfl, dt_dev, (hipStream_t)stream),
                          "compute_dt");
  if (r) (void)hipEventRecord(r->ev[1], (hipStream_t)stream);
  return rc;
}

// work: the step workspace (null: the context's, ppm_set_workspace) and its
// size; timed: record profiling events when profiling is on.
static int hydro_step_impl(ppm_ctx* ctx, const double* U, double* Unew, double* const* flux, double dt,
                           const double* dt_dev, const double dx[3], const ppm_params* params, int32_t mode,
                           void* stream, int upto, double* dt_next = nullptr, void* work = nullptr,
                           size_t work_bytes = 0, bool timed = true) {
  if (!ctx) return PPM_EINVAL;
  std::string m = validate_params(params);
  if (m.empty()) m = validate_dx(dx);
  if (m.empty() && (!U || !Unew)) m = "step: null state";
  if (m.empty() && !dt_dev && !(dt > 0.0 && std::isfinite(dt))) m = "step: dt must be positive and finite";
  if (m.empty() && mode != PPM_LAUNCH_BATCHED && mode != PPM_LAUNCH_PER_BOX) m = "step: bad mode";
  const size_t alen = (size_t)ctx->off.back() * sizeof(double);
  if (m.empty()) {
    const char* a = (const char*)U;
    const char* b = (const char*)Unew;
    if (a < b + alen && b < a + alen) m = "step: U and Unew overlap (the step is out of place)";
  }
  if (!work) {
    work = ctx->work;
    work_bytes = ctx->work_bytes;
  }
  if (m.empty() && (!work || work_bytes < ppm_workspace_bytes(ctx, params->precision)))
    m = "step: workspace missing or too small (ppm_set_workspace)";
  if (m.empty() && dt_next && !(params->cfl > 0.0 && params->cfl < 1.0)) m = "params: cfl must be in (0, 1)";
  if (!m.empty()) return ctx->fail(PPM_EINVAL, m);
  hipStream_t s = (hipStream_t)stream;
  const DevLevel L = ctx->level();
  int rc = ctx->hip(launch_step_consts(L, dt, dt_dev, dx, params->grav, s), "step consts");
  if (rc) return rc;
  SpeedOut so{nullptr, {dx[0], dx[1], dx[2]}, params->gamma, params->gamma - 1.0, params->small_pres};
  if (dt_next) {
    // after the step constants have read dt_dev, which dt_next may alias
    so.bits = (unsigned long long*)(dt_next + 1);
    rc = ctx->hip(launch_speed_clear(so.bits, s), "next dt");
    if (rc) return rc;
  }
  const int grav = (params->grav[0] != 0.0 || params->grav[1] != 0.0 || params->grav[2] != 0.0) ? 1 : 0;
  auto run = [&](int tS0, int tS1, int tE0, int tE1, int tB0, int tB1, int tF0, int tF1, const FrontRanges& fr,
                 hipEvent_t* ev) {
    return ctx->hip(launch_step(L, params->precision, tS0, tS1, tE0, tE1, tB0, tB1, tF0, tF1, fr, U, Unew, flux,
                                work,
                                params->gamma, params->small_dens, params->small_pres, params->limiter,
                                params->flattening, params->riemann_iters, grav, params->grav, s, ev, upto, so),
                    "step");
  };
  if (mode == PPM_LAUNCH_BATCHED) {
    ppm_ctx::ProfRec* r = (timed && ctx->prof) ? ctx->begin_rec(PROF_PRIM, STEP_EVENTS) : nullptr;
    rc = run(0, (int)ctx->tilesS.size(), 0, (int)ctx->tilesE.size(), 0, (int)ctx->bricks.size(), 0,
             (int)ctx->fbricks.size(), front_all(*ctx), r ? r->ev.data() : nullptr);
    if (rc) return rc;
  } else {
    for (int b = 0; b < ctx->layout.nbox; ++b) {
      const FrontRanges fr{ctx->tX_begin[b], ctx->tX_begin[b + 1], ctx->tY_begin[b], ctx->tY_begin[b + 1],
                           ctx->tZ_begin[b], ctx->tZ_begin[b + 1]};
      rc = run(ctx->tS_begin[b], ctx->tS_begin[b + 1], ctx->tE_begin[b], ctx->tE_begin[b + 1], ctx->tB_begin[b],
               ctx->tB_begin[b + 1], ctx->tF_begin[b], ctx->tF_begin[b + 1], fr, nullptr);
      if (rc) return rc;
    }
  }
  if (dt_next) return ctx->hip(launch_speed_finish(dt_next, params->cfl, s), "next dt");
  return PPM_OK;
}

int ppm_hydro_step(ppm_ctx* ctx, const double* U, double* Unew, double* const* flux, double dt,
                   const double* dt_dev, const double dx[3], const ppm_params* params, int32_t mode,
                   void* stream) {
  return hydro_step_impl(ctx, U, Unew, flux, dt, dt_dev, dx, params, mode, stream, STEP_FULL);
}

int ppm_hydro_step_dt(ppm_ctx* ctx, const double* U, double* Unew, double* const* flux, double dt,
                      const double* dt_dev, const double dx[3], const ppm_params* params, int32_t mode,
                      double* dt_next_dev, void* stream) {
  if (!ctx) return PPM_EINVAL;
  if (!dt_next_dev) return ctx->fail(PPM_EINVAL, "step_dt: null dt_next_dev");
  return hydro_step_impl(ctx, U, Unew, flux, dt, dt_dev, dx, params, mode, stream, STEP_FULL, dt_next_dev);
}

int ppm_hydro_step_noalloc(ppm_ctx* ctx, const double* U, double* Unew, double* const* flux, double dt,
                           const double* dt_dev, const double dx[3], const ppm_params* params, int32_t mode,
                           void* stream) {
  if (!ctx) return PPM_EINVAL;
  const std::string m = validate_params(params);
  if (!m.empty()) return ctx->fail(PPM_EINVAL, m);
  const size_t need = ppm_workspace_bytes(ctx, params->precision);
  if (need > (size_t)PPM_NOALLOC_SCRATCH_BYTES) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "step_noalloc: the level needs %zu bytes of step scratch, more than the library's %zu",
                  need, (size_t)PPM_NOALLOC_SCRATCH_BYTES);
    return ctx->fail(PPM_EINVAL, buf);
  }
  hipError_t e = hipSuccess;
  void* ptr = scratch_ptr(ctx->device, &e);
  if (!ptr) return ctx->hip(e == hipSuccess ? hipErrorInvalidSymbol : e, "step_noalloc: scratch address");
  return hydro_step_impl(ctx, U, Unew, flux, dt, dt_dev, dx, params, mode, stream, STEP_FULL, nullptr, ptr,
                         (size_t)PPM_NOALLOC_SCRATCH_BYTES, false);
}

int ppm_set_step_form(ppm_ctx* ctx, int32_t fused) {
  if (!ctx) return PPM_EINVAL;
  if (fused < 0 || fused > 2) return ctx->fail(PPM_EINVAL, "set_step_form: fused must be 0, 1 or 2");
  if (fused == ctx->fused) return PPM_OK;
  ++ctx->gen;
  const bool rebuild = (fused == 2) != (ctx->fused == 2);  // forms 0 and 1 share the brick list
  ctx->fused = fused;
  if (rebuild) return ctx->hip(upload_bricks(*ctx), "set_step_form");
  return PPM_OK;
}

int ppm_set_stream_tiling(ppm_ctx* ctx, int32_t sx, int32_t sy, int32_t sz) {
  if (!ctx) return PPM_EINVAL;
  if (sx < 2 || sy < 2 || sz < 1 || sx * sy > STREAM_MAX_THREADS / 2 || sx * sy % 32 != 0)
    return ctx->fail(PPM_EINVAL, "set_stream_tiling: need sx, sy >= 2, sz >= 1 and sx * sy a multiple of 32 "
                                 "up to 256");
  ++ctx->gen;
  ctx->stream_e[0] = sx;
  ctx->stream_e[1] = sy;
  ctx->stream_e[2] = sz;
  if (ctx->fused == 2) return ctx->hip(upload_bricks(*ctx), "set_stream_tiling");
  return PPM_OK;
}

int ppm_set_front_form(ppm_ctx* ctx, int32_t form) {
  if (!ctx) return PPM_EINVAL;
  if (form < 0 || form > 3) return ctx->fail(PPM_EINVAL, "set_front_form: form must be 0, 1, 2 or 3");
  if (form != ctx->front) ++ctx->gen;
  ctx->front = form;
  return PPM_OK;
}

int ppm_get_front_form(const ppm_ctx* ctx, int32_t* form) {
  if (!ctx || !form) return PPM_EINVAL;
  *form = ctx->front;
  return PPM_OK;
}

int ppm_set_front_tiling(ppm_ctx* ctx, int32_t sx, int32_t sy, int32_t sz) {
  if (!ctx) return PPM_EINVAL;
  if (sx < 1 || sy < 1 || sz < 1 || sx > FRONT_MAX_THREADS || sy > FRONT_MAX_THREADS ||
      front_threads(sx, sy) > FRONT_MAX_THREADS)
    return ctx->fail(PPM_EINVAL, "set_front_tiling: need sx, sy, sz >= 1, sx * sy <= 128 and sx + sy <= 128");
  ++ctx->gen;
  ctx->front_e[0] = sx;
  ctx->front_e[1] = sy;
  ctx->front_e[2] = sz;
  return ctx->hip(upload_front(*ctx), "set_front_tiling");
}

int ppm_get_front_tiling(const ppm_ctx* ctx, int32_t* sx, int32_t* sy, int32_t* sz) {
  if (!ctx || !sx || !sy || !sz) return PPM_EINVAL;
  *sx = ctx->front_e[0];
  *sy = ctx->front_e[1];
  *sz = ctx->front_e[2];
  return PPM_OK;
}

int ppm_get_stream_tiling(const ppm_ctx* ctx, int32_t* sx, int32_t* sy, int32_t* sz) {
  if (!ctx || !sx || !sy || !sz) return PPM_EINVAL;
  *sx = ctx->stream_e[0];
  *sy = ctx->stream_e[1];
  *sz = ctx->stream_e[2];
  return PPM_OK;
}

int ppm_get_step_form(const ppm_ctx* ctx, int32_t* fused) {
  if (!ctx || !fused) return PPM_EINVAL;
  *fused = ctx->fused;
  return PPM_OK;
}

size_t ppm_adjoint_workspace_bytes(const ppm_ctx* ctx, int32_t precision) {
  if (!ctx || precision < 0 || precision > 1) return 0;
  return adjoint_workspace_bytes(ctx->LS, ctx->LE, precision);
}

int ppm_set_adjoint_workspace(ppm_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return PPM_EINVAL;
  if (((uintptr_t)dev_ptr) % 256 != 0) return ctx->fail(PPM_EINVAL, "adjoint workspace must be 256-byte aligned");
  ctx->awork = dev_ptr;
  ctx->awork_bytes = dev_ptr ? bytes : 0;
  return PPM_OK;
}

static int adjoint_step(ppm_ctx* ctx, const double* U, const double* Unew_bar, const double* const* flux_bar,
                        double* U_bar, double dt, const double* dt_dev, const double dx[3],
                        const ppm_params* params, void* stream, bool recompute) {
  if (!ctx) return PPM_EINVAL;
  std::string m = validate_params(params);
  if (m.empty()) m = validate_dx(dx);
  if (m.empty() && (!U || !Unew_bar || !U_bar)) m = "adjoint: null pointer";
  if (m.empty() && !dt_dev && !(dt > 0.0 && std::isfinite(dt))) m = "adjoint: dt must be positive and finite";
  const size_t alen = (size_t)ctx->off.back() * sizeof(double);
  if (m.empty()) {
    const char* a = (const char*)U_bar;
    const char* b = (const char*)U;
    const char* c = (const char*)Unew_bar;
    if ((a < b + alen && b < a + alen) || (a < c + alen && c < a + alen)) m = "adjoint: U_bar overlaps an input";
    for (int d = 0; d < 3 && m.empty() && flux_bar; ++d) {
      const char* f = (const char*)flux_bar[d];
      const size_t flen = (size_t)ctx->foff[d].back() * sizeof(double);
      if (f && a < f + flen && f < a + alen) m = "adjoint: U_bar overlaps a flux adjoint";
    }
  }
  if (m.empty() && (!ctx->work || ctx->work_bytes < ppm_workspace_bytes(ctx, params->precision)))
    m = "adjoint: workspace missing or too small (ppm_set_workspace)";
  if (m.empty() && (!ctx->awork || ctx->awork_bytes < ppm_adjoint_workspace_bytes(ctx, params->precision)))
    m = "adjoint: adjoint workspace missing or too small (ppm_set_adjoint_workspace)";
  if (!m.empty()) return ctx->fail(PPM_EINVAL, m);
  hipStream_t s = (hipStream_t)stream;
  const DevLevel L = ctx->level();
  int rc = ctx->hip(launch_step_consts(L, dt, dt_dev, dx, params->grav, s), "adjoint consts");
  if (rc) return rc;
  const int grav = (params->grav[0] != 0.0 || params->grav[1] != 0.0 || params->grav[2] != 0.0) ? 1 : 0;
  const int nS = (int)ctx->tilesS.size(), nE = (int)ctx->tilesE.size();
  // recompute the forward intermediates through stage 2 (U is not written),
  // unless the workspace holds them from the forward step
  if (recompute) {
    rc = ctx->hip(launch_step(L, params->precision, 0, nS, 0, nE, 0, 0, 0, (int)ctx->fbricks.size(), front_all(*ctx),
                              U, nullptr, nullptr, ctx->work,
                              params->gamma, params->small_dens, params->small_pres, params->limiter,
                              params->flattening, params->riemann_iters, grav, params->grav, s, nullptr,
                              STEP_TO_STAGE2),
                  "adjoint recompute");
    if (rc) return rc;
  }
  FluxBar fb{{nullptr, nullptr, nullptr}};
  if (flux_bar)
    for (int d = 0; d < 3; ++d) fb.p[d] = flux_bar[d];
  return ctx->hip(launch_adjoint(L, params->precision, nS, nE, (int)ctx->tilesX.size(), (int)ctx->tilesXA.size(), U,
                                 Unew_bar, fb, U_bar,
                                 ctx->work, ctx->awork,
                                 params->gamma, params->small_dens, params->small_pres, params->limiter,
                                 params->flattening, params->riemann_iters, grav, params->grav, s),
                  "adjoint");
}

int ppm_species_offsets(const ppm_ctx* ctx, int32_t ns, int64_t* off) {
  if (!ctx || !off || ns < 1 || ns > PPM_MAX_SPECIES) return PPM_EINVAL;
  for (size_t b = 0; b < ctx->off.size(); ++b) off[b] = (int64_t)ns * (ctx->off[b] / 5);
  return PPM_OK;
}

size_t ppm_species_workspace_bytes(const ppm_ctx* ctx, int32_t ns, int32_t precision) {
  if (!ctx || ns < 1 || ns > PPM_MAX_SPECIES || precision < 0 || precision > 1) return 0;
  return species_workspace_bytes(ctx->LS, ctx->LE, ns, precision);
}

int ppm_set_species_workspace(ppm_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return PPM_EINVAL;
  if (((uintptr_t)dev_ptr) % 256 != 0) return ctx->fail(PPM_EINVAL, "species workspace must be 256-byte aligned");
  ctx->swork = dev_ptr;
  ctx->swork_bytes = dev_ptr ? bytes : 0;
  return PPM_OK;
}

int ppm_fill_species(ppm_ctx* ctx, double* RX, int32_t ns, int32_t mode, void* stream) {
  if (!ctx) return PPM_EINVAL;
  for (int f = 0; f < 6; ++f)
    if (ctx->layout.bc[f] == PPM_BC_INFLOW)
      return ctx->fail(PPM_EINVAL, "fill_species: species on a layout with an inflow face are not supported");
  if (!RX) return ctx->fail(PPM_EINVAL, "fill_species: null arena");
  if (ns < 1 || ns > PPM_MAX_SPECIES) return ctx->fail(PPM_EINVAL, "fill_species: ns must be in [1, PPM_MAX_SPECIES]");
  if (mode != PPM_LAUNCH_BATCHED && mode != PPM_LAUNCH_PER_BOX) return ctx->fail(PPM_EINVAL, "fill_species: bad mode");
  hipStream_t s = (hipStream_t)stream;
  const DevLevel L = ctx->level();
  const Plan& P = *ctx->plan;
  if (mode == PPM_LAUNCH_BATCHED)
    return ctx->hip(launch_fill_scalars(L, RX, ns, 0, (int)P.desc.size(), 0, P.start.back(), s), "fill_species");
  for (int b = 0; b < ctx->layout.nbox; ++b) {
    const int d0 = P.box_desc[b], d1 = P.box_desc[b + 1];
    const int rc = ctx->hip(launch_fill_scalars(L, RX, ns, d0, d1, P.start[d0], P.start[d1], s), "fill_species");
    if (rc) return rc;
  }
  return PPM_OK;
}

int ppm_hydro_step_species(ppm_ctx* ctx, const double* U, double* Unew, const double* RX, double* RXnew,
                           int32_t ns, double* const* flux, double dt, const double* dt_dev, const double dx[3],
                           const ppm_params* params, void* stream) {
  if (!ctx) return PPM_EINVAL;
  std::string m;
  if (ns < 1 || ns > PPM_MAX_SPECIES) m = "species step: ns must be in [1, PPM_MAX_SPECIES]";
  if (m.empty() && (!RX || !RXnew)) m = "species step: null species arena";
  if (m.empty() && params && (params->precision == 0 || params->precision == 1) &&
      (!ctx->swork || ctx->swork_bytes < ppm_species_workspace_bytes(ctx, ns, params->precision)))
    m = "species step: species workspace missing or too small (ppm_set_species_workspace)";
  if (m.empty()) {
    const size_t slen = (size_t)ns * (size_t)(ctx->off.back() / 5) * sizeof(double);
    const size_t alen = (size_t)ctx->off.back() * sizeof(double);
    const char* a = (const char*)RX;
    const char* b = (const char*)RXnew;
    const char* u = (const char*)U;
    const char* v = (const char*)Unew;
    if (a < b + slen && b < a + slen) m = "species step: RX and RXnew overlap (the step is out of place)";
    else if (u && v && ((b < u + alen && u < b + slen) || (b < v + alen && v < b + slen)))
      m = "species step: RXnew overlaps a state arena";
  }
  if (!m.empty()) return ctx->fail(PPM_EINVAL, m);
  // the hydro step validates the rest and leaves its intermediates in the
  // step workspace for the species stages
  int rc = hydro_step_impl(ctx, U, Unew, flux, dt, dt_dev, dx, params, PPM_LAUNCH_BATCHED, stream,
                           STEP_FULL_STAGED);
  if (rc) return rc;
  const int grav = (params->grav[0] != 0.0 || params->grav[1] != 0.0 || params->grav[2] != 0.0) ? 1 : 0;
  return ctx->hip(launch_species(ctx->level(), params->precision, (int)ctx->tilesS.size(), (int)ctx->tilesE.size(),
                                 RX, RXnew, ns, ctx->work, ctx->swork, params->gamma, params->small_dens,
                                 params->small_pres, params->limiter, params->flattening, params->riemann_iters,
                                 grav, (hipStream_t)stream),
                  "species step");
}

int ppm_hydro_step_adjoint(ppm_ctx* ctx, const double* U, const double* Unew_bar, const double* const* flux_bar,
                           double* U_bar, double dt, const double* dt_dev, const double dx[3],
                           const ppm_params* params, void* stream) {
  return adjoint_step(ctx, U, Unew_bar, flux_bar, U_bar, dt, dt_dev, dx, params, stream, true);
}

int ppm_hydro_step_adjoint_saved(ppm_ctx* ctx, const double* U, const double* Unew_bar,
                                 const double* const* flux_bar, double* U_bar, double dt, const double* dt_dev,
                                 const double dx[3], const ppm_params* params, void* stream) {
  return adjoint_step(ctx, U, Unew_bar, flux_bar, U_bar, dt, dt_dev, dx, params, stream, false);
}

int ppm_graph_create(ppm_ctx* ctx, double* Ua, double* Ub, const double dx[3], const ppm_params* params,
                     int32_t nsteps, void* stream, ppm_graph** out) {
  if (!ctx || !out) return PPM_EINVAL;
  *out = nullptr;
  std::string m = validate_params(params);
  if (m.empty()) m = validate_dx(dx);
  if (m.empty() && (nsteps < 1 || !Ua || !Ub)) m = "graph: need nsteps >= 1 and two state buffers";
  if (m.empty() && (!ctx->work || ctx->work_bytes < ppm_workspace_bytes(ctx, params->precision)))
    m = "graph: workspace missing or too small (ppm_set_workspace)";
  if (!m.empty()) return ctx->fail(PPM_EINVAL, m);
  hipStream_t s = (hipStream_t)stream;
  double* dtv = nullptr;
  hipError_t e = hipMalloc((void**)&dtv, 2 * sizeof(double));
  if (e != hipSuccess) return ctx->hip(e, "graph alloc");
  auto g = std::make_unique<ppm_graph>();
  g->ctx = ctx;
  e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) { (void)hipFree(dtv); return ctx->hip(e, "graph capture"); }
  int rc = PPM_OK;
  for (int k = 0; k < nsteps && rc == PPM_OK; ++k) {
    double* src = (k % 2 == 0) ? Ua : Ub;
    double* dst = (k % 2 == 0) ? Ub : Ua;
    // the first step's dt from a dt pass, every later one from the update
    // of the step before it (the same bits)
    rc = ppm_fill_boundary(ctx, src, PPM_LAUNCH_BATCHED, stream);
    if (!rc && k == 0) rc = ppm_compute_dt(ctx, src, dx, params, dtv, stream);
    if (!rc) rc = ppm_hydro_step_dt(ctx, src, dst, nullptr, 0.0, dtv, dx, params, PPM_LAUNCH_BATCHED, dtv, stream);
  }
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(s, &graph);
  if (rc || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipFree(dtv);
    return rc ? rc : ctx->hip(e, "graph end capture");
  }
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    (void)hipFree(dtv);
    return ctx->hip(e, "graph instantiate");
  }
  g->graph = graph;
  g->dtv = dtv;
  g->gen = ctx->gen;
  ctx->graphs.insert(g.get());
  *out = g.release();
  return PPM_OK;
}

int ppm_graph_launch(ppm_graph* g, void* stream) {
  if (!g || !g->exec || !g->ctx) return PPM_EINVAL;  // no graph, or its context was destroyed
  if (g->gen != g->ctx->gen)
    return g->ctx->fail(PPM_EINVAL, "graph launch: the context's workspace, tiling, step form or inflow "
                                    "state changed since the graph was captured; capture it again");
  return g->ctx->hip(hipGraphLaunch(g->exec, (hipStream_t)stream), "graph launch");
}

int ppm_graph_destroy(ppm_graph* g) {
  if (!g) return PPM_OK;
  if (g->ctx) g->ctx->graphs.erase(g);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  (void)hipFree(g->dtv);
  delete g;
  return PPM_OK;
}

int ppm_set_tiling(ppm_ctx* ctx, int32_t tile, int32_t strip_rows) {
  if (!ctx) return PPM_EINVAL;
  if (!(tile == 64 || tile == 128 || tile == 256 || tile == 512) || strip_rows < 0)
    return ctx->fail(PPM_EINVAL, "tiling: tile must be 64, 128, 256 or 512 and strip_rows >= 0");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return ctx->hip(e, "tiling");
  ++ctx->gen;  // the tile lists are re-uploaded
  ctx->tile = tile;
  ctx->strip_rows = strip_rows;
  build_tiles(*ctx);
  (void)hipFree(ctx->d_tilesS);
  (void)hipFree(ctx->d_tilesE);
  (void)hipFree(ctx->d_tilesX);
  (void)hipFree(ctx->d_tilesXA);
  (void)hipFree(ctx->d_tilesY);
  (void)hipFree(ctx->d_tilesZ);
  ctx->d_tilesS = nullptr;
  ctx->d_tilesE = nullptr;
  ctx->d_tilesX = nullptr;
  ctx->d_tilesXA = nullptr;
  ctx->d_tilesY = nullptr;
  ctx->d_tilesZ = nullptr;
  if ((e = upload(&ctx->d_tilesS, ctx->tilesS)) != hipSuccess || (e = upload(&ctx->d_tilesE, ctx->tilesE)) != hipSuccess ||
      (e = upload(&ctx->d_tilesX, ctx->tilesX)) != hipSuccess ||
      (e = upload(&ctx->d_tilesXA, ctx->tilesXA)) != hipSuccess || (e = upload(&ctx->d_tilesY, ctx->tilesY)) != hipSuccess ||
      (e = upload(&ctx->d_tilesZ, ctx->tilesZ)) != hipSuccess)
    return ctx->hip(e, "tiling upload");
  return PPM_OK;
}

int ppm_get_tiling(const ppm_ctx* ctx, int32_t* tile, int32_t* strip_rows) {
  if (!ctx || !tile || !strip_rows) return PPM_EINVAL;
  *tile = ctx->tile;
  *strip_rows = ctx->strip_rows;
  return PPM_OK;
}

int ppm_autotune(ppm_ctx* ctx, const double* U, double* Unew, const double dx[3], const ppm_params* params,
                 int32_t reps, const char* cache_path, void* stream, int32_t* tile, int32_t* strip_rows,
                 int32_t* from_cache) {
  if (!ctx) return PPM_EINVAL;
  std::string m = validate_params(params);
  if (m.empty()) m = validate_dx(dx);
  if (m.empty() && (!U || !Unew || reps < 1)) m = "autotune: need U, Unew and reps >= 1";
  if (!m.empty()) return ctx->fail(PPM_EINVAL, m);
  // key: device architecture, precision and the histogram of box extents
  hipDeviceProp_t prop;
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return ctx->hip(e, "autotune");
  std::map<std::array<int, 3>, int> hist;
  for (const ppm_box& B : ctx->boxes)
    hist[{B.hi[0] - B.lo[0] + 1, B.hi[1] - B.lo[1] + 1, B.hi[2] - B.lo[2] + 1}]++;
  std::ostringstream ks;
  ks << prop.gcnArchName << "|p" << params->precision << "|fs|";
  for (const auto& kv : hist) ks << kv.first[0] << "x" << kv.first[1] << "x" << kv.first[2] << ":" << kv.second << ";";
  const std::string key = ks.str();
  if (from_cache) *from_cache = 0;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    const std::string pat = "\"key\": \"" + key + "\"";
    while (std::getline(in, line)) {
      if (line.find(pat) == std::string::npos) continue;
      int t = 0, sr = -1, form = 0, se[3] = {0, 0, 0};
      auto field = [&](const char* name, int dflt) {
        const std::string f = std::string("\"") + name + "\": ";
        const size_t a = line.find(f);
        return a == std::string::npos ? dflt : std::atoi(line.c_str() + a + f.size());
      };
      t = field("tile", 0);
      sr = field("strip_rows", -1);
      form = field("form", 0);
      se[0] = field("sx", ctx->stream_e[0]);
      se[1] = field("sy", ctx->stream_e[1]);
      se[2] = field("sz", ctx->stream_e[2]);
      const int front = field("front", 0);
      const int fe[3] = {field("fx", ctx->front_e[0]), field("fy", ctx->front_e[1]), field("fz", ctx->front_e[2])};
      if (ppm_set_tiling(ctx, t, sr) == PPM_OK && ppm_set_stream_tiling(ctx, se[0], se[1], se[2]) == PPM_OK &&
          ppm_set_step_form(ctx, form) == PPM_OK && ppm_set_front_tiling(ctx, fe[0], fe[1], fe[2]) == PPM_OK &&
          ppm_set_front_form(ctx, front) == PPM_OK) {
        if (tile) *tile = t;
        if (strip_rows) *strip_rows = sr;
        if (from_cache) *from_cache = 1;
        return PPM_OK;
      }
    }
  }
  hipStream_t s = (hipStream_t)stream;
  double* dtv = nullptr;
  // dtv[0..1]: the step's dt; dtv[2..3]: the next dt the timed steps leave,
  // as the graph and the benchmark run them
  if ((e = hipMalloc((void**)&dtv, 4 * sizeof(double))) != hipSuccess) return ctx->hip(e, "autotune");
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int tiles[] = {128, 256, 512};
  const int strips[] = {8, 16, 32, 64, 0};
  (void)ppm_set_front_form(ctx, 0);  // tiling and final stage timed with the staged front end
  float best = 1e30f;
  int bt = ctx->tile, bs = ctx->strip_rows;
  int rc = PPM_OK;
  for (int t : tiles) {
    for (int sr : strips) {
      if ((rc = ppm_set_tiling(ctx, t, sr)) != PPM_OK) break;
      if ((rc = ppm_compute_dt(ctx, U, dx, params, dtv, stream)) != PPM_OK) break;
      if ((rc = ppm_hydro_step_dt(ctx, U, Unew, nullptr, 0.0, dtv, dx, params, PPM_LAUNCH_BATCHED, dtv + 2,
                                  stream)) != PPM_OK)
        break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && rc == PPM_OK; ++r)
        rc = ppm_hydro_step_dt(ctx, U, Unew, nullptr, 0.0, dtv, dx, params, PPM_LAUNCH_BATCHED, dtv + 2, stream);
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if (ms < best) { best = ms; bt = t; bs = sr; }
    }
    if (rc) break;
  }
  if (!rc) rc = ppm_set_tiling(ctx, bt, bs);
  // then the final stage's form: the staged pair of kernels, the brick
  // kernel, or the streamed kernel with one of its tile shapes (x, y
  // extents, z run)
  static const int shapes[][3] = {{16, 8, 32}, {32, 8, 32}, {16, 16, 32}, {32, 4, 32}, {16, 8, 64}, {32, 8, 16},
                                  {64, 4, 32}};
  int bform = 0, bse[3] = {ctx->stream_e[0], ctx->stream_e[1], ctx->stream_e[2]};
  const int form0 = ctx->fused;
  auto timed = [&](float& ms) {
    int r = ppm_compute_dt(ctx, U, dx, params, dtv, stream);
    if (!r) r = ppm_hydro_step_dt(ctx, U, Unew, nullptr, 0.0, dtv, dx, params, PPM_LAUNCH_BATCHED, dtv + 2, stream);
    (void)hipEventRecord(e0, s);
    for (int q = 0; q < reps && !r; ++q)
      r = ppm_hydro_step_dt(ctx, U, Unew, nullptr, 0.0, dtv, dx, params, PPM_LAUNCH_BATCHED, dtv + 2, stream);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= reps;
    return r;
  };
  if (!rc) {
    float ms = 0.f;
    if (!(rc = ppm_set_step_form(ctx, 0)) && !(rc = timed(ms))) best = ms;
    if (!rc && !(rc = ppm_set_step_form(ctx, 1)) && !(rc = timed(ms)) && ms < best) {
      best = ms;
      bform = 1;
    }
    for (const auto& sh : shapes) {
      if (rc) break;
      if (ppm_set_stream_tiling(ctx, sh[0], sh[1], sh[2]) != PPM_OK) continue;
      if ((rc = ppm_set_step_form(ctx, 2)) || (rc = timed(ms))) break;
      if (ms < best) {
        best = ms;
        bform = 2;
        for (int d = 0; d < 3; ++d) bse[d] = sh[d];
      }
      if ((rc = ppm_set_step_form(ctx, 0))) break;
    }
  }
  // then the front end, with the final stage chosen: staged, streamed with
  // one of its tile shapes, or the x axis fused
  static const int fshapes[][3] = {{11, 11, 32}, {16, 8, 32}};
  int bfront = 0, bfe[3] = {ctx->front_e[0], ctx->front_e[1], ctx->front_e[2]};
  const int front0 = ctx->front;
  if (!rc && !(rc = ppm_set_stream_tiling(ctx, bse[0], bse[1], bse[2])) && !(rc = ppm_set_step_form(ctx, bform))) {
    float ms = 0.f;
    for (const auto& sh : fshapes) {
      if ((rc = ppm_set_front_tiling(ctx, sh[0], sh[1], sh[2])) || (rc = ppm_set_front_form(ctx, 1)) ||
          (rc = timed(ms)))
        break;
      if (ms < best) {
        best = ms;
        bfront = 1;
        for (int d = 0; d < 3; ++d) bfe[d] = sh[d];
      }
    }
    for (int f = 2; f <= 3 && !rc; ++f)
      if (!(rc = ppm_set_front_form(ctx, f)) && !(rc = timed(ms)) && ms < best) {
        best = ms;
        bfront = f;
      }
    if (!rc) rc = ppm_set_front_form(ctx, 0);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(dtv);
  if (rc) {
    (void)ppm_set_step_form(ctx, form0);
    (void)ppm_set_front_form(ctx, front0);
    return rc;
  }
  if ((rc = ppm_set_stream_tiling(ctx, bse[0], bse[1], bse[2])) || (rc = ppm_set_step_form(ctx, bform)) ||
      (rc = ppm_set_front_tiling(ctx, bfe[0], bfe[1], bfe[2])) || (rc = ppm_set_front_form(ctx, bfront)))
    return rc;
  if (tile) *tile = bt;
  if (strip_rows) *strip_rows = bs;
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << "{\"key\": \"" << key << "\", \"tile\": " << bt << ", \"strip_rows\": " << bs
        << ", \"form\": " << bform << ", \"sx\": " << bse[0] << ", \"sy\": " << bse[1] << ", \"sz\": " << bse[2]
        << ", \"front\": " << bfront << ", \"fx\": " << bfe[0] << ", \"fy\": " << bfe[1] << ", \"fz\": " << bfe[2]
        << ", \"ms_per_step\": " << best << "}\n";
  }
  return PPM_OK;
}

int ppm_profile_enable(ppm_ctx* ctx, int32_t on) {
  if (!ctx) return PPM_EINVAL;
  ctx->prof = on != 0;
  return PPM_OK;
}

int ppm_profile_read(ppm_ctx* ctx, double* ms, int64_t* count) {
  if (!ctx || !ms || !count) return PPM_EINVAL;
  for (int k = 0; k < PROF_NTAGS; ++k) { ms[k] = 0.0; count[k] = 0; }
  for (auto& r : ctx->recs) {
    hipError_t e = hipEventSynchronize(r.ev[r.n - 1]);
    if (e != hipSuccess) return ctx->hip(e, "profile_read");
    for (int i = 0; i + 1 < r.n; ++i) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, r.ev[i], r.ev[i + 1]);
      if (e != hipSuccess) return ctx->hip(e, "profile_read");
      ms[r.tag0 + i] += t;
      count[r.tag0 + i] += 1;
    }
  }
  for (auto& r : ctx->recs) ctx->pool.push_back(r.ev);
  ctx->recs.clear();
  return PPM_OK;
}

int ppm_check_status(ppm_ctx* ctx, void* stream, int32_t* flags) {
  if (!ctx || !flags) return PPM_EINVAL;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipMemcpy(flags, ctx->d_flags, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(ctx->d_flags, 0, sizeof(int32_t));
  if (e != hipSuccess) return ctx->hip(e, "check_status");
  return *flags ? PPM_ENONPHYS : PPM_OK;
}

static void desc_to20(const FillDesc& D, int32_t* o) {
  o[0] = D.dst; o[1] = D.src;
  for (int d = 0; d < 3; ++d) {
    o[2 + d] = D.lo[d]; o[5 + d] = D.hi[d]; o[8 + d] = D.a[d]; o[11 + d] = D.c[d];
  }
  o[14] = D.sign; o[15] = D.count;
  o[16] = o[17] = o[18] = o[19] = 0;
}

int ppm_plan_build(const ppm_layout* layout, int32_t brute, int32_t max, int32_t* out20, int32_t* count) {
  if (!layout || !count) return PPM_EINVAL;
  const std::string m = validate_layout(*layout);
  if (!m.empty()) {
    std::fprintf(stderr, "ppm_plan_build: %s\n", m.c_str());
    return PPM_EINVAL;
  }
  std::shared_ptr<const Plan> P;
  if (brute) {
    P = std::make_shared<const Plan>(build_plan(*layout, true));
  } else {
    bool hit = false;
    P = plan_cache().get(*layout, hit);
  }
  *count = (int32_t)P->desc.size();
  for (int32_t k = 0; k < *count && k < max && out20; ++k) desc_to20(P->desc[k], out20 + 20 * k);
  return PPM_OK;
}

int ppm_fill_boundary_host(const ppm_layout* layout, double* U) {
  if (!layout || !U) return PPM_EINVAL;
  std::string m = validate_layout(*layout);
  for (int f = 0; m.empty() && f < 6; ++f)
    if (layout->bc[f] == PPM_BC_INFLOW) m = "inflow faces need device state (ppm_set_inflow)";
  if (!m.empty()) {
    std::fprintf(stderr, "ppm_fill_boundary_host: %s\n", m.c_str());
    return PPM_EINVAL;
  }
  bool hit = false;
  std::shared_ptr<const Plan> P = plan_cache().get(*layout, hit);
  const ppm_box* B = layout->boxes;
  std::vector<long long> off(layout->nbox + 1, 0);
  for (int b = 0; b < layout->nbox; ++b) {
    long long ns = 5;
    for (int d = 0; d < 3; ++d) ns *= B[b].hi[d] - B[b].lo[d] + 1 + 2 * NG;
    off[b + 1] = off[b] + ns;
  }
  for (const FillDesc& D : P->desc) {
    int dn[3], sn[3];
    for (int d = 0; d < 3; ++d) {
      dn[d] = B[D.dst].hi[d] - B[D.dst].lo[d] + 1 + 2 * NG;
      sn[d] = B[D.src].hi[d] - B[D.src].lo[d] + 1 + 2 * NG;
    }
    const long long dNS = (long long)dn[0] * dn[1] * dn[2], sNS = (long long)sn[0] * sn[1] * sn[2];
    for (int z = D.lo[2]; z <= D.hi[2]; ++z)
      for (int y = D.lo[1]; y <= D.hi[1]; ++y)
        for (int x = D.lo[0]; x <= D.hi[0]; ++x) {
          const int sx = D.a[0] * x + D.c[0], sy = D.a[1] * y + D.c[1], sz = D.a[2] * z + D.c[2];
          const long long di = off[D.dst] + ((long long)(z + NG) * dn[1] + (y + NG)) * dn[0] + (x + NG);
          const long long si = off[D.src] + ((long long)(sz + NG) * sn[1] + (sy + NG)) * sn[0] + (sx + NG);
          for (int c = 0; c < 5; ++c) {
            const double v = U[si + c * sNS];
            const bool neg = c >= 1 && c <= 3 && ((D.sign >> (c - 1)) & 1);
            U[di + c * dNS] = neg ? -v : v;
          }
        }
  }
  return PPM_OK;
}

int ppm_plan_cache_stats(int64_t* lookups, int64_t* hits, int32_t* entries) {
  PlanCache& c = plan_cache();
  std::lock_guard<std::mutex> g(c.mu);
  if (lookups) *lookups = c.lookups;
  if (hits) *hits = c.hits;
  if (entries) *entries = (int32_t)c.lru.size();
  return PPM_OK;
}

}  // extern "C"
