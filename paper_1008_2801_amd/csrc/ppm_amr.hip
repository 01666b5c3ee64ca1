// Two-level advance with subcycling in time (refinement ratio 2) on one GPU.
//
// The compressible code refines a region of the domain and advances it with
// subcycling: one coarse time step is one step on the coarse level and two
// on the fine level, followed by synchronisation of the two levels (paper
// Sec. 1-3).  The formulas are the standard Berger-Colella ones:
//   dt      one coarse dt = cfl / max(S_c, S_f / 2), two fine steps of dt/2
//   fill    fine ghost zones: the fine level's own plan where another fine
//           box has them; beyond the refined region, conservative linear
//           interpolation (MC-limited slopes, offsets -+1/4) of the coarse
//           state interpolated linearly in time, (1 - th) U_old + th U_new,
//           th = 0 for the first and 1/2 for the second fine step
//   register  per coarse face of the refined region's surface, the fine
//           fluxes of its 4 sub-faces summed pairwise, both fine steps added
//   reflux  the uncovered coarse zone next to such a face gets
//           -+ dt/h (register / 8 - its coarse flux)
//   average down  covered coarse zones = mean of their 8 fine zones
//           (pairwise sums, times 1/8)
// Every sum is evaluated in the stated order, so FP64 results agree with a
// serial evaluation of the same definitions bit for bit.
//
// The refined region is one rectangle of whole coarse zones, at least 3
// coarse zones from every domain face, and the fine boxes start and end on
// coarse-zone boundaries; the fine level's layout has the refined region as
// its domain and PPM_BC_COARSE_FINE on all six faces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "ppm_ctx.h"

namespace ppm {
namespace {

constexpr int AMR_THREADS = 256;
constexpr int MARGIN = 3;

// Fine ghost zones (fine-box-local range, may be negative) of fine box fb
// whose coarse parents are valid zones of coarse box cb.
struct InterpDesc {
  int fb, cb;
  int lo[3], hi[3];
};
// Covered coarse zones (coarse-box-local range) of coarse box cb whose
// children are zones of fine box fb.
struct AvgDesc {
  int cb, fb;
  int lo[3], hi[3];
};
// A coarse face of the refined region's surface: axis d; side 0 = the
// region's low face (the face is the uncovered zone's high face), 1 = its
// high face; the uncovered zone c (local in coarse box cb) and the fine
// sub-face (0,0) f (face-local in fine box fb).
struct RegFace {
  int d, side, cb, fb;
  int c[3], f[3];
};

__device__ __forceinline__ int find_desc(const long long* __restrict__ start, int nd, long long g) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ long long sidx(const DevBox& B, int x, int y, int z) {
  const int N0 = B.n[0] + 2 * NG, N1 = B.n[1] + 2 * NG;
  return ((long long)(z + NG) * N1 + (y + NG)) * N0 + (x + NG);
}

__device__ __forceinline__ long long nstored(const DevBox& B) {
  return (long long)(B.n[0] + 2 * NG) * (B.n[1] + 2 * NG) * (B.n[2] + 2 * NG);
}

__device__ __forceinline__ double mc_slope(double um, double u0, double up) {
  const double dc = 0.5 * (up - um);
  const double dl = u0 - um;
  const double dr = up - u0;
  const double m = fmin(fmin(fabs(dc), 2.0 * fabs(dl)), 2.0 * fabs(dr));
  return (dl * dr > 0.0) ? copysign(m, dc) : 0.0;
}

__global__ void __launch_bounds__(AMR_THREADS) k_cf_interp(const InterpDesc* __restrict__ desc,
                                                       const long long* __restrict__ start, int nd,
                                                       const DevBox* __restrict__ cboxes,
                                                       const DevBox* __restrict__ fboxes,
                                                       const int* __restrict__ cgl, const int* __restrict__ fgl,
                                                       const double* __restrict__ Uold,
                                                       const double* __restrict__ Unew, double th,
                                                       double* __restrict__ Uf) {
  const long long g = (long long)blockIdx.x * AMR_THREADS + threadIdx.x;
  if (g >= start[nd]) return;
  const int k = find_desc(start, nd, g);
  const InterpDesc D = desc[k];
  const long long l = g - start[k];
  const int ex = D.hi[0] - D.lo[0] + 1, ey = D.hi[1] - D.lo[1] + 1;
  const int x[3] = {D.lo[0] + (int)(l % ex), D.lo[1] + (int)((l / ex) % ey),
                    D.lo[2] + (int)(l / ((long long)ex * ey))};
  const DevBox F = fboxes[D.fb], C = cboxes[D.cb];
  int cl[3];
  double o[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int gf = fgl[3 * D.fb + d] + x[d];  // fine global index
    const int gc = gf >> 1;                   // coarse parent (floor)
    o[d] = (gf & 1) ? 0.25 : -0.25;
    cl[d] = gc - cgl[3 * D.cb + d];
  }
  const long long cs = nstored(C), fs = nstored(F);
  const long long c0 = C.soff + sidx(C, cl[0], cl[1], cl[2]);
  const long long sx = 1, sy = C.n[0] + 2 * NG, sz = (long long)sy * (C.n[1] + 2 * NG);
  const long long fi = F.soff + sidx(F, x[0], x[1], x[2]);
  const double a = 1.0 - th;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double* po = Uold + c0 + c * cs;
    const double* pn = Unew + c0 + c * cs;
    auto ut = [&](long long q) { return a * po[q] + th * pn[q]; };
    const double u0 = ut(0);
    const double gx = mc_slope(ut(-sx), u0, ut(sx));
    const double gy = mc_slope(ut(-sy), u0, ut(sy));
    const double gz = mc_slope(ut(-sz), u0, ut(sz));
    Uf[fi + c * fs] = u0 + ((gx * o[0] + gy * o[1]) + gz * o[2]);
  }
}

__global__ void __launch_bounds__(AMR_THREADS) k_reg_zero(double* __restrict__ reg, long long n) {
  const long long i = (long long)blockIdx.x * AMR_THREADS + threadIdx.x;
  if (i < n) reg[i] = 0.0;
}

// Face-centred flux index (extents n + e_d) of face f in a box.
__device__ __forceinline__ long long fidx(const DevBox& B, int d, int x, int y, int z, long long& FN) {
  const int e0 = B.n[0] + (d == 0), e1 = B.n[1] + (d == 1), e2 = B.n[2] + (d == 2);
  FN = (long long)e0 * e1 * e2;
  return ((long long)z * e1 + y) * e0 + x;
}

__global__ void __launch_bounds__(AMR_THREADS) k_reg_accum(const RegFace* __restrict__ faces, int nf,
                                                       const DevBox* __restrict__ fboxes,
                                                       const double* __restrict__ Fx,
                                                       const double* __restrict__ Fy,
                                                       const double* __restrict__ Fz, double* __restrict__ reg) {
  const int i = blockIdx.x * AMR_THREADS + threadIdx.x;
  if (i >= nf) return;
  const RegFace R = faces[i];
  const DevBox B = fboxes[R.fb];
  const int t1 = (R.d == 0) ? 1 : 0, t2 = (R.d == 2) ? 1 : 2;
  const double* F = (R.d == 0 ? Fx : (R.d == 1 ? Fy : Fz)) + B.foff[R.d];
  int f10[3] = {R.f[0], R.f[1], R.f[2]}, f01[3] = {R.f[0], R.f[1], R.f[2]}, f11[3] = {R.f[0], R.f[1], R.f[2]};
  f10[t1] += 1;
  f01[t2] += 1;
  f11[t1] += 1;
  f11[t2] += 1;
  long long FN;
  const long long i00 = fidx(B, R.d, R.f[0], R.f[1], R.f[2], FN);
  const long long i10 = fidx(B, R.d, f10[0], f10[1], f10[2], FN);
  const long long i01 = fidx(B, R.d, f01[0], f01[1], f01[2], FN);
  const long long i11 = fidx(B, R.d, f11[0], f11[1], f11[2], FN);
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double* q = F + c * FN;
    reg[5 * (long long)i + c] = reg[5 * (long long)i + c] + ((q[i00] + q[i10]) + (q[i01] + q[i11]));
  }
}

__global__ void __launch_bounds__(AMR_THREADS) k_reflux(const RegFace* __restrict__ faces, int nf,
                                                    const DevBox* __restrict__ cboxes,
                                                    const double* __restrict__ Fx, const double* __restrict__ Fy,
                                                    const double* __restrict__ Fz,
                                                    const double* __restrict__ reg,
                                                    const StepConsts* __restrict__ sc, double* __restrict__ Uc) {
  const int i = blockIdx.x * AMR_THREADS + threadIdx.x;
  if (i >= nf) return;
  const RegFace R = faces[i];
  const DevBox B = cboxes[R.cb];
  const double* F = (R.d == 0 ? Fx : (R.d == 1 ? Fy : Fz)) + B.foff[R.d];
  int fl[3] = {R.c[0], R.c[1], R.c[2]};
  if (R.side == 0) fl[R.d] += 1;  // the uncovered zone's high face
  long long FN;
  const long long fi = fidx(B, R.d, fl[0], fl[1], fl[2], FN);
  const long long ui = B.soff + sidx(B, R.c[0], R.c[1], R.c[2]);
  const long long NS = nstored(B);
  const double dtdx = sc->dtdx[R.d];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double dF = reg[5 * (long long)i + c] * 0.125 - F[fi + c * FN];
    const double u = Uc[ui + c * NS];
    Uc[ui + c * NS] = (R.side == 0) ? u - dtdx * dF : u + dtdx * dF;
  }
}

__global__ void __launch_bounds__(AMR_THREADS) k_avg_down(const AvgDesc* __restrict__ desc,
                                                      const long long* __restrict__ start, int nd,
                                                      const DevBox* __restrict__ cboxes,
                                                      const DevBox* __restrict__ fboxes,
                                                      const int* __restrict__ cgl, const int* __restrict__ fgl,
                                                      const double* __restrict__ Uf, double* __restrict__ Uc) {
  const long long g = (long long)blockIdx.x * AMR_THREADS + threadIdx.x;
  if (g >= start[nd]) return;
  const int k = find_desc(start, nd, g);
  const AvgDesc D = desc[k];
  const long long l = g - start[k];
  const int ex = D.hi[0] - D.lo[0] + 1, ey = D.hi[1] - D.lo[1] + 1;
  const int x[3] = {D.lo[0] + (int)(l % ex), D.lo[1] + (int)((l / ex) % ey),
                    D.lo[2] + (int)(l / ((long long)ex * ey))};
  const DevBox C = cboxes[D.cb], F = fboxes[D.fb];
  int f0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) f0[d] = 2 * (cgl[3 * D.cb + d] + x[d]) - fgl[3 * D.fb + d];
  const long long fs = nstored(F), cs = nstored(C);
  const long long b = F.soff + sidx(F, f0[0], f0[1], f0[2]);
  const long long sy = F.n[0] + 2 * NG, sz = sy * (F.n[1] + 2 * NG);
  const long long ci = C.soff + sidx(C, x[0], x[1], x[2]);
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double* q = Uf + b + c * fs;
    const double s = ((q[0] + q[1]) + (q[sy] + q[sy + 1])) + ((q[sz] + q[sz + 1]) + (q[sz + sy] + q[sz + sy + 1]));
    Uc[ci + c * cs] = s * 0.125;
  }
}

// d[0..1]: coarse (cfl / S_c, S_c); d[2..3]: fine (cfl / S_f, S_f);
// d[4] = coarse dt, d[5] = fine dt.
__global__ void __launch_bounds__(64) k_amr_dt(double* d, double cfl, double fixed) {
  if (threadIdx.x != 0) return;
  const double dt = fixed > 0.0 ? fixed : cfl / fmax(d[1], 0.5 * d[3]);
  d[4] = dt;
  d[5] = 0.5 * dt;
}

__global__ void __launch_bounds__(64) k_copy2(const double* __restrict__ s, double* __restrict__ o) {
  if (threadIdx.x < 2) o[threadIdx.x] = s[threadIdx.x];
}

unsigned grid_for(long long n) { return (unsigned)((n + AMR_THREADS - 1) / AMR_THREADS); }

}  // namespace
}  // namespace ppm

struct ppm_amr {
  ppm_ctx* c = nullptr;
  ppm_ctx* f = nullptr;
  int rlo[3], rhi[3];  // refined region, coarse indices
  std::vector<ppm::InterpDesc> idesc;
  std::vector<long long> istart;
  std::vector<ppm::AvgDesc> adesc;
  std::vector<long long> astart;
  std::vector<ppm::RegFace> faces;
  ppm::InterpDesc* d_idesc = nullptr;
  long long* d_istart = nullptr;
  ppm::AvgDesc* d_adesc = nullptr;
  long long* d_astart = nullptr;
  ppm::RegFace* d_faces = nullptr;
  int* d_cgl = nullptr;
  int* d_fgl = nullptr;
  double* d_reg = nullptr;
  double* d_dt = nullptr;
  std::string err;
  int fail(int code, const std::string& m) {
    err = m;
    if (c) c->err = m;
    return code;
  }
  int hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return PPM_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    if (c) c->err = err;
    return PPM_EHIP;
  }
};

namespace {
using namespace ppm;

template <class T> hipError_t upload_vec(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  hipError_t e = hipMalloc((void**)dst, bytes);
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

// Painted owner map of a rectangle [lo, hi] (global indices) by a level's boxes.
struct Owner {
  int lo[3], ext[3];
  std::vector<int> m;
  Owner(const ppm_ctx& L, const int l[3], const int h[3]) {
    size_t tot = 1;
    for (int d = 0; d < 3; ++d) { lo[d] = l[d]; ext[d] = h[d] - l[d] + 1; tot *= (size_t)ext[d]; }
    m.assign(tot, -1);
    for (int b = 0; b < L.layout.nbox; ++b) {
      const ppm_box& B = L.boxes[b];
      int a[3], e[3];
      bool any = true;
      for (int d = 0; d < 3; ++d) {
        a[d] = std::max(B.lo[d], lo[d]);
        e[d] = std::min(B.hi[d], lo[d] + ext[d] - 1);
        any = any && a[d] <= e[d];
      }
      if (!any) continue;
      for (int z = a[2]; z <= e[2]; ++z)
        for (int y = a[1]; y <= e[1]; ++y)
          for (int x = a[0]; x <= e[0]; ++x)
            m[((size_t)(z - lo[2]) * ext[1] + (y - lo[1])) * ext[0] + (x - lo[0])] = b;
    }
  }
  int at(const int x[3]) const {
    for (int d = 0; d < 3; ++d)
      if (x[d] < lo[d] || x[d] >= lo[d] + ext[d]) return -1;
    return m[((size_t)(x[2] - lo[2]) * ext[1] + (x[1] - lo[1])) * ext[0] + (x[0] - lo[0])];
  }
};

std::string build(ppm_amr& A) {
  const ppm_ctx& C = *A.c;
  const ppm_ctx& F = *A.f;
  const ppm_layout& fl = F.layout;
  for (int s = 0; s < 6; ++s)
    if (fl.bc[s] != PPM_BC_COARSE_FINE) return "amr: the fine layout needs PPM_BC_COARSE_FINE on all faces";
  int flo[3], fhi[3];
  for (int d = 0; d < 3; ++d) {
    flo[d] = fl.domain.lo[d];
    fhi[d] = fl.domain.hi[d];
    if ((flo[d] & 1) || !(fhi[d] & 1)) return "amr: the fine domain must be the refinement of whole coarse zones";
    A.rlo[d] = flo[d] / 2;
    A.rhi[d] = (fhi[d] - 1) / 2;
    if (A.rlo[d] - C.layout.domain.lo[d] < MARGIN || C.layout.domain.hi[d] - A.rhi[d] < MARGIN)
      return "amr: the refined region must be at least 3 coarse zones from every domain face";
  }
  for (int b = 0; b < fl.nbox; ++b)
    for (int d = 0; d < 3; ++d)
      if ((F.boxes[b].lo[d] & 1) || !(F.boxes[b].hi[d] & 1))
        return "amr: fine boxes must start and end on coarse-zone boundaries";
  // fine ghost zones beyond the refined region, split by coarse owner
  A.idesc.clear();
  for (int b = 0; b < fl.nbox; ++b) {
    const ppm_box& B = F.boxes[b];
    struct Iv { int lo, hi; bool out; };
    std::vector<Iv> iv[3];
    for (int d = 0; d < 3; ++d) {
      const int l = B.lo[d], h = B.hi[d];
      // below: [l-4, l-1]
      if (std::max(l - NG, flo[d]) <= l - 1) iv[d].push_back({std::max(l - NG, flo[d]), l - 1, false});
      if (l - NG <= std::min(l - 1, flo[d] - 1)) iv[d].push_back({l - NG, std::min(l - 1, flo[d] - 1), true});
      iv[d].push_back({l, h, false});
      if (h + 1 <= std::min(h + NG, fhi[d])) iv[d].push_back({h + 1, std::min(h + NG, fhi[d]), false});
      if (std::max(h + 1, fhi[d] + 1) <= h + NG) iv[d].push_back({std::max(h + 1, fhi[d] + 1), h + NG, true});
    }
    for (const Iv& a : iv[0])
      for (const Iv& e : iv[1])
        for (const Iv& g : iv[2]) {
          if (!a.out && !e.out && !g.out) continue;
          const Iv* p[3] = {&a, &e, &g};
          for (int cb = 0; cb < C.layout.nbox; ++cb) {
            const ppm_box& K = C.boxes[cb];
            InterpDesc D;
            D.fb = b;
            D.cb = cb;
            bool any = true;
            for (int d = 0; d < 3; ++d) {
              const int l2 = std::max(p[d]->lo, 2 * K.lo[d]), h2 = std::min(p[d]->hi, 2 * K.hi[d] + 1);
              any = any && l2 <= h2;
              D.lo[d] = l2 - B.lo[d];
              D.hi[d] = h2 - B.lo[d];
            }
            if (any) A.idesc.push_back(D);
          }
        }
  }
  A.istart.assign(A.idesc.size() + 1, 0);
  for (size_t k = 0; k < A.idesc.size(); ++k) {
    long long n = 1;
    for (int d = 0; d < 3; ++d) n *= A.idesc[k].hi[d] - A.idesc[k].lo[d] + 1;
    A.istart[k + 1] = A.istart[k] + n;
  }
  // covered coarse zones, split by coarse and fine box
  A.adesc.clear();
  for (int cb = 0; cb < C.layout.nbox; ++cb)
    for (int b = 0; b < fl.nbox; ++b) {
      const ppm_box& K = C.boxes[cb];
      const ppm_box& B = F.boxes[b];
      AvgDesc D;
      D.cb = cb;
      D.fb = b;
      bool any = true;
      for (int d = 0; d < 3; ++d) {
        const int l2 = std::max(K.lo[d], B.lo[d] / 2), h2 = std::min(K.hi[d], (B.hi[d] - 1) / 2);
        any = any && l2 <= h2;
        D.lo[d] = l2 - K.lo[d];
        D.hi[d] = h2 - K.lo[d];
      }
      if (any) A.adesc.push_back(D);
    }
  A.astart.assign(A.adesc.size() + 1, 0);
  for (size_t k = 0; k < A.adesc.size(); ++k) {
    long long n = 1;
    for (int d = 0; d < 3; ++d) n *= A.adesc[k].hi[d] - A.adesc[k].lo[d] + 1;
    A.astart[k + 1] = A.astart[k] + n;
  }
  // register faces
  int glo[3], ghi[3];
  for (int d = 0; d < 3; ++d) { glo[d] = A.rlo[d] - 1; ghi[d] = A.rhi[d] + 1; }
  const Owner cown(C, glo, ghi);
  const Owner fown(F, flo, fhi);
  A.faces.clear();
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    for (int side = 0; side < 2; ++side) {
      const int fc = side == 0 ? A.rlo[d] : A.rhi[d] + 1;
      for (int k = A.rlo[t2]; k <= A.rhi[t2]; ++k)
        for (int j = A.rlo[t1]; j <= A.rhi[t1]; ++j) {
          RegFace R;
          R.d = d;
          R.side = side;
          int z[3];
          z[d] = side == 0 ? fc - 1 : fc;
          z[t1] = j;
          z[t2] = k;
          R.cb = cown.at(z);
          int fz[3];  // the fine zone inside the region next to sub-face (0,0)
          fz[d] = side == 0 ? 2 * fc : 2 * fc - 1;
          fz[t1] = 2 * j;
          fz[t2] = 2 * k;
          R.fb = fown.at(fz);
          if (R.cb < 0 || R.fb < 0) return "amr: a register face has no owning box";
          for (int e = 0; e < 3; ++e) R.c[e] = z[e] - C.boxes[R.cb].lo[e];
          R.f[d] = 2 * fc - F.boxes[R.fb].lo[d];
          R.f[t1] = 2 * j - F.boxes[R.fb].lo[t1];
          R.f[t2] = 2 * k - F.boxes[R.fb].lo[t2];
          A.faces.push_back(R);
        }
    }
  }
  return "";
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}
}  // namespace

extern "C" {

int ppm_amr_create(ppm_ctx* coarse, ppm_ctx* fine, ppm_amr** out) {
  if (!coarse || !fine || !out) return PPM_EINVAL;
  *out = nullptr;
  auto A = std::make_unique<ppm_amr>();
  A->c = coarse;
  A->f = fine;
  const std::string m = build(*A);
  if (!m.empty()) return coarse->fail(PPM_EINVAL, m);
  std::vector<int> cgl, fgl;
  for (const ppm_box& b : coarse->boxes)
    for (int d = 0; d < 3; ++d) cgl.push_back(b.lo[d]);
  for (const ppm_box& b : fine->boxes)
    for (int d = 0; d < 3; ++d) fgl.push_back(b.lo[d]);
  hipError_t e;
  if ((e = upload_vec(&A->d_idesc, A->idesc)) != hipSuccess ||
      (e = upload_vec(&A->d_istart, A->istart)) != hipSuccess ||
      (e = upload_vec(&A->d_adesc, A->adesc)) != hipSuccess ||
      (e = upload_vec(&A->d_astart, A->astart)) != hipSuccess ||
      (e = upload_vec(&A->d_faces, A->faces)) != hipSuccess ||
      (e = upload_vec(&A->d_cgl, cgl)) != hipSuccess || (e = upload_vec(&A->d_fgl, fgl)) != hipSuccess ||
      (e = hipMalloc((void**)&A->d_reg, std::max<size_t>(1, A->faces.size()) * 5 * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&A->d_dt, 8 * sizeof(double))) != hipSuccess ||
      (e = hipMemset(A->d_dt, 0, 8 * sizeof(double))) != hipSuccess) {
    const int rc = A->hip(e, "amr create");
    ppm_amr_destroy(A.release());
    return rc;
  }
  *out = A.release();
  return PPM_OK;
}

int ppm_amr_destroy(ppm_amr* a) {
  if (!a) return PPM_OK;
  (void)hipFree(a->d_idesc);
  (void)hipFree(a->d_istart);
  (void)hipFree(a->d_adesc);
  (void)hipFree(a->d_astart);
  (void)hipFree(a->d_faces);
  (void)hipFree(a->d_cgl);
  (void)hipFree(a->d_fgl);
  (void)hipFree(a->d_reg);
  (void)hipFree(a->d_dt);
  delete a;
  return PPM_OK;
}

const char* ppm_amr_last_error(const ppm_amr* a) { return a ? a->err.c_str() : "null hierarchy"; }

int ppm_amr_sizes(const ppm_amr* a, int64_t* interp_zones, int64_t* register_faces, int64_t* covered_zones) {
  if (!a) return PPM_EINVAL;
  if (interp_zones) *interp_zones = a->istart.back();
  if (register_faces) *register_faces = (int64_t)a->faces.size();
  if (covered_zones) *covered_zones = a->astart.back();
  return PPM_OK;
}

int ppm_amr_fill_fine(ppm_amr* a, const double* Uc_old, const double* Uc_new, int32_t half, double* Uf,
                      void* stream) {
  if (!a) return PPM_EINVAL;
  if (!Uc_old || !Uc_new || !Uf) return a->fail(PPM_EINVAL, "amr fill: null state");
  if (half != 0 && half != 1) return a->fail(PPM_EINVAL, "amr fill: half must be 0 or 1");
  hipStream_t s = (hipStream_t)stream;
  int rc = ppm_fill_boundary(a->f, Uf, PPM_LAUNCH_BATCHED, stream);
  if (rc) return rc;
  const int nd = (int)a->idesc.size();
  if (nd == 0) return PPM_OK;
  hipLaunchKernelGGL(k_cf_interp, dim3(grid_for(a->istart.back())), dim3(AMR_THREADS), 0, s, a->d_idesc,
                     a->d_istart, nd, a->c->d_boxes, a->f->d_boxes, a->d_cgl, a->d_fgl, Uc_old, Uc_new,
                     half ? 0.5 : 0.0, Uf);
  return a->hip(hipGetLastError(), "amr interpolation");
}

int ppm_amr_step(ppm_amr* a, const double* Uc, double* Uc_new, double* Uf, double* Uf_tmp, double* const* Fc,
                 double* const* Ff, const double dxc[3], const ppm_params* params, double dt, double* dt_out,
                 void* stream) {
  if (!a) return PPM_EINVAL;
  if (!Uc || !Uc_new || !Uf || !Uf_tmp || !Fc || !Ff || !dxc || !params)
    return a->fail(PPM_EINVAL, "amr step: null argument");
  for (int d = 0; d < 3; ++d)
    if (!Fc[d] || !Ff[d]) return a->fail(PPM_EINVAL, "amr step: the six flux arenas are required");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return a->fail(PPM_EINVAL, "amr step: dt must be >= 0 (0: CFL rule)");
  if (!(params->cfl > 0.0 && params->cfl < 1.0)) return a->fail(PPM_EINVAL, "amr step: cfl must be in (0, 1)");
  const size_t cl = (size_t)a->c->off.back() * sizeof(double), fl = (size_t)a->f->off.back() * sizeof(double);
  if (overlap(Uc, cl, Uc_new, cl) || overlap(Uf, fl, Uf_tmp, fl) || overlap(Uc, cl, Uf, fl) ||
      overlap(Uc, cl, Uf_tmp, fl) || overlap(Uc_new, cl, Uf, fl) || overlap(Uc_new, cl, Uf_tmp, fl))
    return a->fail(PPM_EINVAL, "amr step: state arenas overlap");
  hipStream_t s = (hipStream_t)stream;
  const double dxf[3] = {0.5 * dxc[0], 0.5 * dxc[1], 0.5 * dxc[2]};
  double* Ucm = const_cast<double*>(Uc);  // ghosts of Uc are filled in place
  int rc;
  // time step
  if ((rc = ppm_fill_boundary(a->c, Ucm, PPM_LAUNCH_BATCHED, stream))) return rc;
  if (dt == 0.0) {
    if ((rc = ppm_compute_dt(a->c, Uc, dxc, params, a->d_dt, stream))) return rc;
    if ((rc = ppm_compute_dt(a->f, Uf, dxf, params, a->d_dt + 2, stream))) return rc;
  }
  hipLaunchKernelGGL(k_amr_dt, dim3(1), dim3(64), 0, s, a->d_dt, params->cfl, dt);
  if ((rc = a->hip(hipGetLastError(), "amr dt"))) return rc;
  // coarse step with its fluxes, then the new coarse ghosts (for the time
  // interpolation)
  if ((rc = ppm_hydro_step(a->c, Uc, Uc_new, Fc, 0.0, a->d_dt + 4, dxc, params, PPM_LAUNCH_BATCHED, stream)))
    return rc;
  if ((rc = ppm_fill_boundary(a->c, Uc_new, PPM_LAUNCH_BATCHED, stream))) return rc;
  const int nf = (int)a->faces.size();
  const long long nreg = 5LL * nf;
  if (nf > 0) hipLaunchKernelGGL(k_reg_zero, dim3(grid_for(nreg)), dim3(AMR_THREADS), 0, s, a->d_reg, nreg);
  // two fine steps: Uf -> Uf_tmp -> Uf
  for (int k = 0; k < 2; ++k) {
    double* src = k == 0 ? Uf : Uf_tmp;
    double* dst = k == 0 ? Uf_tmp : Uf;
    if ((rc = ppm_amr_fill_fine(a, Uc, Uc_new, k, src, stream))) return rc;
    if ((rc = ppm_hydro_step(a->f, src, dst, Ff, 0.0, a->d_dt + 5, dxf, params, PPM_LAUNCH_BATCHED, stream)))
      return rc;
    if (nf > 0)
      hipLaunchKernelGGL(k_reg_accum, dim3(grid_for(nf)), dim3(AMR_THREADS), 0, s, a->d_faces, nf, a->f->d_boxes,
                         Ff[0], Ff[1], Ff[2], a->d_reg);
  }
  // synchronisation
  if (nf > 0)
    hipLaunchKernelGGL(k_reflux, dim3(grid_for(nf)), dim3(AMR_THREADS), 0, s, a->d_faces, nf, a->c->d_boxes,
                       Fc[0], Fc[1], Fc[2], a->d_reg, a->c->d_consts, Uc_new);
  const int na = (int)a->adesc.size();
  if (na > 0)
    hipLaunchKernelGGL(k_avg_down, dim3(grid_for(a->astart.back())), dim3(AMR_THREADS), 0, s, a->d_adesc,
                       a->d_astart, na, a->c->d_boxes, a->f->d_boxes, a->d_cgl, a->d_fgl, Uf, Uc_new);
  if (dt_out) hipLaunchKernelGGL(k_copy2, dim3(1), dim3(64), 0, s, a->d_dt + 4, dt_out);
  return a->hip(hipGetLastError(), "amr synchronisation");
}

}  // extern "C"
