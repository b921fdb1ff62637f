// Host runtime and C ABI (include/ksc.h): problem object, metric and symbol
// tables, tile lists, launch policy, FP64 cost finalization, descent loop
// captured as HIP graphs, launch-shape tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ksc.h"
#include "ksc_launch.hpp"
#include "ksc_launch_odd.hpp"
#include "ksc_launch_spec.hpp"
#include "ksc_launch_simp.hpp"

using ksc::cplx;
using ksc::CurveDev;
using ksc::KernelArgs;
using ksc::SpecDev;
using ksc::TileDev;

namespace {

thread_local std::string g_err;

ksc_status fail(ksc_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define KSC_HIP(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(KSC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

bool nx_supported(int nx) {
  return nx == 8 || nx == 16 || nx == 32 || nx == 64 || nx == 128 || nx == 256;
}
int modes_of(int nx) { return (nx - 1) / 3 + 1; }

// ---------------------------------------------------------------- kernels --

__global__ void precond_kernel(int n, const float* A, float* pre, float dtau) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pre[i] = -dtau / (1.0f + dtau * A[i] * A[i]);
}
__global__ void precond_kernel_d(int n, const double* A, double* pre, double dtau) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pre[i] = -dtau / (1.0 + dtau * A[i] * A[i]);
}

__device__ __forceinline__ bool finite_bits(double v) {
  unsigned long long b = __double_as_longlong(v);
  return ((b >> 52) & 0x7ffull) != 0x7ffull;
}

// Tile boundary after tile t: row L = last row of tile t and F = L + 1 =
// first row of tile t + 1 of the same curve.  offL < 0: nothing to finish
// (last tile of a curve, or L or F is a pinned end row).  The row-table
// values are stored as doubles that are exact in the run dtype.
struct BoundDev {
  long long offL;  // state offset (complex elements) of row L; row F follows
  int c, km, mode_off, pad_;
  double csL, csF, wlL, wlF;  // g/(2 dsigma) and 2 w L of rows L and F
};

template <typename T>
struct PostArgs {
  int nc;
  const CurveDev* curves;
  const BoundDev* bounds;
  int n_tiles;
  const double* partials;
  int part_stride;       // as in KernelArgs
  const double* sqrtL;
  double* J2;            // nullable
  double* Jarc;          // nullable
  double* prevJ2;
  unsigned* flags;
  unsigned char* rose;   // with track: 1 where the cost rose against the previous evaluation
  const unsigned char* active;
  int track;
  int fin_blocks;        // blocks [0, fin_blocks): one wave per curve reduces its cost
  int mode;              // MODE_GRAD / MODE_STEP: finish the tile-boundary rows
  int odd;               // rows of K reals (inversion-symmetric subspace), modes 1..K
  int waves;
  int km_max;
  const cplx<T>* edge;
  const cplx<T>* in;
  cplx<T>* out;
  const T* pre;
  const double* scale;
};

// Fixed-shape butterfly sum over a wave: every lane ends with the same value,
// and the order of additions does not depend on timing (deterministic).
__device__ __forceinline__ double wave_sum_fixed(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Runs after every fused launch (256 threads per block).
//  * blocks [0, fin_blocks): one block per curve loads its tiles' FP64
//    partials in parallel (thread i takes slots i, i+256, ...) and sums them
//    with a fixed reduction tree into J2 and J_arc = sqrt(L) num/den; raises
//    the curve's flags (non-finite cost; with track, a rise of the cost).
//  * the other blocks: one thread per (tile boundary, mode) completes the two
//    boundary rows L | F = L+1 of a curve, whose neighbouring residual row was
//    computed by the other tile:  adj_L += cs_L r_F,  adj_F -= cs_F r_L, and
//    writes the gradient or the stepped state of both rows.
template <typename T>
__global__ __launch_bounds__(256) void post_kernel(PostArgs<T> a) {
  if (int(blockIdx.x) < a.fin_blocks) {
    const int c = blockIdx.x;
    if (a.active != nullptr && a.active[c] == 0) return;
    double s0 = 0, s1 = 0, s2 = 0;
    long long first;
    int nw;  // one partial triple per wave of each tile
    if (a.part_stride > 0) {
      // fixed stride: no descriptor read; slots past the curve's tiles hold 0
      first = (long long)c * a.part_stride;
      nw = a.part_stride;
    } else {
      const CurveDev cd = a.curves[c];
      first = (long long)cd.tile_begin * a.waves;
      nw = cd.n_tiles * a.waves;
    }
    // thread i adds the slots i, i + 256, ... in that order, four loads in
    // flight at a time
    for (int t0 = threadIdx.x; t0 < nw; t0 += 1024) {
      double v[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + 256 * u;
        const double* p = a.partials + 3 * (first + t);
        v[u][0] = (t < nw) ? p[0] : 0.0;
        v[u][1] = (t < nw) ? p[1] : 0.0;
        v[u][2] = (t < nw) ? p[2] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s0 += v[u][0];
        s1 += v[u][1];
        s2 += v[u][2];
      }
    }
    s0 = wave_sum_fixed(s0);
    s1 = wave_sum_fixed(s1);
    s2 = wave_sum_fixed(s2);
    // the four wave sums, added in a fixed order
    __shared__ double wsum[4][3];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      wsum[wv][0] = s0;
      wsum[wv][1] = s1;
      wsum[wv][2] = s2;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    s0 = (wsum[0][0] + wsum[1][0]) + (wsum[2][0] + wsum[3][0]);
    s1 = (wsum[0][1] + wsum[1][1]) + (wsum[2][1] + wsum[3][1]);
    s2 = (wsum[0][2] + wsum[1][2]) + (wsum[2][2] + wsum[3][2]);
    if (a.J2) a.J2[c] = s0;
    if (a.Jarc) a.Jarc[c] = (s2 > 0) ? a.sqrtL[c] * s1 / s2 : 0.0;
    unsigned f = 0;
    if (!finite_bits(s0)) f |= KSC_FLAG_NONFINITE;
    if (a.track) {
      const double pv = a.prevJ2[c];
      const bool up = finite_bits(pv) && pv >= 0 && s0 > pv * (1.0 + 1e-12) + 1e-300;
      if (up) f |= KSC_FLAG_INCREASED;
      a.rose[c] = up ? 1 : 0;
      a.prevJ2[c] = s0;
    }
    if (f) a.flags[c] |= f;
    return;
  }
  const long long g = (long long)(blockIdx.x - a.fin_blocks) * blockDim.x + threadIdx.x;
  const int t = int(g / a.km_max), k = int(g % a.km_max);
  if (t >= a.n_tiles - 1) return;
  if (a.odd) {
    // element k of a row is mode k + 1; every kept mode has c_k = 2
    const BoundDev b = a.bounds[t];
    const long long km = a.km_max;
    const T* edge = reinterpret_cast<const T*>(a.edge);
    const T pL = edge[(t * 4ll + 2) * km + k], rL = edge[(t * 4ll + 3) * km + k];
    const T pF = edge[((t + 1) * 4ll + 0) * km + k], rF = edge[((t + 1) * 4ll + 1) * km + k];
    if (b.offL < 0 || k >= b.km) return;
    if (a.active != nullptr && a.active[b.c] == 0) return;
    const T aL = pL + T(b.csL) * rF, aF = pF - T(b.csF) * rL;
    T* oL = reinterpret_cast<T*>(a.out) + b.offL + k;
    T* oF = oL + b.km;
    if (a.mode == ksc::MODE_GRAD) {
      const T sc = a.scale ? T(a.scale[b.c]) : T(1);
      *oL = (T(2) * (T(b.wlL) * sc)) * aL;
      *oF = (T(2) * (T(b.wlF) * sc)) * aF;
    } else {
      const T pk = a.pre[b.mode_off + k + 1];
      const T* in = reinterpret_cast<const T*>(a.in);
      *oL = in[b.offL + k] + pk * aL;
      *oF = in[b.offL + b.km + k] + pk * aF;
    }
    return;
  }
  // every load below depends only on (t, k): one round trip to memory
  const BoundDev b = a.bounds[t];
  const long long km = a.km_max;
  const cplx<T> pL = a.edge[(t * 4ll + 2) * km + k], rL = a.edge[(t * 4ll + 3) * km + k];
  const cplx<T> pF = a.edge[((t + 1) * 4ll + 0) * km + k], rF = a.edge[((t + 1) * 4ll + 1) * km + k];
  if (b.offL < 0 || k >= b.km) return;
  if (a.active != nullptr && a.active[b.c] == 0) return;
  const T csL = T(b.csL), csF = T(b.csF);
  const T aLr = pL.r + csL * rF.r, aLi = pL.i + csL * rF.i;
  const T aFr = pF.r - csF * rL.r, aFi = pF.i - csF * rL.i;
  cplx<T>* oL = a.out + b.offL + k;
  cplx<T>* oF = oL + b.km;
  if (a.mode == ksc::MODE_GRAD) {
    const T sc = a.scale ? T(a.scale[b.c]) : T(1);
    const T ck = (k == 0) ? T(1) : T(2);
    const T fL = ck * T(b.wlL) * sc, fF = ck * T(b.wlF) * sc;
    *oL = cplx<T>{fL * aLr, (k == 0) ? T(0) : fL * aLi};
    *oF = cplx<T>{fF * aFr, (k == 0) ? T(0) : fF * aFi};
  } else {
    const T pk = a.pre[b.mode_off + k];
    const cplx<T> xL = a.in[b.offL + k];
    const cplx<T> xF = a.in[b.offL + b.km + k];
    *oL = cplx<T>{xL.r + pk * aLr, (k == 0) ? T(0) : xL.i + pk * aLi};
    *oF = cplx<T>{xF.r + pk * aFr, (k == 0) ? T(0) : xF.i + pk * aFi};
  }
}

}  // namespace

// ----------------------------------------------------------------- problem --

struct ksc_problem {
  int nc = 0;
  int dtype = KSC_F32;
  int space = KSC_SPACE_FULL;
  int ds = KSC_DS_STENCIL;
  hipStream_t stream = nullptr;
  int device = 0;
  size_t lds_limit = 65536;
  int n_cu = 256;

  std::vector<ksc_curve_desc> desc;
  std::vector<CurveDev> cd;
  std::vector<TileDev> tiles;
  std::vector<int> curve_order;  // curves in tile-list order (largest n_x first)
  long long numel_c = 0;         // state elements (complex; real in the odd subspace)
  long long phys_numel = 0;
  int rows_total = 0, modes_total = 0;
  int max_nx = 0, min_nx = 1 << 30;
  bool uniform = true;
  bool mixed_ok = true;  // every n_x in {32, 64, 128}

  int policy = KSC_LAUNCH_AUTO;
  int W = 1;

  // device workspace
  CurveDev* d_cd = nullptr;
  TileDev* d_tiles = nullptr;
  BoundDev* d_bounds = nullptr;
  std::vector<double> h_cs, h_wl2;  // per-row tables (host copies, FP64)
  void* d_cs = nullptr;
  void* d_wlT = nullptr;
  double* d_wlD = nullptr;
  void* d_A = nullptr;
  void* d_edge = nullptr;
  int km_max = 0;
  void* d_pre = nullptr;
  double* d_sqrtL = nullptr;
  double* d_part = nullptr;
  int part_stride = 0;        // see KernelArgs::part_stride
  long long part_slots = 0;   // allocated partial slots (3 doubles each)
  double* d_prevJ2 = nullptr;
  unsigned* d_flags = nullptr;
  unsigned char* d_rose = nullptr;  // per curve: the last tracked cost rose (momentum restart)
  double* d_J2 = nullptr;
  int part_cap = 0;
  double pre_dtau = std::nan("");

  // spectral d/ds: D~ = S D_t per distinct n_s, per-curve descriptors ordered
  // by (n_x, n_s), one group of curves per (n_x, n_s), and three state-sized
  // work arrays
  void* d_dpool = nullptr;
  SpecDev* d_spec = nullptr;
  struct SpecGroup {
    int nx, first, count, n_s;
  };
  std::vector<SpecGroup> spec_groups;
  // one product launch per n_x over its groups (device table d_sgroups)
  struct SpecLaunch {
    int nx, gfirst, ngroups, n_blocks;
    int kparts;  // parts of the k range (small launches split k to fill the chip)
    int nk_max;  // k steps of the group with the largest n_s
  };
  std::vector<SpecLaunch> spec_launches;
  ksc::SpecGroupDev* d_sgroups = nullptr;
  double* d_kpart = nullptr;  // split-k partial products: [max kparts][state scalars]
  void* d_Y = nullptr;
  void* d_WR = nullptr;
  void* d_P = nullptr;

  // descent scheme (ksc_set_scheme); the implicit-in-s step keeps the
  // gradient in d_G and walks the solve table d_simp
  int scheme = KSC_SCHEME_PAPER;
  double momentum = 0.0;  // heavy-ball momentum of the implicit-in-s descent (ksc_set_momentum)
  void* d_G = nullptr;
  void* d_zero = nullptr;  // a zero state: the base of ksc_precondition's solve
  ksc::SimpBlock* d_simp = nullptr;
  int n_simp = 0;
  int simp_chunk = 16;

  // descent graph cache
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  struct Key {
    void* state = nullptr;
    void* scratch = nullptr;
    double dtau = 0;
    int every = 0;
    const void* active = nullptr;
    int W = 0, policy = 0;
    double momentum = 0;
    hipStream_t stream = nullptr;
  } gkey;

  // kernel timing (ksc_set_timing): four events per evaluation, stamped by
  // the fused tile kernel's and the post kernel's dispatches
  bool timing = false;
  bool timing_overflow = false;
  std::vector<hipEvent_t> tev;
  size_t tev_used = 0;

  size_t esize() const { return dtype == KSC_F64 ? 8 : 4; }
  bool odd() const { return space == KSC_SPACE_ODD; }
  bool spectral() const { return ds == KSC_DS_SPECTRAL; }
  // bytes of one state element, elements per row of curve d, whole-state bytes
  size_t elem_bytes() const { return odd() ? esize() : 2 * esize(); }
  int row_elems(const CurveDev& d) const { return odd() ? d.km - 1 : d.km; }
  size_t state_bytes() const { return size_t(numel_c) * elem_bytes(); }
};

namespace {

// Lanes per row (mirrors lanes_per_row<NX, T>() of the kernels) and rows per
// tile of W waves for grid size nx.
int lanes_per_row(const ksc_problem* p, int nx) {
  if (p->odd() || p->spectral()) return 1;
  if (p->esize() == 4 && nx == 256) return ksc::kLanesF32N256;  // tile_body_lanes
  return nx * int(p->esize()) > 512 ? 2 : 1;
}
int rows_per_tile(const ksc_problem* p, int W, int nx) { return 64 * W / lanes_per_row(p, nx); }

// LDS staging buffer of one tile: rows j0-1 .. j0+R, 16 bytes of alignment slack.
size_t lds_for(const ksc_problem* p, int W, int nx) {
  if (p->spectral()) {  // state rows and d/ds rows of the tile, each with slack
    const size_t cs = p->elem_bytes(), E = 16 / cs;
    const size_t per_row = p->odd() ? modes_of(nx) - 1 : modes_of(nx);
    return 2 * (size_t(rows_per_tile(p, W, nx)) * per_row + 2 * E) * cs;
  }
  // (odd subspace: the last 16-byte chunk of a staged block may start up to
  // 16 bytes past the block and end 16 bytes after that)
  if (p->odd()) return size_t(rows_per_tile(p, W, nx) + 2) * (modes_of(nx) - 1) * p->esize() + 32;
  if (lanes_per_row(p, nx) > 2)
    return size_t(ksc::lanes_lds_bytes(nx, modes_of(nx), rows_per_tile(p, W, nx),
                                       lanes_per_row(p, nx), int(p->esize())));
  const size_t cs = 2 * p->esize();
  // plus the samples of u that each lane parks in LDS between the passes
  // (ksc::u_stash of the tile kernels)
  const size_t park = size_t(64 * W) * ksc::u_stash_n(nx, int(p->esize())) * p->esize();
  return (size_t(rows_per_tile(p, W, nx) + 2) * modes_of(nx) + 2) * cs + park;
}
// Largest staging buffer over the grid sizes of the problem (one launch may
// serve several).
size_t lds_max(const ksc_problem* p, int W) {
  size_t m = 0;
  for (int nx : {8, 16, 32, 64, 128, 256})
    if (nx >= p->min_nx && nx <= p->max_nx) m = std::max(m, lds_for(p, W, nx));
  return m;
}

// Largest W in {4, 2, 1} (at most `cap`) whose staging buffers fit in LDS.
int fit_W(const ksc_problem* p, int cap) {
  for (int W : {4, 2, 1})
    if (W <= cap && lds_max(p, W) <= p->lds_limit) return W;
  return 0;
}

int default_W(const ksc_problem* p) {
  // The widest tile that fits: 256 rows per tile keeps the tile count of a
  // 1024-row curve at exactly 4.
  return fit_W(p, 4);
}

ksc_status build_tiles(ksc_problem* p) {
  p->tiles.clear();
  for (int c : p->curve_order) {
    CurveDev& d = p->cd[c];
    const int R = rows_per_tile(p, p->W, d.n_x);
    const int nt = (d.n_s + R - 1) / R;
    d.tile_begin = int(p->tiles.size());
    d.n_tiles = nt;
    for (int i = 0; i < nt; ++i) p->tiles.push_back(TileDev{c, i * R});
  }
  // boundary descriptors, one per tile (values rounded to the run dtype)
  std::vector<BoundDev> bounds(p->tiles.size());
  auto rt = [&](double v) { return p->dtype == KSC_F64 ? v : double(float(v)); };
  for (size_t t = 0; t < p->tiles.size(); ++t) {
    BoundDev& b = bounds[t];
    b = BoundDev{-1, 0, 0, 0, 0, 0.0, 0.0, 0.0, 0.0};
    if (t + 1 >= p->tiles.size() || p->tiles[t + 1].curve != p->tiles[t].curve) continue;
    const CurveDev& d = p->cd[p->tiles[t].curve];
    const int L = p->tiles[t].j0 + rows_per_tile(p, p->W, d.n_x) - 1, F = L + 1;
    if (!(L >= 1 && F <= d.n_s - 2)) continue;
    b.offL = d.off + (long long)L * p->row_elems(d);
    b.c = p->tiles[t].curve;
    b.km = p->row_elems(d);
    b.mode_off = d.mode_off;
    b.csL = rt(p->h_cs[d.row_off + L]);
    b.csF = rt(p->h_cs[d.row_off + F]);
    b.wlL = rt(p->h_wl2[d.row_off + L]);
    b.wlF = rt(p->h_wl2[d.row_off + F]);
  }
  if (p->d_tiles) hipFree(p->d_tiles);
  if (p->d_bounds) hipFree(p->d_bounds);
  p->d_tiles = nullptr;
  p->d_bounds = nullptr;
  KSC_HIP(hipMalloc(&p->d_tiles, p->tiles.size() * sizeof(TileDev)));
  KSC_HIP(hipMemcpy(p->d_tiles, p->tiles.data(), p->tiles.size() * sizeof(TileDev),
                    hipMemcpyHostToDevice));
  KSC_HIP(hipMalloc(&p->d_bounds, bounds.size() * sizeof(BoundDev)));
  KSC_HIP(hipMemcpy(p->d_bounds, bounds.data(), bounds.size() * sizeof(BoundDev),
                    hipMemcpyHostToDevice));
  KSC_HIP(hipMemcpy(p->d_cd, p->cd.data(), p->cd.size() * sizeof(CurveDev),
                    hipMemcpyHostToDevice));
  if (int(p->tiles.size()) > p->part_cap) {
    if (p->d_edge) hipFree(p->d_edge);
    p->d_edge = nullptr;
    p->part_cap = int(p->tiles.size());
    KSC_HIP(hipMalloc(&p->d_edge, size_t(p->part_cap) * 4 * p->km_max * 2 * p->esize()));
  }
  // partial-sum slots: per curve at a fixed stride unless that would take
  // far more memory than the tile-ordered layout
  int max_w = 0;
  for (const CurveDev& d : p->cd) max_w = std::max(max_w, d.n_tiles * p->W);
  const long long compact = (long long)p->tiles.size() * p->W;
  const long long strided = (long long)p->nc * max_w;
  p->part_stride = (strided <= 4 * compact + 65536) ? max_w : 0;
  const long long need = p->part_stride > 0 ? strided : compact;
  if (need > p->part_slots) {
    if (p->d_part) hipFree(p->d_part);
    p->d_part = nullptr;
    p->part_slots = need;
    KSC_HIP(hipMalloc(&p->d_part, 3 * sizeof(double) * size_t(need)));
  }
  // slots past a curve's tiles must read as 0 (stream-ordered after any
  // evaluation already enqueued)
  KSC_HIP(hipMemsetAsync(p->d_part, 0, 3 * sizeof(double) * size_t(need), p->stream));
  return KSC_OK;
}

void drop_graph(ksc_problem* p) {
  if (p->gexec) hipGraphExecDestroy(p->gexec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
}

template <typename T>
hipError_t launch_uniform(int nx, int W, int mode, int grid, size_t lds, hipStream_t s,
                          const KernelArgs<T>& a, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_odd(int nx, int W, int mode, int grid, size_t lds, hipStream_t s,
                      const KernelArgs<T>& a, hipEvent_t e0, hipEvent_t e1);

template <>
hipError_t launch_odd<float>(int nx, int W, int mode, int grid, size_t lds, hipStream_t s,
                             const KernelArgs<float>& a, hipEvent_t e0, hipEvent_t e1) {
  switch (nx) {
    case 8: return ksc::launch_odd_f32_8(W, mode, grid, lds, s, a, e0, e1);
    case 16: return ksc::launch_odd_f32_16(W, mode, grid, lds, s, a, e0, e1);
    case 32: return ksc::launch_odd_f32_32(W, mode, grid, lds, s, a, e0, e1);
    case 64: return ksc::launch_odd_f32_64(W, mode, grid, lds, s, a, e0, e1);
    case 128: return ksc::launch_odd_f32_128(W, mode, grid, lds, s, a, e0, e1);
    default: return ksc::launch_odd_f32_256(W, mode, grid, lds, s, a, e0, e1);
  }
}
template <>
hipError_t launch_odd<double>(int nx, int W, int mode, int grid, size_t lds, hipStream_t s,
                              const KernelArgs<double>& a, hipEvent_t e0, hipEvent_t e1) {
  switch (nx) {
    case 8: return ksc::launch_odd_f64_8(W, mode, grid, lds, s, a, e0, e1);
    case 16: return ksc::launch_odd_f64_16(W, mode, grid, lds, s, a, e0, e1);
    case 32: return ksc::launch_odd_f64_32(W, mode, grid, lds, s, a, e0, e1);
    case 64: return ksc::launch_odd_f64_64(W, mode, grid, lds, s, a, e0, e1);
    case 128: return ksc::launch_odd_f64_128(W, mode, grid, lds, s, a, e0, e1);
    default: return ksc::launch_odd_f64_256(W, mode, grid, lds, s, a, e0, e1);
  }
}

template <>
hipError_t launch_uniform<float>(int nx, int W, int mode, int grid, size_t lds, hipStream_t s,
                                 const KernelArgs<float>& a, hipEvent_t e0, hipEvent_t e1) {
  switch (nx) {
    case 8: return ksc::launch_fused_f32_8(W, mode, grid, lds, s, a, e0, e1);
    case 16: return ksc::launch_fused_f32_16(W, mode, grid, lds, s, a, e0, e1);
    case 32: return ksc::launch_fused_f32_32(W, mode, grid, lds, s, a, e0, e1);
    case 64: return ksc::launch_fused_f32_64(W, mode, grid, lds, s, a, e0, e1);
    case 128: return ksc::launch_fused_f32_128(W, mode, grid, lds, s, a, e0, e1);
    default: return ksc::launch_fused_f32_256(W, mode, grid, lds, s, a, e0, e1);
  }
}
template <>
hipError_t launch_uniform<double>(int nx, int W, int mode, int grid, size_t lds, hipStream_t s,
                                  const KernelArgs<double>& a, hipEvent_t e0, hipEvent_t e1) {
  switch (nx) {
    case 8: return ksc::launch_fused_f64_8(W, mode, grid, lds, s, a, e0, e1);
    case 16: return ksc::launch_fused_f64_16(W, mode, grid, lds, s, a, e0, e1);
    case 32: return ksc::launch_fused_f64_32(W, mode, grid, lds, s, a, e0, e1);
    case 64: return ksc::launch_fused_f64_64(W, mode, grid, lds, s, a, e0, e1);
    case 128: return ksc::launch_fused_f64_128(W, mode, grid, lds, s, a, e0, e1);
    default: return ksc::launch_fused_f64_256(W, mode, grid, lds, s, a, e0, e1);
  }
}
hipError_t launch_mixed(const KernelArgs<float>& a, int W, int mode, int grid, size_t lds,
                        hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return ksc::launch_mixed_f32(W, mode, grid, lds, s, a, e0, e1);
}
hipError_t launch_mixed(const KernelArgs<double>& a, int W, int mode, int grid, size_t lds,
                        hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return ksc::launch_mixed_f64(W, mode, grid, lds, s, a, e0, e1);
}

template <typename T>
KernelArgs<T> make_args(ksc_problem* p, const void* in, void* out, const double* scale,
                        const uint8_t* active) {
  KernelArgs<T> a{};
  a.in = static_cast<const cplx<T>*>(in);
  a.out = static_cast<cplx<T>*>(out);
  a.curves = p->d_cd;
  a.tiles = p->d_tiles;
  a.cs = static_cast<const T*>(p->d_cs);
  a.wlT = static_cast<const T*>(p->d_wlT);
  a.wlD = p->d_wlD;
  a.pre = static_cast<const T*>(p->d_pre);
  a.scale = scale;
  a.active = active;
  a.partials = p->d_part;
  a.part_stride = p->part_stride;
  a.edge = static_cast<cplx<T>*>(p->d_edge);
  a.km_max = p->km_max;
  a.n_tiles = int(p->tiles.size());
  a.tile_base = 0;
  return a;
}

// Enqueue the fused kernel(s) for `mode` on stream s according to the policy.
// ev (nullable) = {start, stop}: the first launch stamps start when it
// begins, the last one stop when it ends.
template <typename T>
ksc_status launch_fused(ksc_problem* p, int mode, const void* in, void* out, const double* scale,
                        const uint8_t* active, hipStream_t s, const hipEvent_t* ev) {
  KernelArgs<T> a = make_args<T>(p, in, out, scale, active);
  const int W = p->W;
  hipEvent_t e_first = ev ? ev[0] : nullptr, e_last = ev ? ev[1] : nullptr;
  auto launch_nx = [&](int nx, int grid, size_t lds, const KernelArgs<T>& ag, hipEvent_t e0,
                       hipEvent_t e1) {
    return p->odd() ? launch_odd<T>(nx, W, mode, grid, lds, s, ag, e0, e1)
                    : launch_uniform<T>(nx, W, mode, grid, lds, s, ag, e0, e1);
  };
  if (p->policy == KSC_LAUNCH_PLAIN) {
    for (int c = 0; c < p->nc; ++c) {
      const CurveDev& d = p->cd[c];
      KernelArgs<T> ac = a;
      ac.tile_base = d.tile_begin;
      ac.n_tiles = d.n_tiles;
      const size_t lds = lds_for(p, W, d.n_x);
      hipError_t e = launch_nx(d.n_x, d.n_tiles, lds, ac, c == 0 ? e_first : nullptr,
                               c == p->nc - 1 ? e_last : nullptr);
      if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
    }
    return KSC_OK;
  }
  const int nt = int(p->tiles.size());
  int grid = nt;
  if (p->policy == KSC_LAUNCH_PERSISTENT) grid = std::min(nt, p->n_cu * (W == 1 ? 4 : 2));
  if (p->uniform) {
    const size_t lds = lds_for(p, W, p->max_nx);
    hipError_t e = launch_nx(p->max_nx, grid, lds, a, e_first, e_last);
    if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
    return KSC_OK;
  }
  // (the J-only evaluation of a mixed batch runs one launch per grid size: the
  // J-only form of the mixed kernel returned wrong costs on its N_x = 128
  // tiles for a reason not found, while the gradient and step kernels of the
  // same form agree with the oracle on every curve)
  if (p->mixed_ok && mode != ksc::MODE_J) {
    const size_t lds = lds_max(p, W);
    hipError_t e = launch_mixed(a, W, mode, grid, lds, s, e_first, e_last);
    if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
    return KSC_OK;
  }
  // Other mixtures: one launch per distinct n_x over that group's tiles
  // (tiles of a group are contiguous because curves are ordered by n_x).
  int t0 = 0;
  while (t0 < nt) {
    const int nx = p->cd[p->tiles[t0].curve].n_x;
    int t1 = t0;
    while (t1 < nt && p->cd[p->tiles[t1].curve].n_x == nx) ++t1;
    KernelArgs<T> ag = a;
    ag.tile_base = t0;
    ag.n_tiles = t1 - t0;
    const size_t lds = lds_for(p, W, nx);
    hipError_t e = launch_nx(nx, t1 - t0, lds, ag, t0 == 0 ? e_first : nullptr,
                             t1 == nt ? e_last : nullptr);
    if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
    t0 = t1;
  }
  return KSC_OK;
}

template <typename T>
ksc_status launch_post(ksc_problem* p, int mode, const void* in, void* out, const double* scale,
                       const uint8_t* active, double* J2, double* Jarc, int track,
                       bool finalize, hipStream_t s, const hipEvent_t* ev) {
  PostArgs<T> a{};
  a.nc = p->nc;
  a.curves = p->d_cd;
  a.bounds = p->d_bounds;
  a.n_tiles = int(p->tiles.size());
  a.partials = p->d_part;
  a.part_stride = p->part_stride;
  a.sqrtL = p->d_sqrtL;
  a.J2 = J2;
  a.Jarc = Jarc;
  a.prevJ2 = p->d_prevJ2;
  a.flags = p->d_flags;
  a.rose = p->d_rose;
  a.active = active;
  a.track = track;
  const int b = 256;
  a.fin_blocks = finalize ? p->nc : 0;
  a.mode = mode;
  a.odd = p->odd() ? 1 : 0;
  a.waves = p->W;
  a.km_max = p->km_max;
  a.edge = static_cast<const cplx<T>*>(p->d_edge);
  a.in = static_cast<const cplx<T>*>(in);
  a.out = static_cast<cplx<T>*>(out);
  a.pre = static_cast<const T*>(p->d_pre);
  a.scale = scale;
  const long long nfix = (mode == ksc::MODE_J) ? 0 : (long long)a.n_tiles * p->km_max;
  const int fix_blocks = int((nfix + b - 1) / b);
  const int grid = a.fin_blocks + fix_blocks;
  if (grid == 0) {
    // nothing to do: keep the timing pair well formed
    if (ev) {
      KSC_HIP(hipEventRecord(ev[0], s));
      KSC_HIP(hipEventRecord(ev[1], s));
    }
    return KSC_OK;
  }
  hipExtLaunchKernelGGL(post_kernel<T>, dim3(grid), dim3(b), 0, s, ev ? ev[0] : nullptr,
                        ev ? ev[1] : nullptr, 0, a);
  KSC_HIP(hipGetLastError());
  return KSC_OK;
}

// ------------------------------------------------------- spectral d/ds --

hipError_t spec_gemm(int nx, int odd, int epi, const ksc::SpecGroupDev* g, int ng, int nb,
                     hipStream_t s, const ksc::SpecArgs<float>& a, hipEvent_t e0, hipEvent_t e1) {
  switch (nx) {
    case 8: return ksc::launch_spec_gemm_f32_8(odd, epi, g, ng, nb, s, a, e0, e1);
    case 16: return ksc::launch_spec_gemm_f32_16(odd, epi, g, ng, nb, s, a, e0, e1);
    case 32: return ksc::launch_spec_gemm_f32_32(odd, epi, g, ng, nb, s, a, e0, e1);
    case 64: return ksc::launch_spec_gemm_f32_64(odd, epi, g, ng, nb, s, a, e0, e1);
    case 128: return ksc::launch_spec_gemm_f32_128(odd, epi, g, ng, nb, s, a, e0, e1);
    default: return hipErrorInvalidValue;
  }
}
hipError_t spec_gemm(int nx, int odd, int epi, const ksc::SpecGroupDev* g, int ng, int nb,
                     hipStream_t s, const ksc::SpecArgs<double>& a, hipEvent_t e0, hipEvent_t e1) {
  switch (nx) {
    case 8: return ksc::launch_spec_gemm_f64_8(odd, epi, g, ng, nb, s, a, e0, e1);
    case 16: return ksc::launch_spec_gemm_f64_16(odd, epi, g, ng, nb, s, a, e0, e1);
    case 32: return ksc::launch_spec_gemm_f64_32(odd, epi, g, ng, nb, s, a, e0, e1);
    case 64: return ksc::launch_spec_gemm_f64_64(odd, epi, g, ng, nb, s, a, e0, e1);
    default: return hipErrorInvalidValue;
  }
}
hipError_t spec_row(int nx, int odd, int W, int mode, int grid, size_t lds, hipStream_t s,
                    const ksc::SpecRowArgs<float>& a, hipEvent_t e0, hipEvent_t e1) {
  switch (nx) {
    case 8: return ksc::launch_spec_row_f32_8(odd, W, mode, grid, lds, s, a, e0, e1);
    case 16: return ksc::launch_spec_row_f32_16(odd, W, mode, grid, lds, s, a, e0, e1);
    case 32: return ksc::launch_spec_row_f32_32(odd, W, mode, grid, lds, s, a, e0, e1);
    case 64: return ksc::launch_spec_row_f32_64(odd, W, mode, grid, lds, s, a, e0, e1);
    case 128: return ksc::launch_spec_row_f32_128(odd, W, mode, grid, lds, s, a, e0, e1);
    default: return hipErrorInvalidValue;
  }
}
hipError_t spec_row(int nx, int odd, int W, int mode, int grid, size_t lds, hipStream_t s,
                    const ksc::SpecRowArgs<double>& a, hipEvent_t e0, hipEvent_t e1) {
  switch (nx) {
    case 8: return ksc::launch_spec_row_f64_8(odd, W, mode, grid, lds, s, a, e0, e1);
    case 16: return ksc::launch_spec_row_f64_16(odd, W, mode, grid, lds, s, a, e0, e1);
    case 32: return ksc::launch_spec_row_f64_32(odd, W, mode, grid, lds, s, a, e0, e1);
    case 64: return ksc::launch_spec_row_f64_64(odd, W, mode, grid, lds, s, a, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

// One evaluation with the spectral d/ds: Y = D_t U, the row kernel, and (not
// for MODE_J) the transposed product whose epilogue writes the gradient or
// the stepped state.  ev (nullable): start of the first launch, end of the last.
template <typename T>
ksc_status launch_spectral(ksc_problem* p, int mode, const void* in, void* out,
                           const double* scale, const uint8_t* active, hipStream_t s,
                           const hipEvent_t* ev) {
  const int W = p->W;
  const int nl = int(p->spec_launches.size());
  hipEvent_t e_first = ev ? ev[0] : nullptr, e_last = ev ? ev[1] : nullptr;
  ksc::SpecArgs<T> ga{};
  ga.dpool = static_cast<const double*>(p->d_dpool);
  ga.wlT = static_cast<const T*>(p->d_wlT);
  ga.pre = static_cast<const T*>(p->d_pre);
  ga.scale = scale;
  ga.active = active;
  ga.curves = p->d_spec;
  ga.part = p->d_kpart;
  ga.part_stride = (long long)(p->state_bytes() / p->esize());
  // 1. Y = D_t U
  for (int l = 0; l < nl; ++l) {
    const auto& G = p->spec_launches[l];
    ksc::SpecArgs<T> a = ga;
    a.kparts = G.kparts;
    a.b = static_cast<const T*>(in);
    a.out = static_cast<T*>(p->d_Y);
    hipError_t e = spec_gemm(G.nx, p->odd(), ksc::EPI_Y, p->d_sgroups + G.gfirst, G.ngroups,
                             G.n_blocks, s, a, l == 0 ? e_first : nullptr, nullptr);
    if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("spectral product: ") + hipGetErrorString(e));
  }
  // 2. rows: residual, cost partials, row-local adjoint part
  ksc::SpecRowArgs<T> ra{};
  ra.a = make_args<T>(p, in, nullptr, scale, active);
  ra.y = static_cast<const cplx<T>*>(p->d_Y);
  ra.wr = static_cast<cplx<T>*>(p->d_WR);
  ra.pl = static_cast<cplx<T>*>(p->d_P);
  const int nt = int(p->tiles.size());
  int t0 = 0;
  while (t0 < nt) {
    const int nx = p->cd[p->tiles[t0].curve].n_x;
    int t1 = t0;
    while (t1 < nt && p->cd[p->tiles[t1].curve].n_x == nx) ++t1;
    ksc::SpecRowArgs<T> rg = ra;
    rg.a.tile_base = t0;
    rg.a.n_tiles = t1 - t0;
    int grid = t1 - t0;
    if (p->policy == KSC_LAUNCH_PERSISTENT) grid = std::min(grid, p->n_cu * (W == 1 ? 4 : 2));
    const bool last = (mode == ksc::MODE_J) && t1 == nt;
    hipError_t e = spec_row(nx, p->odd(), W, mode == ksc::MODE_J ? ksc::MODE_J : ksc::MODE_GRAD,
                            grid, lds_for(p, W, nx), s, rg, nullptr, last ? e_last : nullptr);
    if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("spectral rows: ") + hipGetErrorString(e));
    t0 = t1;
  }
  if (mode == ksc::MODE_J) return KSC_OK;
  // 3. Z' = D_t^T (2 w L r_hat) and the output
  for (int l = 0; l < nl; ++l) {
    const auto& G = p->spec_launches[l];
    ksc::SpecArgs<T> a = ga;
    a.kparts = G.kparts;
    a.b = static_cast<const T*>(p->d_WR);
    a.p = static_cast<const T*>(p->d_P);
    a.u = static_cast<const T*>(in);
    a.out = static_cast<T*>(out);
    hipError_t e = spec_gemm(G.nx, p->odd(), mode == ksc::MODE_GRAD ? ksc::EPI_GRAD : ksc::EPI_STEP,
                             p->d_sgroups + G.gfirst, G.ngroups, G.n_blocks, s, a, nullptr,
                             l == nl - 1 ? e_last : nullptr);
    if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("spectral product: ") + hipGetErrorString(e));
  }
  return KSC_OK;
}

// D~ = S D_t on n points in the row order used here (row 0 is s = -inf): the
// derivative of the Chebyshev-Gauss-Lobatto interpolant in x = cos(theta)
// times dx/ds = sin^3(theta) / S, i.e. D_t = diag(sin^3 theta / S) D_x with
// D_x[i][j] = (c_i / c_j) (-1)^(i+j) / (x_i - x_j) off the diagonal
// (c_0 = c_N = 2, else 1), the diagonal from the zero row sums, and
// x_i - x_j = -2 sin((i+j) pi / 2N) sin((i-j) pi / 2N).  This is the closed
// form of the sum in eq. rational_diff_matrix (the derivative of the same
// interpolant).
std::vector<double> make_dtilde(int n) {
  const int N = n - 1;
  std::vector<double> Dp(size_t(n) * n, 0.0);  // paper's numbering (i = 0: s = +inf)
  for (int i = 0; i < n; ++i) {
    const double ci = (i == 0 || i == N) ? 2.0 : 1.0;
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double cj = (j == 0 || j == N) ? 2.0 : 1.0;
      const double dx = -2.0 * std::sin((i + j) * M_PI / (2.0 * N)) * std::sin((i - j) * M_PI / (2.0 * N));
      const double v = (ci / cj) * (((i + j) % 2) ? -1.0 : 1.0) / dx;
      Dp[size_t(i) * n + j] = v;
      diag -= v;
    }
    Dp[size_t(i) * n + i] = diag;
    const double sn = std::sin(i * M_PI / N);
    const double f = sn * sn * sn;
    for (int j = 0; j < n; ++j) Dp[size_t(i) * n + j] *= f;
  }
  std::vector<double> D(size_t(n) * n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) D[size_t(a) * n + b] = Dp[size_t(N - a) * n + (N - b)];
  return D;
}

// Matrix pool, per-curve descriptors (tile order) and work arrays.
ksc_status setup_spectral(ksc_problem* p) {
  std::vector<int> sizes;
  for (const CurveDev& d : p->cd) sizes.push_back(d.n_s);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  std::vector<long long> moff(sizes.size());
  long long total = 0;
  for (size_t i = 0; i < sizes.size(); ++i) {
    moff[i] = total;
    total += 2 * (long long)sizes[i] * sizes[i];  // D~, then its transpose
  }
  KSC_HIP(hipMalloc(&p->d_dpool, size_t(total) * sizeof(double)));  // FP64 for both dtypes
  for (size_t i = 0; i < sizes.size(); ++i) {
    const int n = sizes[i];
    std::vector<double> D = make_dtilde(n);
    std::vector<double> DT(D.size());
    for (int r = 0; r < n; ++r)
      for (int q = 0; q < n; ++q) DT[size_t(q) * n + r] = D[size_t(r) * n + q];
    double* dst = static_cast<double*>(p->d_dpool) + moff[i];
    KSC_HIP(hipMemcpy(dst, D.data(), D.size() * 8, hipMemcpyHostToDevice));
    KSC_HIP(hipMemcpy(dst + size_t(n) * n, DT.data(), DT.size() * 8, hipMemcpyHostToDevice));
  }
  std::vector<SpecDev> sd;
  p->spec_groups.clear();
  std::vector<int> order(p->curve_order);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const CurveDev &x = p->cd[a], &y = p->cd[b];
    return x.n_x != y.n_x ? x.n_x > y.n_x : x.n_s < y.n_s;
  });
  for (int c : order) {
    const CurveDev& d = p->cd[c];
    const size_t mi = std::lower_bound(sizes.begin(), sizes.end(), d.n_s) - sizes.begin();
    SpecDev s{};
    s.off = d.off;
    s.dmat = moff[mi];
    s.dmatT = moff[mi] + (long long)d.n_s * d.n_s;
    s.n_s = d.n_s;
    s.km = d.km;
    s.row_off = d.row_off;
    s.mode_off = d.mode_off;
    s.c = c;
    s.inv_S = 1.0 / p->desc[c].scale;
    if (p->spec_groups.empty() || p->spec_groups.back().nx != d.n_x ||
        p->spec_groups.back().n_s != d.n_s)
      p->spec_groups.push_back({d.n_x, int(sd.size()), 0, d.n_s});
    p->spec_groups.back().count++;
    sd.push_back(s);
  }
  KSC_HIP(hipMalloc(&p->d_spec, sd.size() * sizeof(SpecDev)));
  KSC_HIP(hipMemcpy(p->d_spec, sd.data(), sd.size() * sizeof(SpecDev), hipMemcpyHostToDevice));
  // product launches: one per n_x, its groups' workgroups laid end to end
  std::vector<ksc::SpecGroupDev> gd;
  p->spec_launches.clear();
  for (const auto& G : p->spec_groups) {
    if (p->spec_launches.empty() || p->spec_launches.back().nx != G.nx)
      p->spec_launches.push_back({G.nx, int(gd.size()), 0, 0, 1, 0});
    auto& Lh = p->spec_launches.back();
    const int cb = ksc::spec_curves_per_block(G.nx, p->odd());
    const int rb = (G.n_s + ksc::kSpecRowsPerBlock - 1) / ksc::kSpecRowsPerBlock;
    gd.push_back({G.first, G.count, rb, Lh.n_blocks});
    Lh.ngroups++;
    Lh.n_blocks += rb * ((G.count + cb - 1) / cb);
    Lh.nk_max = std::max(Lh.nk_max, (G.n_s + 31) / 32);
  }
  // A launch of fewer than 512 workgroups splits its k range into up to 8
  // parts (at least two k steps of 32 each for the largest n_s): the partial
  // products go to a work array and a second kernel adds them in part order.
  int kmax = 1;
  for (auto& Lh : p->spec_launches) {
    Lh.kparts = 1;
    if (Lh.n_blocks < 512)
      Lh.kparts = std::max(1, std::min({8, (512 + Lh.n_blocks - 1) / Lh.n_blocks, Lh.nk_max / 2}));
    kmax = std::max(kmax, Lh.kparts);
  }
  if (kmax > 1)
    KSC_HIP(hipMalloc(&p->d_kpart, size_t(kmax) * (p->state_bytes() / p->esize()) * sizeof(double)));
  KSC_HIP(hipMalloc(&p->d_sgroups, gd.size() * sizeof(ksc::SpecGroupDev)));
  KSC_HIP(hipMemcpy(p->d_sgroups, gd.data(), gd.size() * sizeof(ksc::SpecGroupDev),
                    hipMemcpyHostToDevice));
  KSC_HIP(hipMalloc(&p->d_Y, p->state_bytes()));
  KSC_HIP(hipMalloc(&p->d_WR, p->state_bytes()));
  KSC_HIP(hipMalloc(&p->d_P, p->state_bytes()));
  return KSC_OK;
}

constexpr size_t kMaxTimedEvals = 1 << 16;

// Next event of the timing pool, or nullptr when the pool is full.
hipEvent_t timing_event(ksc_problem* p) {
  if (p->tev_used == p->tev.size()) {
    if (p->tev.size() >= 4 * kMaxTimedEvals) return nullptr;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->tev.push_back(e);
  }
  return p->tev[p->tev_used++];
}

// One evaluation: the fused tile kernel(s) and the post kernel.  With timing
// on, the dispatches themselves stamp four events: fused start/end, post
// start/end.
ksc_status run(ksc_problem* p, int mode, const void* in, void* out, const double* scale,
               const uint8_t* active, double* J2, double* Jarc, int track, bool finalize,
               hipStream_t s) {
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
  if (p->timing && s == p->stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      if (p->tev_used + 4 > 4 * kMaxTimedEvals) {
        p->timing_overflow = true;
      } else {
        timed = true;
        for (hipEvent_t& e : ev) {
          e = timing_event(p);
          timed = timed && e != nullptr;
        }
        if (!timed) p->timing_overflow = true;
      }
    }
  }
  const hipEvent_t* evf = timed ? ev : nullptr;
  const hipEvent_t* evp = timed ? ev + 2 : nullptr;
  ksc_status st;
  if (p->spectral()) {
    // the post kernel only reduces the cost (no tile-boundary rows to finish)
    if (p->dtype == KSC_F64) {
      st = launch_spectral<double>(p, mode, in, out, scale, active, s, evf);
      if (st == KSC_OK)
        st = launch_post<double>(p, ksc::MODE_J, in, out, scale, active, J2, Jarc, track, finalize,
                                 s, evp);
    } else {
      st = launch_spectral<float>(p, mode, in, out, scale, active, s, evf);
      if (st == KSC_OK)
        st = launch_post<float>(p, ksc::MODE_J, in, out, scale, active, J2, Jarc, track, finalize,
                                s, evp);
    }
  } else if (p->dtype == KSC_F64) {
    st = launch_fused<double>(p, mode, in, out, scale, active, s, evf);
    if (st == KSC_OK)
      st = launch_post<double>(p, mode, in, out, scale, active, J2, Jarc, track, finalize, s, evp);
  } else {
    st = launch_fused<float>(p, mode, in, out, scale, active, s, evf);
    if (st == KSC_OK)
      st = launch_post<float>(p, mode, in, out, scale, active, J2, Jarc, track, finalize, s, evp);
  }
  if (st != KSC_OK && timed) p->tev_used -= 4;  // drop an incomplete record
  return st;
}

ksc_status ensure_pre(ksc_problem* p, double dtau, hipStream_t s) {
  if (p->pre_dtau == dtau) return KSC_OK;
  const int n = p->modes_total, b = 256, g = (n + b - 1) / b;
  if (p->dtype == KSC_F64)
    hipLaunchKernelGGL(precond_kernel_d, dim3(g), dim3(b), 0, s, n,
                       static_cast<const double*>(p->d_A), static_cast<double*>(p->d_pre), dtau);
  else
    hipLaunchKernelGGL(precond_kernel, dim3(g), dim3(b), 0, s, n,
                       static_cast<const float*>(p->d_A), static_cast<float*>(p->d_pre),
                       float(dtau));
  KSC_HIP(hipGetLastError());
  p->pre_dtau = dtau;
  return KSC_OK;
}

// Solve table of the implicit-in-s step: per curve and chain (odd rows, even
// rows), P chunks (a power of two with P * chunk >= chain rows, at least
// 256 / CW for CW the mode columns rounded up to a power of two) and the mode
// columns in groups of 256 / P; chunk = 8 rows per thread when every chain
// fits 256 * 8 rows, else 16.
ksc_status build_simp(ksc_problem* p) {
  std::vector<ksc::SimpBlock> b;
  // chunks of 8 rows (half the registers of 16) while every chain fits
  int longest = 0;
  for (const CurveDev& d : p->cd) longest = std::max(longest, (d.n_s - 1) / 2);
  if (longest > ksc::kSimpMaxChunks * ksc::kSimpChunkMax)
    return fail(KSC_ERR_UNSUPPORTED, "ksc_set_scheme: n_s too large for the banded solve");
  const int chunk = longest <= ksc::kSimpMaxChunks * 8 ? 8 : 16;
  for (int c = 0; c < p->nc; ++c) {
    const CurveDev& d = p->cd[c];
    const int nm = p->row_elems(d);
    int cw = 1;
    while (cw < nm) cw *= 2;
    for (int par = 0; par < 2; ++par) {
      const int n = (d.n_s - 1 - par) / 2;
      if (n < 1) continue;
      int lp = 0;
      while ((1 << lp) * chunk < n) ++lp;
      while ((ksc::kSimpThreads >> lp) > cw) ++lp;
      if ((1 << lp) > ksc::kSimpMaxChunks)
        return fail(KSC_ERR_UNSUPPORTED, "ksc_set_scheme: too few mode columns");
      const int CW = ksc::kSimpThreads >> lp;
      for (int c0 = 0; c0 < nm; c0 += CW) b.push_back(ksc::SimpBlock{c, par, c0, lp});
    }
  }
  if (p->d_simp) hipFree(p->d_simp);
  p->d_simp = nullptr;
  p->n_simp = int(b.size());
  p->simp_chunk = chunk;
  KSC_HIP(hipMalloc(&p->d_simp, b.size() * sizeof(ksc::SimpBlock)));
  KSC_HIP(hipMemcpy(p->d_simp, b.data(), b.size() * sizeof(ksc::SimpBlock),
                    hipMemcpyHostToDevice));
  if (!p->d_G) KSC_HIP(hipMalloc(&p->d_G, p->state_bytes()));
  if (!p->d_zero) {
    KSC_HIP(hipMalloc(&p->d_zero, p->state_bytes()));
    KSC_HIP(hipMemset(p->d_zero, 0, p->state_bytes()));
  }
  return KSC_OK;
}

template <typename T>
ksc_status launch_simp_t(ksc_problem* p, const void* in, const void* grad, void* out, double dtau,
                         double beta, const uint8_t* active, hipStream_t s) {
  ksc::SimpArgs<T> a{};
  a.in = static_cast<const T*>(in);
  a.grad = static_cast<const T*>(grad);
  a.out = static_cast<T*>(out);
  a.curves = p->d_cd;
  a.cs = static_cast<const T*>(p->d_cs);
  a.wlT = static_cast<const T*>(p->d_wlT);
  a.A = static_cast<const T*>(p->d_A);
  a.blocks = p->d_simp;
  a.active = active;
  a.dtau = T(dtau);
  a.beta = T(beta);
  a.rose = p->d_rose;
  a.odd = p->odd() ? 1 : 0;
  hipError_t e;
  if constexpr (sizeof(T) == 8)
    e = ksc::launch_simp_f64(p->simp_chunk, p->n_simp, s, a);
  else
    e = ksc::launch_simp_f32(p->simp_chunk, p->n_simp, s, a);
  if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("simp kernel: ") + hipGetErrorString(e));
  return KSC_OK;
}

// One descent step in -> out under the problem's scheme; beta > 0 (the
// implicit-in-s scheme only) adds beta (in - out on entry).
ksc_status step_once(ksc_problem* p, const void* in, void* out, double dtau, double beta,
                     const uint8_t* active, double* J2, int track, bool finalize, hipStream_t s) {
  if (p->scheme == KSC_SCHEME_PAPER)
    return run(p, ksc::MODE_STEP, in, out, nullptr, active, J2, nullptr, track, finalize, s);
  ksc_status st = run(p, ksc::MODE_GRAD, in, p->d_G, nullptr, active, J2, nullptr, track,
                      finalize, s);
  if (st != KSC_OK) return st;
  return p->dtype == KSC_F64 ? launch_simp_t<double>(p, in, p->d_G, out, dtau, beta, active, s)
                             : launch_simp_t<float>(p, in, p->d_G, out, dtau, beta, active, s);
}

template <typename T>
std::vector<T> cast_vec(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

}  // namespace

// ------------------------------------------------------------------- C ABI --

// ------------------------------------------------- allocation-free J^2 --
//
// ksc_eval_J_noalloc evaluates J^2 of curves that share one descriptor with
// no problem object and no device allocation: the per-row metric tables, the
// curve and tile lists and the per-wave partial sums live in `scratch`, one
// fixed array per GPU (held until the process ends).  In host code the
// array's name is only a stand-in; its device address comes from
// hipGetSymbolAddress, once per device, and only that address is passed on.

namespace {

constexpr size_t kNoallocBytes = KSC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Byte offsets of the pieces inside the scratch array (256-byte aligned).
struct NoallocLayout {
  size_t curves, tiles, cs, wlT, wlD, part, end;
};
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
NoallocLayout noalloc_layout(int n_curves, int n_s, int n_tiles, int W, size_t es) {
  NoallocLayout l{};
  size_t o = 0;
  l.curves = o; o = align256(o + size_t(n_curves) * sizeof(CurveDev));
  l.tiles = o;  o = align256(o + size_t(n_tiles) * sizeof(TileDev));
  l.cs = o;     o = align256(o + size_t(n_s) * es);
  l.wlT = o;    o = align256(o + size_t(n_s) * es);
  l.wlD = o;    o = align256(o + size_t(n_s) * 8);
  l.part = o;   o = align256(o + size_t(n_tiles) * W * 3 * 8);
  l.end = o;
  return l;
}

// The same tables ksc_create builds on the host (FP64, cast to T), for one
// descriptor shared by every curve: one thread per row, per curve, per tile.
template <typename T>
__global__ void noalloc_setup_kernel(ksc_curve_desc d, int n_curves, int rows_per_tile,
                                     int tiles_per_curve, unsigned char* base, NoallocLayout l) {
  CurveDev* cdv = reinterpret_cast<CurveDev*>(base + l.curves);
  TileDev* tl = reinterpret_cast<TileDev*>(base + l.tiles);
  T* cs = reinterpret_cast<T*>(base + l.cs);
  T* wlT = reinterpret_cast<T*>(base + l.wlT);
  double* wlD = reinterpret_cast<double*>(base + l.wlD);
  const int km = (d.n_x - 1) / 3 + 1;
  const long long n_tiles = (long long)n_curves * tiles_per_curve;
  const long long total = d.n_s + n_curves + n_tiles;
  const double dsig = 1.0 / (d.n_s - 1);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    if (i < d.n_s) {
      const int j = int(i);
      double g;
      if (d.map == KSC_MAP_RATIONAL) {
        const double sn = sin(M_PI * (1.0 - j * dsig));
        g = sn * sn / (M_PI * d.scale);
      } else {
        g = 1.0 / d.scale;
      }
      const bool interior = (j > 0 && j < d.n_s - 1);
      cs[j] = T(interior ? g / (2.0 * dsig) : 0.0);
      wlT[j] = T(interior ? 2.0 * dsig / g * d.L : 0.0);
      wlD[j] = interior ? dsig / g * d.L : 0.0;
    } else if (i < d.n_s + n_curves) {
      const int c = int(i - d.n_s);
      CurveDev v{};
      v.off = (long long)c * d.n_s * km;
      v.poff = (long long)c * d.n_s * d.n_x;
      v.n_s = d.n_s;
      v.n_x = d.n_x;
      v.km = km;
      v.row_off = 0;  // every curve shares the row tables
      v.mode_off = 0;
      v.tile_begin = c * tiles_per_curve;
      v.n_tiles = tiles_per_curve;
      v.q1 = 2.0 * M_PI / d.L;
      cdv[c] = v;
    } else {
      const long long t = i - d.n_s - n_curves;
      tl[t] = TileDev{int(t / tiles_per_curve), int(t % tiles_per_curve) * rows_per_tile};
    }
  }
}

// J^2[c] = the curve's per-wave partials summed by one wave in a fixed order.
__global__ __launch_bounds__(256) void noalloc_reduce_kernel(const double* part, int slots_per_curve,
                                                             int n_curves, double* J2) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= n_curves) return;
  double s = 0.0;
  for (int t = lane; t < slots_per_curve; t += 64) s += part[3 * ((long long)c * slots_per_curve + t)];
  s = wave_sum_fixed(s);
  if (lane == 0) J2[c] = s;
}

template <typename T>
ksc_status eval_J_noalloc_t(const ksc_curve_desc& d, int n_curves, const void* state, double* J2,
                            hipStream_t s, void* base) {
  const int lanes = (sizeof(T) == 4 && d.n_x == 256) ? ksc::kLanesF32N256
                    : (d.n_x * int(sizeof(T)) > 512) ? 2 : 1;
  const int km = modes_of(d.n_x);
  int dev = 0;
  KSC_HIP(hipGetDevice(&dev));
  int lds_dev = 0;
  KSC_HIP(hipDeviceGetAttribute(&lds_dev, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // the widest tile whose staging buffer (and parked u samples) fits in LDS,
  // as for a problem object (lds_for)
  int W = 0;
  size_t lds = 0;
  for (int w : {4, 2, 1}) {
    const size_t rows = size_t(64 * w / lanes) + 2;
    const size_t park = size_t(64 * w) * ksc::u_stash_n(d.n_x, int(sizeof(T))) * sizeof(T);
    const size_t b = (lanes > 2)
                         ? size_t(ksc::lanes_lds_bytes(d.n_x, km, 64 * w / lanes, lanes, int(sizeof(T))))
                         : (rows * km + 2) * 2 * sizeof(T) + park;
    if (b <= size_t(lds_dev)) {
      W = w;
      lds = b;
      break;
    }
  }
  if (W == 0) return fail(KSC_ERR_UNSUPPORTED, "ksc_eval_J_noalloc: tile does not fit in LDS");
  const int R = 64 * W / lanes;
  const int tpc = (d.n_s + R - 1) / R;
  const long long n_tiles = (long long)tpc * n_curves;
  if (n_tiles > (1ll << 30))
    return fail(KSC_ERR_SHAPE, "ksc_eval_J_noalloc: too many tiles");
  const NoallocLayout l = noalloc_layout(n_curves, d.n_s, int(n_tiles), W, sizeof(T));
  if (l.end > kNoallocBytes)
    return fail(KSC_ERR_SHAPE, "ksc_eval_J_noalloc: the batch needs " + std::to_string(l.end) +
                                   " bytes of scratch, more than KSC_NOALLOC_SCRATCH_BYTES (" +
                                   std::to_string(kNoallocBytes) + ")");
  unsigned char* b = static_cast<unsigned char*>(base);
  const long long items = d.n_s + n_curves + n_tiles;
  const int sg = int(std::min<long long>((items + 255) / 256, 4096));
  hipLaunchKernelGGL((noalloc_setup_kernel<T>), dim3(sg), dim3(256), 0, s, d, n_curves, R, tpc, b, l);
  KSC_HIP(hipGetLastError());
  KernelArgs<T> a{};
  a.in = static_cast<const cplx<T>*>(state);
  a.curves = reinterpret_cast<const CurveDev*>(b + l.curves);
  a.tiles = reinterpret_cast<const TileDev*>(b + l.tiles);
  a.cs = reinterpret_cast<const T*>(b + l.cs);
  a.wlT = reinterpret_cast<const T*>(b + l.wlT);
  a.wlD = reinterpret_cast<const double*>(b + l.wlD);
  a.partials = reinterpret_cast<double*>(b + l.part);
  a.part_stride = 0;  // slots in tile order: curve c owns tiles [c tpc, (c+1) tpc)
  a.km_max = km;
  a.n_tiles = int(n_tiles);
  a.tile_base = 0;
  hipError_t e = launch_uniform<T>(d.n_x, W, ksc::MODE_J, int(n_tiles), lds, s, a, nullptr, nullptr);
  if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
  hipLaunchKernelGGL(noalloc_reduce_kernel, dim3((n_curves + 3) / 4), dim3(256), 0, s,
                     reinterpret_cast<const double*>(b + l.part), tpc * W, n_curves, J2);
  KSC_HIP(hipGetLastError());
  return KSC_OK;
}

}  // namespace

extern "C" {

const char* ksc_last_error(void) { return g_err.c_str(); }

int32_t ksc_n_modes(int32_t n_x) { return nx_supported(n_x) ? modes_of(n_x) : -1; }

ksc_status ksc_create(const ksc_curve_desc* descs, int32_t n_curves, int32_t dtype,
                      void* hip_stream, ksc_problem** out) {
  return ksc_create2(descs, n_curves, dtype, KSC_SPACE_FULL, hip_stream, out);
}

ksc_status ksc_create2(const ksc_curve_desc* descs, int32_t n_curves, int32_t dtype,
                       int32_t space, void* hip_stream, ksc_problem** out) {
  const ksc_options o{dtype, space, KSC_DS_STENCIL, 0};
  return ksc_create_opts(descs, n_curves, &o, hip_stream, out);
}

ksc_status ksc_create_opts(const ksc_curve_desc* descs, int32_t n_curves, const ksc_options* opts,
                           void* hip_stream, ksc_problem** out) {
  g_err.clear();
  if (!descs || !out || !opts) return fail(KSC_ERR_ARG, "ksc_create: null pointer");
  *out = nullptr;
  const int dtype = opts->dtype, space = opts->space, ds = opts->ds;
  if (n_curves < 1) return fail(KSC_ERR_SHAPE, "ksc_create: n_curves must be >= 1");
  if (dtype != KSC_F32 && dtype != KSC_F64) return fail(KSC_ERR_ARG, "ksc_create: bad dtype");
  if (space != KSC_SPACE_FULL && space != KSC_SPACE_ODD)
    return fail(KSC_ERR_ARG, "ksc_create: bad state space");
  if (ds != KSC_DS_STENCIL && ds != KSC_DS_SPECTRAL)
    return fail(KSC_ERR_ARG, "ksc_create: bad d/ds option");
  if (opts->reserved != 0) return fail(KSC_ERR_ARG, "ksc_create: reserved option must be 0");
  for (int c = 0; c < n_curves; ++c) {
    const ksc_curve_desc& d = descs[c];
    if (!nx_supported(d.n_x))
      return fail(KSC_ERR_UNSUPPORTED, "ksc_create: curve " + std::to_string(c) + ": n_x=" +
                                           std::to_string(d.n_x) + " not in {8,...,256}");
    if (space == KSC_SPACE_ODD && dtype == KSC_F64 && d.n_x > 128)
      return fail(KSC_ERR_UNSUPPORTED, "ksc_create: curve " + std::to_string(c) +
                                           ": the inversion-symmetric subspace in FP64 "
                                           "supports n_x <= 128");
    if (ds == KSC_DS_SPECTRAL) {
      if (d.map != KSC_MAP_RATIONAL)
        return fail(KSC_ERR_ARG, "ksc_create: curve " + std::to_string(c) +
                                     ": the spectral d/ds needs the rational map");
      if (d.n_x * (dtype == KSC_F64 ? 8 : 4) > 512)
        return fail(KSC_ERR_UNSUPPORTED, "ksc_create: curve " + std::to_string(c) +
                                             ": the spectral d/ds supports n_x <= " +
                                             (dtype == KSC_F64 ? "64 in FP64" : "128 in FP32"));
      if (d.n_s > 16384)
        return fail(KSC_ERR_UNSUPPORTED, "ksc_create: curve " + std::to_string(c) +
                                             ": the spectral d/ds supports n_s <= 16384");
    }
    if (d.n_s < 3)
      return fail(KSC_ERR_SHAPE, "ksc_create: curve " + std::to_string(c) + ": n_s < 3");
    if (d.n_s > (1 << 26))
      return fail(KSC_ERR_SHAPE, "ksc_create: curve " + std::to_string(c) + ": n_s too large");
    if (!(d.L > 0) || !std::isfinite(d.L))
      return fail(KSC_ERR_ARG, "ksc_create: curve " + std::to_string(c) + ": L must be > 0");
    if (d.map != KSC_MAP_RATIONAL && d.map != KSC_MAP_FINITE)
      return fail(KSC_ERR_ARG, "ksc_create: curve " + std::to_string(c) + ": bad map");
    if (!(d.scale > 0) || !std::isfinite(d.scale))
      return fail(KSC_ERR_ARG, "ksc_create: curve " + std::to_string(c) + ": scale must be > 0");
    if (!std::isfinite(d.s0)) return fail(KSC_ERR_ARG, "ksc_create: s0 must be finite");
  }
  auto* p = new ksc_problem();
  p->nc = n_curves;
  p->dtype = dtype;
  p->space = space;
  p->ds = ds;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->desc.assign(descs, descs + n_curves);
  auto cleanup = [&](ksc_status st) {
    ksc_destroy(p);
    return st;
  };
  if (hipGetDevice(&p->device) != hipSuccess) return cleanup(fail(KSC_ERR_HIP, "no HIP device"));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) != hipSuccess)
    return cleanup(fail(KSC_ERR_HIP, "hipGetDeviceProperties failed"));
  p->lds_limit = prop.sharedMemPerBlock;
  p->n_cu = prop.multiProcessorCount;

  // layout, tables (FP64 on the host, cast to the run precision)
  std::vector<double> cs, wl, wl2, A, sqrtL;
  p->cd.resize(n_curves);
  for (int c = 0; c < n_curves; ++c) {
    const ksc_curve_desc& d = descs[c];
    CurveDev& cd = p->cd[c];
    cd.n_s = d.n_s;
    cd.n_x = d.n_x;
    cd.km = modes_of(d.n_x);
    cd.off = p->numel_c;
    cd.poff = p->phys_numel;
    cd.row_off = int(cs.size());
    cd.mode_off = int(A.size());
    cd.q1 = 2.0 * M_PI / d.L;
    p->numel_c += (long long)d.n_s * p->row_elems(cd);
    p->phys_numel += (long long)d.n_s * d.n_x;
    const double dsig = 1.0 / (d.n_s - 1);
    for (int j = 0; j < d.n_s; ++j) {
      double g;
      if (d.map == KSC_MAP_RATIONAL) {
        const double th = M_PI * (1.0 - j * dsig);
        const double sn = std::sin(th);
        g = sn * sn / (M_PI * d.scale);
      } else {
        g = 1.0 / d.scale;
      }
      const bool interior = (j > 0 && j < d.n_s - 1);
      cs.push_back(interior ? g / (2.0 * dsig) : 0.0);
      wl.push_back(interior ? dsig / g * d.L : 0.0);
      wl2.push_back(interior ? 2.0 * dsig / g * d.L : 0.0);
    }
    for (int k = 0; k < cd.km; ++k) {
      const double qk = 2.0 * M_PI * k / d.L;
      A.push_back(qk * qk - qk * qk * qk * qk);
    }
    sqrtL.push_back(std::sqrt(d.L));
    p->max_nx = std::max(p->max_nx, d.n_x);
    p->min_nx = std::min(p->min_nx, d.n_x);
    if (d.n_x != 32 && d.n_x != 64 && d.n_x != 128) p->mixed_ok = false;
  }
  if (p->odd() || p->spectral()) p->mixed_ok = false;  // one launch per distinct n_x
  p->uniform = (p->max_nx == p->min_nx);
  p->rows_total = int(cs.size());
  p->modes_total = int(A.size());
  p->km_max = modes_of(p->max_nx);
  p->curve_order.resize(n_curves);
  for (int c = 0; c < n_curves; ++c) p->curve_order[c] = c;
  std::stable_sort(p->curve_order.begin(), p->curve_order.end(),
                   [&](int a, int b) { return p->cd[a].n_x > p->cd[b].n_x; });

  const size_t es = p->esize();
  auto upload = [&](void** dst, const std::vector<double>& v) -> ksc_status {
    KSC_HIP(hipMalloc(dst, std::max<size_t>(1, v.size()) * es));
    if (p->dtype == KSC_F64) {
      KSC_HIP(hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> f = cast_vec<float>(v);
      KSC_HIP(hipMemcpy(*dst, f.data(), f.size() * 4, hipMemcpyHostToDevice));
    }
    return KSC_OK;
  };
  ksc_status st;
  p->h_cs = cs;
  p->h_wl2 = wl2;
  if ((st = upload(&p->d_cs, cs)) != KSC_OK) return cleanup(st);
  if ((st = upload(&p->d_wlT, wl2)) != KSC_OK) return cleanup(st);
  if ((st = upload(&p->d_A, A)) != KSC_OK) return cleanup(st);
  if ((st = upload(&p->d_pre, A)) != KSC_OK) return cleanup(st);  // overwritten per dtau
  auto upload_d = [&](double** dst, const std::vector<double>& v) -> ksc_status {
    KSC_HIP(hipMalloc(dst, std::max<size_t>(1, v.size()) * 8));
    KSC_HIP(hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice));
    return KSC_OK;
  };
  if ((st = upload_d(&p->d_wlD, wl)) != KSC_OK) return cleanup(st);
  if ((st = upload_d(&p->d_sqrtL, sqrtL)) != KSC_OK) return cleanup(st);
  if (hipMalloc(&p->d_cd, n_curves * sizeof(CurveDev)) != hipSuccess ||
      hipMalloc(&p->d_prevJ2, n_curves * sizeof(double)) != hipSuccess ||
      hipMalloc(&p->d_J2, n_curves * sizeof(double)) != hipSuccess ||
      hipMalloc(&p->d_flags, n_curves * sizeof(unsigned)) != hipSuccess ||
      hipMalloc(&p->d_rose, n_curves) != hipSuccess)
    return cleanup(fail(KSC_ERR_HIP, "ksc_create: workspace allocation failed"));
  if (hipMemset(p->d_flags, 0, n_curves * sizeof(unsigned)) != hipSuccess ||
      hipMemset(p->d_rose, 0, n_curves) != hipSuccess)
    return cleanup(fail(KSC_ERR_HIP, "ksc_create: hipMemset failed"));
  {
    std::vector<double> nanv(n_curves, std::nan(""));
    if (hipMemcpy(p->d_prevJ2, nanv.data(), n_curves * 8, hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(KSC_ERR_HIP, "ksc_create: hipMemcpy failed"));
  }
  p->W = default_W(p);
  if (p->W == 0)
    return cleanup(fail(KSC_ERR_UNSUPPORTED, "ksc_create: tile staging buffer exceeds LDS"));
  if ((st = build_tiles(p)) != KSC_OK) return cleanup(st);
  if (p->spectral() && (st = setup_spectral(p)) != KSC_OK) return cleanup(st);
  if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return cleanup(fail(KSC_ERR_HIP, "ksc_create: stream creation failed"));
  *out = p;
  return KSC_OK;
}

ksc_status ksc_destroy(ksc_problem* p) {
  if (!p) return fail(KSC_ERR_ARG, "ksc_destroy: null problem");
  drop_graph(p);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  for (hipEvent_t e : p->tev) hipEventDestroy(e);
  void* bufs[] = {p->d_bounds, p->d_cd,  p->d_tiles, p->d_cs,    p->d_wlT,    p->d_wlD,
                  p->d_A,   p->d_pre,   p->d_sqrtL, p->d_part,   p->d_prevJ2,
                  p->d_flags, p->d_rose, p->d_J2,  p->d_edge,  p->d_dpool,  p->d_spec,  p->d_Y,
                  p->d_WR,  p->d_P,   p->d_sgroups, p->d_kpart, p->d_G, p->d_zero, p->d_simp};
  for (void* b : bufs)
    if (b) hipFree(b);
  delete p;
  return KSC_OK;
}

ksc_status ksc_set_stream(ksc_problem* p, void* hip_stream) {
  if (!p) return fail(KSC_ERR_ARG, "ksc_set_stream: null problem");
  p->stream = static_cast<hipStream_t>(hip_stream);
  return KSC_OK;
}

int64_t ksc_state_numel(const ksc_problem* p) {
  return p ? int64_t(p->state_bytes() / p->esize()) : -1;
}
int64_t ksc_state_offset(const ksc_problem* p, int32_t c) {
  if (!p || c < 0 || c >= p->nc) return -1;
  return p->cd[c].off * int64_t(p->elem_bytes() / p->esize());
}
int64_t ksc_phys_numel(const ksc_problem* p) { return p ? p->phys_numel : -1; }
int64_t ksc_phys_offset(const ksc_problem* p, int32_t c) {
  if (!p || c < 0 || c >= p->nc) return -1;
  return p->cd[c].poff;
}

ksc_status ksc_set_endpoints(ksc_problem* p, void* state, int32_t curve, const void* a_hat,
                             const void* b_hat) {
  if (!p || !state || !a_hat || !b_hat) return fail(KSC_ERR_ARG, "ksc_set_endpoints: null pointer");
  if (curve < 0 || curve >= p->nc) return fail(KSC_ERR_SHAPE, "ksc_set_endpoints: bad curve");
  const CurveDev& d = p->cd[curve];
  const size_t rowb = size_t(p->row_elems(d)) * p->elem_bytes();
  char* base = static_cast<char*>(state) + d.off * p->elem_bytes();
  KSC_HIP(hipMemcpyAsync(base, a_hat, rowb, hipMemcpyDeviceToDevice, p->stream));
  KSC_HIP(hipMemcpyAsync(base + size_t(d.n_s - 1) * rowb, b_hat, rowb, hipMemcpyDeviceToDevice,
                         p->stream));
  return KSC_OK;
}

static ksc_status convert(ksc_problem* p, bool to_spec, const void* src, void* dst) {
  if (!p || !src || !dst) return fail(KSC_ERR_ARG, "conversion: null pointer");
  for (int c = 0; c < p->nc; ++c) {
    const CurveDev& d = p->cd[c];
    hipError_t e;
    if (p->odd()) {
      if (p->dtype == KSC_F64) {
        const double* ph = static_cast<const double*>(to_spec ? src : dst) + d.poff;
        double* sp = static_cast<double*>(const_cast<void*>(to_spec ? dst : src)) + d.off;
        e = to_spec ? ksc::launch_p2s_odd_f64(d.n_x, d.n_s, p->stream, ph, sp)
                    : ksc::launch_s2p_odd_f64(d.n_x, d.n_s, p->stream, sp, const_cast<double*>(ph));
      } else {
        const float* ph = static_cast<const float*>(to_spec ? src : dst) + d.poff;
        float* sp = static_cast<float*>(const_cast<void*>(to_spec ? dst : src)) + d.off;
        e = to_spec ? ksc::launch_p2s_odd_f32(d.n_x, d.n_s, p->stream, ph, sp)
                    : ksc::launch_s2p_odd_f32(d.n_x, d.n_s, p->stream, sp, const_cast<float*>(ph));
      }
    } else if (p->dtype == KSC_F64) {
      const double* ph = static_cast<const double*>(to_spec ? src : dst) + d.poff;
      cplx<double>* sp = reinterpret_cast<cplx<double>*>(const_cast<void*>(to_spec ? dst : src)) + d.off;
      e = to_spec ? ksc::launch_p2s_f64(d.n_x, d.n_s, p->stream, ph, sp)
                  : ksc::launch_s2p_f64(d.n_x, d.n_s, p->stream, sp, const_cast<double*>(ph));
    } else {
      const float* ph = static_cast<const float*>(to_spec ? src : dst) + d.poff;
      cplx<float>* sp = reinterpret_cast<cplx<float>*>(const_cast<void*>(to_spec ? dst : src)) + d.off;
      e = to_spec ? ksc::launch_p2s_f32(d.n_x, d.n_s, p->stream, ph, sp)
                  : ksc::launch_s2p_f32(d.n_x, d.n_s, p->stream, sp, const_cast<float*>(ph));
    }
    if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("conversion: ") + hipGetErrorString(e));
  }
  return KSC_OK;
}

ksc_status ksc_phys_to_spec(ksc_problem* p, const void* phys, void* state) {
  return convert(p, true, phys, state);
}
ksc_status ksc_spec_to_phys(ksc_problem* p, const void* state, void* phys) {
  return convert(p, false, state, phys);
}

ksc_status ksc_eval_J(ksc_problem* p, const void* state, double* J2, double* Jarc) {
  if (!p || !state || !J2) return fail(KSC_ERR_ARG, "ksc_eval_J: null pointer");
  return run(p, ksc::MODE_J, state, nullptr, nullptr, nullptr, J2, Jarc, 0, true, p->stream);
}

ksc_status ksc_eval_grad(ksc_problem* p, const void* state, void* grad, double* J2,
                         const double* scale) {
  if (!p || !state || !grad) return fail(KSC_ERR_ARG, "ksc_eval_grad: null pointer");
  if (grad == state) return fail(KSC_ERR_ARG, "ksc_eval_grad: grad must not alias state");
  return run(p, ksc::MODE_GRAD, state, grad, scale, nullptr, J2, nullptr, 0, J2 != nullptr,
             p->stream);
}

ksc_status ksc_step(ksc_problem* p, const void* in, void* out, double dtau, double* J2) {
  if (!p || !in || !out) return fail(KSC_ERR_ARG, "ksc_step: null pointer");
  if (in == out) return fail(KSC_ERR_ARG, "ksc_step: in and out must differ");
  if (!(dtau > 0) || !std::isfinite(dtau)) return fail(KSC_ERR_ARG, "ksc_step: dtau must be > 0");
  ksc_status st = ensure_pre(p, dtau, p->stream);
  if (st != KSC_OK) return st;
  return step_once(p, in, out, dtau, 0.0, nullptr, J2, 0, J2 != nullptr, p->stream);
}

// Record `every` steps (state -> scratch -> state ...) plus per-step
// finalization into one graph on the capture stream.
static ksc_status capture_descent(ksc_problem* p, void* state, void* scratch, double dtau,
                                  int every, const uint8_t* active) {
  drop_graph(p);
  hipStream_t s = p->cap_stream;
  KSC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  ksc_status st = KSC_OK;
  for (int i = 0; i < every && st == KSC_OK; ++i) {
    const void* in = (i % 2 == 0) ? state : scratch;
    void* out = (i % 2 == 0) ? scratch : state;
    st = step_once(p, in, out, dtau, p->momentum, active, p->d_J2, 1, true, s);
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (st != KSC_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(KSC_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
  p->graph = g;
  e = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(p);
    return fail(KSC_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e));
  }
  p->gkey = ksc_problem::Key{state, scratch, dtau, every, active, p->W, p->policy, p->momentum,
                             p->stream};
  return KSC_OK;
}

ksc_status ksc_descend(ksc_problem* p, void* state, void* scratch, int64_t n_steps, double dtau,
                       double* J2_trace, int32_t every, const uint8_t* active) {
  if (!p || !state || !scratch) return fail(KSC_ERR_ARG, "ksc_descend: null pointer");
  if (state == scratch) return fail(KSC_ERR_ARG, "ksc_descend: scratch must differ from state");
  if (n_steps < 0) return fail(KSC_ERR_ARG, "ksc_descend: n_steps < 0");
  if (every < 1) return fail(KSC_ERR_ARG, "ksc_descend: every must be >= 1");
  if (!(dtau > 0) || !std::isfinite(dtau)) return fail(KSC_ERR_ARG, "ksc_descend: dtau must be > 0");
  if (p->momentum > 0 && p->scheme != KSC_SCHEME_IMPLICIT_S)
    return fail(KSC_ERR_UNSUPPORTED, "ksc_descend: momentum needs the implicit-in-s scheme");
  if (p->momentum > 0 && every % 2 != 0)
    return fail(KSC_ERR_ARG, "ksc_descend: momentum needs an even `every`");
  if (n_steps == 0) return KSC_OK;
  ksc_status st = ensure_pre(p, dtau, p->stream);
  if (st != KSC_OK) return st;
  // the endpoint rows of scratch must match the state's: copy the whole state once
  KSC_HIP(hipMemcpyAsync(scratch, state, p->state_bytes(), hipMemcpyDeviceToDevice, p->stream));
  // groups of `every` steps; an odd group ends in scratch and is copied back
  const int G = every;
  const ksc_problem::Key want{state, scratch, dtau, G, active, p->W, p->policy, p->momentum,
                              p->stream};
  const bool same = p->gexec && want.state == p->gkey.state && want.scratch == p->gkey.scratch &&
                    want.dtau == p->gkey.dtau && want.every == p->gkey.every &&
                    want.active == p->gkey.active && want.W == p->gkey.W &&
                    want.policy == p->gkey.policy && want.momentum == p->gkey.momentum;
  if (!same) {
    // the capture stream must not run ahead of work already queued on p->stream
    KSC_HIP(hipStreamSynchronize(p->stream));
    if ((st = capture_descent(p, state, scratch, dtau, G, active)) != KSC_OK) return st;
  }
  const int64_t groups = n_steps / G;
  const int64_t rem = n_steps % G;
  for (int64_t gi = 0; gi < groups; ++gi) {
    KSC_HIP(hipGraphLaunch(p->gexec, p->stream));
    if (G % 2 == 1)
      KSC_HIP(hipMemcpyAsync(state, scratch, p->state_bytes(), hipMemcpyDeviceToDevice,
                             p->stream));
    if (J2_trace)
      KSC_HIP(hipMemcpyAsync(J2_trace + gi * p->nc, p->d_J2, p->nc * sizeof(double),
                             hipMemcpyDeviceToDevice, p->stream));
  }
  for (int64_t i = 0; i < rem; ++i) {
    const void* in = (i % 2 == 0) ? state : scratch;
    void* out = (i % 2 == 0) ? scratch : state;
    st = step_once(p, in, out, dtau, p->momentum, active, p->d_J2, 1, true, p->stream);
    if (st != KSC_OK) return st;
  }
  if (rem % 2 == 1)
    KSC_HIP(hipMemcpyAsync(state, scratch, p->state_bytes(), hipMemcpyDeviceToDevice, p->stream));
  return KSC_OK;
}

ksc_status ksc_set_scheme(ksc_problem* p, int32_t scheme) {
  if (!p) return fail(KSC_ERR_ARG, "ksc_set_scheme: null problem");
  if (scheme != KSC_SCHEME_PAPER && scheme != KSC_SCHEME_IMPLICIT_S)
    return fail(KSC_ERR_ARG, "ksc_set_scheme: bad scheme");
  if (scheme == KSC_SCHEME_IMPLICIT_S) {
    if (p->spectral())
      return fail(KSC_ERR_UNSUPPORTED,
                  "ksc_set_scheme: the implicit-in-s step needs the central-difference d/ds");
    if (p->scheme == KSC_SCHEME_IMPLICIT_S && p->d_simp) return KSC_OK;  // already set up
    // (a captured descent graph points at the solve table build_simp replaces)
    drop_graph(p);
    ksc_status st = build_simp(p);
    if (st != KSC_OK) return st;
  }
  if (scheme != p->scheme) drop_graph(p);
  p->scheme = scheme;
  return KSC_OK;
}

ksc_status ksc_set_momentum(ksc_problem* p, double beta) {
  if (!p) return fail(KSC_ERR_ARG, "ksc_set_momentum: null problem");
  if (!(beta >= 0.0 && beta < 1.0)) return fail(KSC_ERR_ARG, "ksc_set_momentum: beta must be in [0, 1)");
  if (beta != p->momentum) drop_graph(p);
  p->momentum = beta;
  return KSC_OK;
}

ksc_status ksc_get_momentum(const ksc_problem* p, double* beta) {
  if (!p || !beta) return fail(KSC_ERR_ARG, "ksc_get_momentum: null pointer");
  *beta = p->momentum;
  return KSC_OK;
}

ksc_status ksc_precondition(ksc_problem* p, const void* grad, void* out, double dtau) {
  if (!p || !grad || !out) return fail(KSC_ERR_ARG, "ksc_precondition: null pointer");
  if (grad == out) return fail(KSC_ERR_ARG, "ksc_precondition: grad and out must differ");
  if (!(dtau > 0) || !std::isfinite(dtau))
    return fail(KSC_ERR_ARG, "ksc_precondition: dtau must be > 0");
  if (p->scheme != KSC_SCHEME_IMPLICIT_S || !p->d_simp || !p->d_zero)
    return fail(KSC_ERR_UNSUPPORTED,
                "ksc_precondition: needs ksc_set_scheme(KSC_SCHEME_IMPLICIT_S) first");
  // the implicit-in-s solve of the step, on a zero state: out = 0 + delta(grad)
  return p->dtype == KSC_F64
             ? launch_simp_t<double>(p, p->d_zero, grad, out, dtau, 0.0, nullptr, p->stream)
             : launch_simp_t<float>(p, p->d_zero, grad, out, dtau, 0.0, nullptr, p->stream);
}

ksc_status ksc_get_scheme(const ksc_problem* p, int32_t* scheme) {
  if (!p || !scheme) return fail(KSC_ERR_ARG, "ksc_get_scheme: null pointer");
  *scheme = p->scheme;
  return KSC_OK;
}

ksc_status ksc_set_launch(ksc_problem* p, int32_t policy, int32_t waves) {
  if (!p) return fail(KSC_ERR_ARG, "ksc_set_launch: null problem");
  if (policy != KSC_LAUNCH_AUTO && policy != KSC_LAUNCH_PLAIN && policy != KSC_LAUNCH_PERSISTENT)
    return fail(KSC_ERR_ARG, "ksc_set_launch: bad policy");
  if (waves != 0 && waves != 1 && waves != 2 && waves != 4)
    return fail(KSC_ERR_ARG, "ksc_set_launch: waves must be 0, 1, 2 or 4");
  if (waves != 0) {
    if (lds_max(p, waves) > p->lds_limit)
      return fail(KSC_ERR_UNSUPPORTED, "ksc_set_launch: tile does not fit in LDS");
    if (waves != p->W) {
      p->W = waves;
      ksc_status st = build_tiles(p);
      if (st != KSC_OK) return st;
      drop_graph(p);
    }
  }
  if (policy != p->policy) drop_graph(p);
  p->policy = policy;
  return KSC_OK;
}

ksc_status ksc_get_launch(const ksc_problem* p, int32_t* policy, int32_t* waves) {
  if (!p || !policy || !waves) return fail(KSC_ERR_ARG, "ksc_get_launch: null pointer");
  *policy = p->policy;
  *waves = p->W;
  return KSC_OK;
}

ksc_status ksc_set_timing(ksc_problem* p, int32_t enable) {
  if (!p) return fail(KSC_ERR_ARG, "ksc_set_timing: null problem");
  p->timing = enable != 0;
  if (p->timing) {
    p->tev_used = 0;
    p->timing_overflow = false;
  }
  return KSC_OK;
}

ksc_status ksc_read_timing(ksc_problem* p, double* fused_ms, double* post_ms, int64_t* n_evals) {
  if (!p || !fused_ms || !post_ms || !n_evals) return fail(KSC_ERR_ARG, "ksc_read_timing: null pointer");
  double f = 0, q = 0;
  const size_t n = p->tev_used / 4;
  for (size_t i = 0; i < n; ++i) {
    hipEvent_t* e = &p->tev[4 * i];
    KSC_HIP(hipEventSynchronize(e[3]));
    float a = 0, b = 0;
    KSC_HIP(hipEventElapsedTime(&a, e[0], e[1]));
    KSC_HIP(hipEventElapsedTime(&b, e[2], e[3]));
    f += a;
    q += b;
  }
  *fused_ms = f;
  *post_ms = q;
  *n_evals = int64_t(n);
  if (p->timing_overflow)
    return fail(KSC_ERR_STATE, "ksc_read_timing: more evaluations than the timing window holds");
  return KSC_OK;
}

ksc_status ksc_eval_J_noalloc(const ksc_curve_desc* desc, int32_t n_curves, int32_t dtype,
                              const void* state, double* J2, void* hip_stream) {
  if (!desc || !state || !J2) return fail(KSC_ERR_ARG, "ksc_eval_J_noalloc: null pointer");
  if (n_curves < 1) return fail(KSC_ERR_ARG, "ksc_eval_J_noalloc: n_curves < 1");
  if (dtype != KSC_F32 && dtype != KSC_F64) return fail(KSC_ERR_ARG, "ksc_eval_J_noalloc: bad dtype");
  const ksc_curve_desc& d = *desc;
  if (!nx_supported(d.n_x)) return fail(KSC_ERR_UNSUPPORTED, "ksc_eval_J_noalloc: n_x not in {8,...,256}");
  if (d.n_s < 3 || d.n_s > (1 << 26)) return fail(KSC_ERR_SHAPE, "ksc_eval_J_noalloc: bad n_s");
  if (!(d.L > 0) || !std::isfinite(d.L)) return fail(KSC_ERR_ARG, "ksc_eval_J_noalloc: L must be > 0");
  if (d.map != KSC_MAP_RATIONAL && d.map != KSC_MAP_FINITE)
    return fail(KSC_ERR_ARG, "ksc_eval_J_noalloc: bad map");
  if (!(d.scale > 0) || !std::isfinite(d.scale))
    return fail(KSC_ERR_ARG, "ksc_eval_J_noalloc: scale must be > 0");
  void* base = nullptr;
  KSC_HIP(scratch_address(&base));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  return dtype == KSC_F64 ? eval_J_noalloc_t<double>(d, n_curves, state, J2, s, base)
                          : eval_J_noalloc_t<float>(d, n_curves, state, J2, s, base);
}

ksc_status ksc_query_flags(ksc_problem* p, uint32_t* flags_host) {
  if (!p || !flags_host) return fail(KSC_ERR_ARG, "ksc_query_flags: null pointer");
  KSC_HIP(hipStreamSynchronize(p->stream));
  KSC_HIP(hipMemcpy(flags_host, p->d_flags, p->nc * sizeof(unsigned), hipMemcpyDeviceToHost));
  KSC_HIP(hipMemset(p->d_flags, 0, p->nc * sizeof(unsigned)));
  return KSC_OK;
}

// Time each admissible (policy, W) on scratch state buffers and keep the
// fastest for J + gradient; the result is cached in a small JSON file.
ksc_status ksc_tune(ksc_problem* p, const char* cache_path) {
  if (!p) return fail(KSC_ERR_ARG, "ksc_tune: null problem");
  hipDeviceProp_t prop;
  KSC_HIP(hipGetDeviceProperties(&prop, p->device));
  int rt = 0;
  hipRuntimeGetVersion(&rt);
  std::ostringstream key;
  key << prop.gcnArchName << "|" << rt << "|" << (p->dtype == KSC_F64 ? "f64" : "f32") << "|";
  if (p->odd()) key << "odd|";
  if (p->spectral()) key << "spec|";
  for (const auto& d : p->desc) key << d.n_x << "x" << d.n_s << ";";
  std::string kstr = key.str();
  // a long key is hashed to keep the file small
  if (kstr.size() > 200) {
    unsigned long long h = 1469598103934665603ull;
    for (char ch : kstr) h = (h ^ (unsigned char)ch) * 1099511628211ull;
    kstr = kstr.substr(0, 64) + "#" + std::to_string(h);
  }
  if (cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      auto pos = line.find("\"" + kstr + "\"");
      if (pos == std::string::npos) continue;
      int pol = 0, w = 0;
      auto pp = line.find("\"policy\":", pos), pw = line.find("\"waves\":", pos);
      if (pp != std::string::npos && pw != std::string::npos) {
        pol = std::atoi(line.c_str() + pp + 9);
        w = std::atoi(line.c_str() + pw + 8);
        return ksc_set_launch(p, pol, w);
      }
    }
  }
  const size_t bytes = p->state_bytes();
  void *x = nullptr, *g = nullptr;
  double* j2 = nullptr;
  KSC_HIP(hipMalloc(&x, bytes));
  KSC_HIP(hipMalloc(&g, bytes));
  KSC_HIP(hipMalloc(&j2, p->nc * sizeof(double)));
  KSC_HIP(hipMemsetAsync(x, 0, bytes, p->stream));
  hipEvent_t e0, e1;
  KSC_HIP(hipEventCreate(&e0));
  KSC_HIP(hipEventCreate(&e1));
  // Candidates in order of preference; a later one must be at least 5% faster
  // (best of five 10-evaluation trials) to replace the incumbent, so the
  // choice does not flip on timing noise (tile shapes within a few percent of
  // each other are common).
  const bool timing = p->timing;
  p->timing = false;
  int best_pol = KSC_LAUNCH_AUTO, best_w = default_W(p);
  float best = 1e30f;
  std::vector<std::pair<int, int>> cand;
  cand.push_back({KSC_LAUNCH_AUTO, default_W(p)});
  for (int pol : {KSC_LAUNCH_AUTO, KSC_LAUNCH_PERSISTENT})
    for (int w : {4, 2, 1})
      if (!(pol == cand[0].first && w == cand[0].second)) cand.push_back({pol, w});
  for (const auto& pw : cand) {
    const int pol = pw.first, w = pw.second;
    if (lds_max(p, w) > p->lds_limit) continue;
    if (ksc_set_launch(p, pol, w) != KSC_OK) continue;
    for (int r = 0; r < 2; ++r) ksc_eval_grad(p, x, g, j2, nullptr);  // warm-up
    float ms_best = 1e30f;
    for (int trial = 0; trial < 5; ++trial) {
      hipEventRecord(e0, p->stream);
      const int reps = 10;
      for (int r = 0; r < reps; ++r) ksc_eval_grad(p, x, g, j2, nullptr);
      hipEventRecord(e1, p->stream);
      hipEventSynchronize(e1);
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      ms_best = std::min(ms_best, ms);
    }
    if (best == 1e30f || ms_best < 0.95f * best) {
      best = ms_best;
      best_pol = pol;
      best_w = w;
    }
  }
  p->timing = timing;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(x);
  hipFree(g);
  hipFree(j2);
  ksc_status st = ksc_set_launch(p, best_pol, best_w);
  if (st != KSC_OK) return st;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << "{\"" << kstr << "\": {\"policy\": " << best_pol << ", \"waves\": " << best_w
      << ", \"ms_per_eval\": " << best / 10 << "}}\n";
  }
  return KSC_OK;
}

}  // extern "C"
