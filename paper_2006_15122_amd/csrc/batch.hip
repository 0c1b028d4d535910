// Batched ensembles of independent scalar lattices (sizes may differ).
//
// Every pass of every run goes through one batched kernel whose blocks are
// the tiles of all runs (tile table built on the host), followed by one
// finish block per run that reduces that run's FP64 partials in a fixed order
// and advances its a, b (Sec. 4.3.2).  Kernel boundaries make each pass's
// results visible across XCDs with one L2 write-back per XCD, so no block
// ever waits on another.  A whole lattice_batch_step call is captured into a
// HIP graph and launched once; the graph is cached per (nsteps, buffer
// parity) and replayed by later calls with the same key.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "scalar_tile.hpp"

namespace cl {

template <typename T, int NF, int TZ, int BY, int RY>
__global__ __launch_bounds__(TZ* BY) void batch_pass_kernel(const ScalarArgs<T>* runs, const int* tile_run,
                                                            const int* tile_local, double* partials, PassDesc pd) {
  // blocks are dealt to the XCDs in turn; this gives each XCD a contiguous
  // range of the tile table (neighbouring tiles of a run), so the halo rows
  // two tiles share are read through the same L2
  int b = blockIdx.x;
  if ((gridDim.x & 7) == 0) b = (b & 7) * (gridDim.x >> 3) + (b >> 3);
  ScalarArgs<T> A = runs[tile_run[b]];
  A.pd = pd;
  A.partials = partials;
  const DevState* st = A.st;
  scalar_tile<T, NF, false, TZ, BY, RY>(A, tile_local[b], b, [st](double& a, double& bb) {
    a = st->a;
    bb = st->b;
  });
}

template <typename T, int NF>
__global__ __launch_bounds__(256) void batch_finish_kernel(const ScalarArgs<T>* runs, const int* tile_offset,
                                                           const double* partials, PassDesc pd) {
  const int r = blockIdx.x;
  constexpr int NACC = Acc<NF, false>::N;
  double S[NACC];
  const int first = tile_offset[r];
  if (!reduce_partials<NACC, 256>(partials, first, tile_offset[r + 1] - first, S)) return;
  ScalarArgs<T> A = runs[r];
  A.pd = pd;
  finish_from_sums<T, NF, false>(A, S);
}

#define CL_BATCH_SHAPES(X) \
  X(32, 8, 2)              \
  X(32, 4, 4)              \
  X(32, 8, 4)              \
  X(64, 4, 2)              \
  X(64, 4, 4)

static const int kBatchShapes[][3] = {{32, 8, 2}, {32, 4, 4}, {32, 8, 4}, {64, 4, 2}, {64, 4, 4}};

template <typename T, int NF>
static hipError_t launch_batch_t(const Tiling& t, int ntiles, int nruns, const void* runs, const int* tile_run,
                                 const int* tile_local, const int* tile_offset, double* partials,
                                 const PassDesc& pd, hipStream_t s) {
  const ScalarArgs<T>* R = static_cast<const ScalarArgs<T>*>(runs);
  bool ok = false;
#define X(a, b, c)                                                                                          \
  if (!ok && t.tz == a && t.by == b && t.ry == c) {                                                         \
    hipLaunchKernelGGL((batch_pass_kernel<T, NF, a, b, c>), dim3(ntiles), dim3(a * b), 0, s, R, tile_run, \
                       tile_local, partials, pd);                                                           \
    ok = true;                                                                                              \
  }
  CL_BATCH_SHAPES(X)
#undef X
  if (!ok) return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_finish_kernel<T, NF>), dim3(nruns), dim3(256), 0, s, R, tile_offset, partials, pd);
  return hipGetLastError();
}

}  // namespace cl

struct lattice_batch {
  std::vector<lattice*> runs;
  int nruns;
  hipStream_t stream;
  int fp32, nf;
  cl::Tiling tile;
  // device tables
  void* args[2];        // ScalarArgs<T>[nruns] for buffer parity 0 (buf0 -> buf1) and 1
  int* tile_run;
  int* tile_local;
  int* tile_offset;
  double* partials;
  size_t args_bytes;
  int64_t max_tiles;
  int ntiles;
  int parity;           // common ping-pong index of all runs
  int use_graph;
  std::map<std::pair<int64_t, int>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  std::vector<double> weights;
};

namespace cl {

static size_t aup(size_t x) { return (x + 255) / 256 * 256; }

static int batch_validate(const lattice_params* ps, int nruns) {
  if (!ps || nruns < 1) { set_error("batch needs nruns >= 1"); return LAT_EINVAL; }
  for (int r = 0; r < nruns; ++r) {
    const int rc = validate(&ps[r]);
    if (rc) return rc;
    const lattice_params& p = ps[r];
    if (p.model != LAT_MODEL_SCALAR) { set_error("batches hold scalar models"); return LAT_EINVAL; }
    if (p.integrator == LAT_LF2) { set_error("batches use the velocity-Verlet integrators (LAT_VV2 .. LAT_VV10)"); return LAT_EINVAL; }
    if (p.nf != ps[0].nf || p.integrator != ps[0].integrator || p.precision != ps[0].precision ||
        p.dt != ps[0].dt) {
      set_error("batch runs must share nf, integrator, precision and dt");
      return LAT_EINVAL;
    }
  }
  return LAT_OK;
}

// Header: two ScalarArgs arrays, tile tables sized for the smallest tile, partials.
static void batch_header(const lattice_params* ps, int nruns, size_t* args_bytes, int64_t* max_tiles,
                         size_t* header) {
  int64_t mt = 0;
  for (int r = 0; r < nruns; ++r) {
    const int64_t N = ps[r].N;
    mt += (N / 32) * (N / 8) * (N / 4);
  }
  const size_t ab = aup((size_t)nruns * 512);  // ScalarArgs<T> is below 512 bytes
  *args_bytes = ab;
  *max_tiles = mt;
  size_t o = 2 * ab;
  o += aup((size_t)mt * 4) * 2 + aup((size_t)(nruns + 1) * 4);
  o += aup((size_t)mt * 4 * sizeof(double));
  *header = o;
}

static bool batch_tiling_ok(const lattice_batch* B, const Tiling& t) {
  bool compiled = false;
  for (const auto& s : kBatchShapes)
    if (s[0] == t.tz && s[1] == t.by && s[2] == t.ry) compiled = true;
  if (!compiled) return false;
  int64_t nt = 0;
  for (lattice* h : B->runs) {
    const int N = h->p.N, ty = t.by * t.ry;
    if (N % t.tz || N % ty || t.xc < 1 || N % t.xc) return false;
    nt += (int64_t)(N / t.tz) * (N / ty) * (N / t.xc);
  }
  return nt <= B->max_tiles;
}

// tile tables and per-run kernel arguments for the current tiling
template <typename T>
static int batch_upload_tables(lattice_batch* B) {
  std::vector<int> trun, tloc, toff(1, 0);
  const int ty = B->tile.by * B->tile.ry;
  for (int r = 0; r < B->nruns; ++r) {
    const int N = B->runs[r]->p.N;
    const int nt = (N / B->tile.tz) * (N / ty) * (N / B->tile.xc);
    for (int t = 0; t < nt; ++t) {
      trun.push_back(r);
      tloc.push_back(t);
    }
    toff.push_back(toff.back() + nt);
  }
  B->ntiles = (int)trun.size();
  std::vector<ScalarArgs<T>> a0(B->nruns), a1(B->nruns);
  for (int r = 0; r < B->nruns; ++r) {
    lattice* h = B->runs[r];
    double phys[8];
    phys_of(h, phys);
    for (int par = 0; par < 2; ++par) {
      ScalarArgs<T>& A = par ? a1[r] : a0[r];
      std::memset(&A, 0, sizeof(A));
      const int nf = h->p.nf;
      for (int f = 0; f < nf; ++f) {
        A.src[f] = static_cast<const T*>(h->buf[par][f]);
        A.src[2 + f] = static_cast<const T*>(h->buf[par][nf + f]);
        A.dst[f] = static_cast<T*>(h->buf[1 - par][f]);
        A.dst[2 + f] = static_cast<T*>(h->buf[1 - par][nf + f]);
      }
      A.N = h->p.N;
      A.XC = B->tile.xc;
      A.swizzle = 0;
      A.dx = phys[0];
      A.alpha = phys[1];
      A.fmp2 = phys[2];
      A.m2_0 = phys[3];
      A.m2_1 = phys[4];
      A.lam = phys[5];
      A.q = phys[6];
      A.h = phys[7];
      A.expand = h->p.expansion;
      A.st = h->st;
    }
  }
  static_assert(sizeof(ScalarArgs<double>) <= 512, "ScalarArgs too large for the batch table");
  CL_HIP(hipMemcpyAsync(B->args[0], a0.data(), sizeof(ScalarArgs<T>) * B->nruns, hipMemcpyHostToDevice, B->stream));
  CL_HIP(hipMemcpyAsync(B->args[1], a1.data(), sizeof(ScalarArgs<T>) * B->nruns, hipMemcpyHostToDevice, B->stream));
  CL_HIP(hipMemcpyAsync(B->tile_run, trun.data(), trun.size() * 4, hipMemcpyHostToDevice, B->stream));
  CL_HIP(hipMemcpyAsync(B->tile_local, tloc.data(), tloc.size() * 4, hipMemcpyHostToDevice, B->stream));
  CL_HIP(hipMemcpyAsync(B->tile_offset, toff.data(), toff.size() * 4, hipMemcpyHostToDevice, B->stream));
  CL_HIP(hipStreamSynchronize(B->stream));
  return LAT_OK;
}

static int batch_upload(lattice_batch* B) {
  return B->fp32 ? batch_upload_tables<float>(B) : batch_upload_tables<double>(B);
}

static hipError_t batch_launch(lattice_batch* B, const PassDesc& pd, int parity) {
  const void* args = B->args[parity];
  if (B->fp32)
    return B->nf == 1 ? launch_batch_t<float, 1>(B->tile, B->ntiles, B->nruns, args, B->tile_run, B->tile_local,
                                                 B->tile_offset, B->partials, pd, B->stream)
                      : launch_batch_t<float, 2>(B->tile, B->ntiles, B->nruns, args, B->tile_run, B->tile_local,
                                                 B->tile_offset, B->partials, pd, B->stream);
  return B->nf == 1 ? launch_batch_t<double, 1>(B->tile, B->ntiles, B->nruns, args, B->tile_run, B->tile_local,
                                                B->tile_offset, B->partials, pd, B->stream)
                    : launch_batch_t<double, 2>(B->tile, B->ntiles, B->nruns, args, B->tile_run, B->tile_local,
                                                B->tile_offset, B->partials, pd, B->stream);
}

static void drop_graphs(lattice_batch* B) {
  for (auto& kv : B->graphs) {
    (void)hipGraphExecDestroy(kv.second.second);
    (void)hipGraphDestroy(kv.second.first);
  }
  B->graphs.clear();
}

// every run must be at the batch parity (a run stepped alone flips its own)
static int sync_parity(lattice_batch* B) {
  for (lattice* h : B->runs)
    if (h->cur != B->runs[0]->cur) {
      set_error("batch runs are at different buffer parities (a run was stepped alone an odd number of passes)");
      return LAT_ESTATE;
    }
  B->parity = B->runs[0]->cur;
  return LAT_OK;
}

static int batch_autotune(lattice_batch* B) {
  hipEvent_t e0, e1;
  CL_HIP(hipEventCreate(&e0));
  CL_HIP(hipEventCreate(&e1));
  const int xcs[] = {8, 16, 32};
  float best = 1e30f;
  Tiling bt = B->tile;
  for (const auto& s : kBatchShapes)
    for (int xc : xcs) {
      Tiling t{s[0], s[1], s[2], xc};
      if (!batch_tiling_ok(B, t)) continue;
      B->tile = t;
      int rc = batch_upload(B);
      if (rc) return rc;
      // full passes into the scratch buffers, a and b untouched
      PassDesc pd = pass(1.0, 0.5, 0.5, MODE_VV, 1, 0);
      CL_HIP(batch_launch(B, pd, B->parity));
      CL_HIP(hipEventRecord(e0, B->stream));
      for (int k = 0; k < 3; ++k) CL_HIP(batch_launch(B, pd, B->parity));
      CL_HIP(hipEventRecord(e1, B->stream));
      CL_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      CL_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) { best = ms; bt = t; }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  B->tile = bt;
  return batch_upload(B);
}

}  // namespace cl

using namespace cl;

extern "C" {

int lattice_batch_workspace_size(const lattice_params* ps, int nruns, size_t* bytes) {
  int rc = batch_validate(ps, nruns);
  if (rc) return rc;
  if (!bytes) { set_error("bytes is NULL"); return LAT_EINVAL; }
  size_t ab, hdr;
  int64_t mt;
  batch_header(ps, nruns, &ab, &mt, &hdr);
  size_t tot = hdr;
  for (int r = 0; r < nruns; ++r) {
    size_t b = 0;
    rc = lattice_workspace_size(&ps[r], &b);
    if (rc) return rc;
    tot += aup(b);
  }
  *bytes = tot;
  return LAT_OK;
}

int lattice_batch_init(const lattice_params* ps, int nruns, void* dev_ws, size_t ws_bytes, void* hip_stream,
                       lattice_batch_t** out) {
  size_t need = 0;
  int rc = lattice_batch_workspace_size(ps, nruns, &need);
  if (rc) return rc;
  if (!dev_ws || !out) { set_error("NULL argument"); return LAT_EINVAL; }
  if (ws_bytes < need) { set_error("batch workspace too small: need " + std::to_string(need)); return LAT_ENOMEM; }
  if (((uintptr_t)dev_ws) % 256) { set_error("workspace must be 256-byte aligned"); return LAT_EINVAL; }
  lattice_batch* B = new lattice_batch();
  B->nruns = nruns;
  B->stream = (hipStream_t)hip_stream;
  B->fp32 = ps[0].precision == LAT_FP32;
  B->nf = ps[0].nf;
  B->use_graph = hip_stream != nullptr;
  size_t ab, hdr;
  int64_t mt;
  batch_header(ps, nruns, &ab, &mt, &hdr);
  char* ws = (char*)dev_ws;
  B->args_bytes = ab;
  B->max_tiles = mt;
  B->args[0] = ws;
  B->args[1] = ws + ab;
  size_t o = 2 * ab;
  B->tile_run = (int*)(ws + o);
  o += aup((size_t)mt * 4);
  B->tile_local = (int*)(ws + o);
  o += aup((size_t)mt * 4);
  B->tile_offset = (int*)(ws + o);
  o += aup((size_t)(nruns + 1) * 4);
  B->partials = (double*)(ws + o);
  o = hdr;
  for (int r = 0; r < nruns; ++r) {
    size_t b = 0;
    lattice_workspace_size(&ps[r], &b);
    lattice* h = nullptr;
    rc = lattice_init(&ps[r], ws + o, b, hip_stream, &h);
    if (rc) {
      for (lattice* x : B->runs) lattice_destroy(x);
      delete B;
      return rc;
    }
    B->runs.push_back(h);
    o += aup(b);
  }
  B->weights = vv_weights(ps[0].integrator);
  B->parity = 0;
  B->tile = Tiling{32, 8, 2, 8};
  rc = batch_autotune(B);
  if (rc) {
    for (lattice* x : B->runs) lattice_destroy(x);
    delete B;
    return rc;
  }
  *out = B;
  return LAT_OK;
}

int lattice_batch_step(lattice_batch_t* B, int64_t nsteps) {
  if (!B) { set_error("NULL batch"); return LAT_EINVAL; }
  if (nsteps < 0) { set_error("nsteps < 0"); return LAT_EINVAL; }
  if (nsteps == 0) return LAT_OK;
  int rc = sync_parity(B);
  if (rc) return rc;
  int stag = 0;
  const std::vector<PassDesc> sched = pass_schedule(B->runs[0]->p.integrator, B->weights, &stag, nsteps);
  const int start = B->parity;
  if (B->use_graph) {
    auto key = std::make_pair(nsteps, start);
    auto it = B->graphs.find(key);
    if (it == B->graphs.end()) {
      hipGraph_t g;
      hipGraphExec_t ge;
      CL_HIP(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
      int par = start;
      for (const PassDesc& pd : sched) {
        hipError_t e = batch_launch(B, pd, par);
        if (e != hipSuccess) {
          hipGraph_t dummy;
          (void)hipStreamEndCapture(B->stream, &dummy);
          set_error(std::string("batch capture: ") + hipGetErrorString(e));
          return LAT_EHIP;
        }
        par ^= 1;
      }
      CL_HIP(hipStreamEndCapture(B->stream, &g));
      CL_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
      it = B->graphs.emplace(key, std::make_pair(g, ge)).first;
    }
    CL_HIP(hipGraphLaunch(it->second.second, B->stream));
  } else {
    int par = start;
    for (const PassDesc& pd : sched) {
      CL_HIP(batch_launch(B, pd, par));
      par ^= 1;
    }
  }
  const int flips = (int)(sched.size() & 1);
  for (lattice* h : B->runs) {
    h->cur ^= flips;
    h->step += nsteps;
  }
  B->parity ^= flips;
  return LAT_OK;
}

int lattice_batch_energies(lattice_batch_t* B, lattice_obs* out) {
  if (!B || !out) { set_error("NULL argument"); return LAT_EINVAL; }
  for (int r = 0; r < B->nruns; ++r) {
    const int rc = lattice_energies(B->runs[r], &out[r]);
    if (rc) return rc;
  }
  return LAT_OK;
}

int lattice_batch_run(lattice_batch_t* B, int run, lattice_t** out) {
  if (!B || !out || run < 0 || run >= B->nruns) { set_error("bad batch run index"); return LAT_EINVAL; }
  *out = B->runs[run];
  return LAT_OK;
}

int lattice_batch_get_tiling(lattice_batch_t* B, int32_t* tz, int32_t* by, int32_t* ry, int32_t* xc) {
  if (!B) { set_error("NULL batch"); return LAT_EINVAL; }
  if (tz) *tz = B->tile.tz;
  if (by) *by = B->tile.by;
  if (ry) *ry = B->tile.ry;
  if (xc) *xc = B->tile.xc;
  return LAT_OK;
}

int lattice_batch_set_tiling(lattice_batch_t* B, int32_t tz, int32_t by, int32_t ry, int32_t xc) {
  if (!B) { set_error("NULL batch"); return LAT_EINVAL; }
  Tiling t{tz, by, ry, xc};
  if (!batch_tiling_ok(B, t)) { set_error("tile shape not compiled for batches or does not divide every N"); return LAT_EINVAL; }
  CL_HIP(hipStreamSynchronize(B->stream));
  drop_graphs(B);
  B->tile = t;
  return batch_upload(B);
}

int lattice_batch_use_graph(lattice_batch_t* B, int on) {
  if (!B) { set_error("NULL batch"); return LAT_EINVAL; }
  if (on && B->stream == nullptr) { set_error("graph capture needs a created stream"); return LAT_EINVAL; }
  B->use_graph = on ? 1 : 0;
  return LAT_OK;
}

int lattice_batch_destroy(lattice_batch_t* B) {
  if (!B) return LAT_OK;
  (void)hipStreamSynchronize(B->stream);
  drop_graphs(B);
  for (lattice* h : B->runs) lattice_destroy(h);
  delete B;
  return LAT_OK;
}

}  // extern "C"
