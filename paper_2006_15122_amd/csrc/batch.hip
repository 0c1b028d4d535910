// Batched ensembles of independent scalar lattices (sizes may differ).
//
// Every pass of every run goes through one batched kernel whose blocks are
// the tiles of all runs (tile table built on the host).  The finish of a pass
// (Sec. 4.3.2: each run's FP64 partials reduced in a fixed order, then a and
// b advanced) is carried by the next pass of the chain: every block reduces
// its own run's records of the previous pass before its first plane is
// consumed, the run's first tile stores the resulting state, and the records
// and states alternate between two regions and two slots per run.  One
// finish block per run closes the chain.  Kernel boundaries make each pass's
// results visible across XCDs with one L2 write-back per XCD, so no block
// ever waits on another.  A whole lattice_batch_step call is captured into a
// HIP graph and launched once; the graph is cached per (nsteps, buffer
// parity) and replayed by later calls with the same key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "scalar_tile.hpp"

namespace cl {

// The pending finish of a chain: pass `pd` wrote its records to `partials`
// (run r's at tile_offset[r] ..) starting from state slot `rd` of every run.
struct BatchPrev {
  const double* partials;  // nullptr: nothing pending
  PassDesc pd;
};

// slots[2 r + k]: state slot k of run r (k = 0 is the run's canonical state).
// Up to four rows per thread the kernel is held to four waves per SIMD, as
// the single-lattice pass is.
template <typename T, int NF, int TZ, int BY, int RY>
__global__ __launch_bounds__(TZ* BY, RY <= 4 ? 4 : 1) void batch_pass_kernel(
    const ScalarArgs<T>* runs, const int* tile_run, const int* tile_local, const int* tile_offset,
    DevState* const* slots, int rd, BatchPrev prev, double* partials, PassDesc pd) {
  // blocks are dealt to the XCDs in turn; this gives each XCD a contiguous
  // range of the tile table (neighbouring tiles of a run), so the halo rows
  // two tiles share are read through the same L2
  int b = blockIdx.x;
  if ((gridDim.x & 7) == 0) b = (b & 7) * (gridDim.x >> 3) + (b >> 3);
  const int r = tile_run[b], local = tile_local[b];
  ScalarArgs<T> A = runs[r];
  A.pd = pd;
  A.partials = partials;
  A.st = slots[2 * r + rd];
  const int first = tile_offset[r], nrec = tile_offset[r + 1] - first;
  DevState* const out = slots[2 * r + (rd ^ 1)];
  scalar_tile<T, NF, false, TZ, BY, RY>(A, local, b, [&](double& a_in, double& b_in) {
    if (prev.partials) {
      constexpr int NP = Acc<NF, false>::N;
      __shared__ double ab[2];
      double S[NP];
      if (reduce_partials<NP, TZ * BY>(prev.partials, first, nrec, S)) {
        double an, bn;
        finish_state<T, NF, false>(A, prev.pd, A.st, S, local == 0 ? out : nullptr, an, bn);
        ab[0] = an;
        ab[1] = bn;
      }
      __syncthreads();
      a_in = ab[0];
      b_in = ab[1];
    } else {
      a_in = A.st->a;
      b_in = A.st->b;
    }
  });
}

// Closing finish of a chain, one block per run: slot rd plus the last pass's
// records give the run's canonical state (slot 0).
template <typename T, int NF>
__global__ __launch_bounds__(256) void batch_finish_kernel(const ScalarArgs<T>* runs, const int* tile_offset,
                                                           DevState* const* slots, int rd, BatchPrev prev) {
  const int r = blockIdx.x;
  constexpr int NACC = Acc<NF, false>::N;
  double S[NACC];
  const int first = tile_offset[r];
  if (!reduce_partials<NACC, 256>(prev.partials, first, tile_offset[r + 1] - first, S)) return;
  ScalarArgs<T> A = runs[r];
  double an, bn;
  finish_state<T, NF, false>(A, prev.pd, slots[2 * r + rd], S, slots[2 * r], an, bn);
}

#define CL_BATCH_SHAPES(X) \
  X(32, 8, 2)              \
  X(32, 4, 4)              \
  X(32, 8, 4)              \
  X(64, 4, 2)              \
  X(64, 4, 4)

static const int kBatchShapes[][3] = {{32, 8, 2}, {32, 4, 4}, {32, 8, 4}, {64, 4, 2}, {64, 4, 4}};

// The chain of one lattice_batch_step call (or of an autotuning run).
struct BatchChain {
  int k = 0;         // passes launched
  int rd = 0;        // state slot the next pass starts from
  BatchPrev prev{};  // finish still to be applied
};

template <typename T, int NF>
static hipError_t launch_batch_t(const Tiling& t, int ntiles, const void* runs, const int* tile_run,
                                 const int* tile_local, const int* tile_offset, DevState* const* slots,
                                 double* partials, const PassDesc& pd, const BatchChain& c, hipStream_t s) {
  const ScalarArgs<T>* R = static_cast<const ScalarArgs<T>*>(runs);
  bool ok = false;
#define X(a, b, cc)                                                                                            \
  if (!ok && t.tz == a && t.by == b && t.ry == cc) {                                                           \
    hipLaunchKernelGGL((batch_pass_kernel<T, NF, a, b, cc>), dim3(ntiles), dim3(a * b), 0, s, R, tile_run,   \
                       tile_local, tile_offset, slots, c.rd, c.prev, partials, pd);                           \
    ok = true;                                                                                                 \
  }
  CL_BATCH_SHAPES(X)
#undef X
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T, int NF>
static hipError_t launch_batch_end_t(int nruns, const void* runs, const int* tile_offset, DevState* const* slots,
                                     const BatchChain& c, hipStream_t s) {
  hipLaunchKernelGGL((batch_finish_kernel<T, NF>), dim3(nruns), dim3(256), 0, s,
                     static_cast<const ScalarArgs<T>*>(runs), tile_offset, slots, c.rd, c.prev);
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
  cl::DevState** slots;  // [2 nruns]: each run's two state slots
  double* partials[2];   // the records of consecutive passes alternate
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
  o += aup((size_t)nruns * 2 * sizeof(void*));
  o += 2 * aup((size_t)mt * 4 * sizeof(double));
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

// One pass of a chain; the records go to the region the pass number picks.
static hipError_t batch_launch(lattice_batch* B, const PassDesc& pd, int parity, BatchChain& c) {
  const void* args = B->args[parity];
  double* part = B->partials[c.k & 1];
  hipError_t e;
  auto go = [&](auto* tag, auto nf) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return launch_batch_t<T, decltype(nf)::value>(B->tile, B->ntiles, args, B->tile_run, B->tile_local,
                                                  B->tile_offset, B->slots, part, pd, c, B->stream);
  };
  if (B->fp32)
    e = B->nf == 1 ? go((float*)nullptr, std::integral_constant<int, 1>{})
                   : go((float*)nullptr, std::integral_constant<int, 2>{});
  else
    e = B->nf == 1 ? go((double*)nullptr, std::integral_constant<int, 1>{})
                   : go((double*)nullptr, std::integral_constant<int, 2>{});
  if (e != hipSuccess) return e;
  if (c.prev.partials) c.rd ^= 1;
  c.prev = BatchPrev{part, pd};
  ++c.k;
  return hipSuccess;
}

// Closing finish: every run's canonical state from the chain's last pass.
static hipError_t batch_chain_end(lattice_batch* B, const BatchChain& c) {
  if (c.k == 0) return hipSuccess;
  const void* args = B->args[0];
  if (B->fp32)
    return B->nf == 1 ? launch_batch_end_t<float, 1>(B->nruns, args, B->tile_offset, B->slots, c, B->stream)
                      : launch_batch_end_t<float, 2>(B->nruns, args, B->tile_offset, B->slots, c, B->stream);
  return B->nf == 1 ? launch_batch_end_t<double, 1>(B->nruns, args, B->tile_offset, B->slots, c, B->stream)
                    : launch_batch_end_t<double, 2>(B->nruns, args, B->tile_offset, B->slots, c, B->stream);
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

// Time every shape and x-chunk in two sweeps (six chained passes each, after
// a warm-up pass) and keep the one with the smallest time of the two: one
// short timing picked x-chunks 8 and 16 in turn between runs of the same
// ensemble, a spread of 6% in the pass time.
static int batch_autotune(lattice_batch* B) {
  hipEvent_t e0, e1;
  CL_HIP(hipEventCreate(&e0));
  CL_HIP(hipEventCreate(&e1));
  const int xcs[] = {8, 16, 32};
  std::vector<Tiling> cands;
  for (const auto& s : kBatchShapes)
    for (int xc : xcs) {
      Tiling t{s[0], s[1], s[2], xc};
      if (batch_tiling_ok(B, t)) cands.push_back(t);
    }
  std::vector<float> tmin(cands.size(), 1e30f);
  // chained passes into the other buffers that leave a and b as they are
  // (update 0), as lattice_batch_step chains them; the closing finish
  // stores only observables
  const PassDesc pd = pass(1.0, 0.5, 0.5, MODE_VV, 1, 0);
  for (int sweep = 0; sweep < 2; ++sweep)
    for (size_t i = 0; i < cands.size(); ++i) {
      B->tile = cands[i];
      int rc = batch_upload(B);
      if (rc) return rc;
      BatchChain warm;
      CL_HIP(batch_launch(B, pd, B->parity, warm));
      CL_HIP(batch_chain_end(B, warm));
      BatchChain c;
      CL_HIP(hipEventRecord(e0, B->stream));
      for (int k = 0; k < 6; ++k) CL_HIP(batch_launch(B, pd, B->parity, c));
      CL_HIP(batch_chain_end(B, c));
      CL_HIP(hipEventRecord(e1, B->stream));
      CL_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      CL_HIP(hipEventElapsedTime(&ms, e0, e1));
      tmin[i] = std::min(tmin[i], ms);
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  size_t bi = 0;
  for (size_t i = 1; i < cands.size(); ++i)
    if (tmin[i] < tmin[bi]) bi = i;
  if (!cands.empty()) B->tile = cands[bi];
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
  B->slots = (DevState**)(ws + o);
  o += aup((size_t)nruns * 2 * sizeof(void*));
  B->partials[0] = (double*)(ws + o);
  o += aup((size_t)mt * 4 * sizeof(double));
  B->partials[1] = (double*)(ws + o);
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
  {
    std::vector<DevState*> sl;
    for (lattice* h : B->runs) {
      sl.push_back(h->st);
      sl.push_back(h->st2);
    }
    rc = LAT_OK;
    if (hipMemcpyAsync(B->slots, sl.data(), sl.size() * sizeof(DevState*), hipMemcpyHostToDevice, B->stream) !=
            hipSuccess ||
        hipStreamSynchronize(B->stream) != hipSuccess) {
      set_error("batch: uploading the state-slot table failed");
      rc = LAT_EHIP;
    }
    if (rc) {
      for (lattice* x : B->runs) lattice_destroy(x);
      delete B;
      return rc;
    }
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
      BatchChain c;
      for (size_t i = 0; i <= sched.size(); ++i) {
        hipError_t e = (i < sched.size()) ? batch_launch(B, sched[i], par, c) : batch_chain_end(B, c);
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
    BatchChain c;
    for (const PassDesc& pd : sched) {
      CL_HIP(batch_launch(B, pd, par, c));
      par ^= 1;
    }
    CL_HIP(batch_chain_end(B, c));
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
