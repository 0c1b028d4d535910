// Internal declarations shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.hpp"

namespace cl {

// Per-block shell histograms of a spectrum: the binning kernel's blocks, or
// the blocks of the transform's binning pass, at most spec_blocks(N).  Up to
// 256^3, 1024 (four per CU) make the quickest spectrum (at 256^3 the x pass
// takes the same time with 4096 and the reduction of the histograms half);
// larger lattices take more so that each block bins fewer line batches.
constexpr int kSpecBlocks = 1024;
inline int spec_blocks(int N) { return N > 256 ? 4 * kSpecBlocks : kSpecBlocks; }

struct Tiling {
  int tz, by, ry, xc;
};

}  // namespace cl

// Opaque handle of the C ABI.
struct lattice {
  lattice_params p;
  hipStream_t stream;
  char* ws;
  cl::DevState* st;     // state of the lattice between calls
  cl::DevState* st2;    // second state slot of a chain of passes
  double* partials;
  double* partials2;    // partial records of every other pass in a chain
  char* spec;           // spectrum partial histograms
  int64_t max_blocks;
  int ncomp;
  size_t comp_bytes;
  void* buf[2][40];     // ping-pong state buffers, per component
  void* fft;            // complex FP64 scratch of N^3 entries
  void* twiddle;        // N complex FP64 roots of unity for the FFT
  bool twiddle_ready = false;
  bool spec_geom_ready = false;  // shell centres and mode counts binned
  int cur;
  double dx;
  std::vector<double> weights;
  int staggered;
  int64_t step;
  cl::Tiling tile;
  std::vector<hipEvent_t> timer;  // start/stop pairs of timed pass launches
  size_t timer_used = 0;          // pairs recorded since the last read
};

namespace cl {

// compact or non-compact U(1) (10 components, the U(1) pass)
inline bool is_u1(const lattice_params& p) { return p.model == LAT_MODEL_U1 || p.model == LAT_MODEL_U1_NC; }
int ncomponents(const lattice_params* p);
int validate(const lattice_params* p);
PassDesc pass(double wd, double wk1, double wk2, int mode, int write, int update);
std::vector<PassDesc> pass_schedule(int integrator, const std::vector<double>& w, int* staggered, int64_t n);
void phys_of(const lattice* h, double* phys);
std::vector<double> vv_weights(int integrator);
int upload_components(lattice* h, const double* const* comps, int n);
int download_components(lattice* h, double* const* comps, int n);
int upload_scalars(lattice* h, double a, double b, double eta);
int init_state(lattice* h);
// A chain of stepping passes whose finishes are deferred: pass k reduces the
// partial records of pass k-1 at its start (PrevPass), the records alternate
// between two regions and the state between two slots, and one finish kernel
// closes the chain after its last pass.
struct PassChain {
  int k = 0;        // passes launched
  int rd = 0;       // state slot the next pass starts from (0: h->st, 1: h->st2)
  PrevPass prev{};  // finish still to be applied
};
int scalar_pass(lattice* h, const PassDesc& pd, bool full = false, PassChain* chain = nullptr);
int scalar_step(lattice* h, int64_t n);
int scalar_energies(lattice* h);
int u1_step(lattice* h, int64_t n);
int u1_energies(lattice* h);
int u1_init_state(lattice* h);
int u1_gauss(lattice* h);
// B_i of the U(1) model on the sites, into out (N^3 values, storage precision)
int u1_magnetic_field(lattice* h, int i, void* out);
// initial-state helpers shared by the charged-scalar models (u1.hip)
int charged_mode_field(lattice* h, int comp, int deriv, double m2eff, double Hhom, double base, double* out);
int gauss_solve_fields(lattice* h, const double2* R, void* const out[3], bool fp32);
// the SU(2) x U(1) doublet model (su2.hip)
inline bool is_su2(const lattice_params& p) { return p.model == LAT_MODEL_SU2U1; }
int su2_step(lattice* h, int64_t n);
int su2_energies(lattice* h);
int su2_init_state(lattice* h);
// device address of the static scratch of lattice_energies_noalloc, recorded
// once per device (noalloc.hip)
int noalloc_setup();
int run_fft3d(lattice* h, int sign, double scale);
bool tiling_ok(const lattice* h, const Tiling& t);
void default_tiling(lattice* h);
int autotune(lattice* h);

int u1_num_shapes(int fp32);
void u1_get_shape(int fp32, int i, int* tz, int* by, int* ry);
int u1_pass(lattice* h, const PassDesc& pd, PassChain* chain = nullptr);
int u1_chain_end(lattice* h, const PassChain& chain);
int scalar_chain_end(lattice* h, const PassChain& chain);
// blocks of a scalar observation pass (its fixed tile) at size N
int64_t scalar_obs_blocks(int N);
int num_shapes(int fp32, int nf);
void get_shape(int fp32, int nf, int i, int* tz, int* by, int* ry);
hipError_t launch_scalar_pass(int fp32, int nf, const void* const* src, void* const* dst, int N, int tz, int by,
                              int ry, int xc, int swizzle, const double* phys, int expand, const PassDesc& pd,
                              double* partials, DevState* st, hipStream_t s, int* nblocks_out, int full,
                              hipEvent_t ev0, hipEvent_t ev1, const PrevPass& prev, DevState* fin);
hipError_t launch_scalar_finish(int fp32, int nf, int N, const double* phys, int expand, const PassDesc& pd,
                                double* partials, int nblocks, DevState* in, DevState* out, hipStream_t s);

}  // namespace cl
