// Internal declarations shared by the host API and the kernel launchers of
// libbfly.  Not installed; the public interface is include/bfly.h.
//
// Weight layout (in place across all levels).  The N^d (A,B) pairs of every
// level live in N^d slots of r complex values per right-hand side.  The
// right-hand sides are processed in chunks of RC (the phase factors are
// shared within a chunk); a chunk's weights are [slot][node][RC], and the
// chunks follow one another (right-hand side k's chunk starts at k N^d r).
// Viewing a slot index as L digits of d bits, at level l the low l digits
// hold the target box A (digit k = the bits of A's (k+1)-th split, coarsest
// first) and the high L - l digits hold the source box B in Morton order
// (finest digit lowest).  Stage l merges the 2^d source children (digit l)
// and splits the target into 2^d children, which land in the same digit:
// each merge-and-split group reads and writes the same 2^d slots.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bfly {

constexpr int kQMax = 16;

// Geometry and phase of one apply, in the roles of that apply: for the
// adjoint the plan's target box plays the source role and vice versa, and
// `adj` negates and transposes the phase.  Passed to kernels by value.
struct Geo {
  int d, L, q, r;      // dimension, log2 N, nodes per dim, q^d
  int ls, phase, adj;  // switch level, phase id, adjoint flag
  int nc;              // 2^d
  double Nd;           // N as a double (scale inside the phase)
  double slo[3], sD[3];  // source-role box: lower corner, extent
  double tlo[3], tD[3];  // target-role box
  double z[kQMax];       // 1-D Chebyshev nodes of the first kind
};

// Device workspace carved into typed pieces (see carve()).
struct Work {
  void* W = nullptr;            // weights: per chunk of RC right-hand sides [P][r][RC] complex
  uint32_t* keys = nullptr;     // leaf key per input point
  uint32_t* keys_sorted = nullptr;
  int32_t* idx = nullptr;       // batched: index of each point inside its instance
  int32_t* perm = nullptr;      // input points sorted by leaf (stable)
  int32_t* offs = nullptr;      // CSR offsets per leaf, P + 1
  int32_t* empty = nullptr;     // set by binning: 1 if some leaf holds no input point
  uint8_t* tocc = nullptr;      // target-box occupancy, levels 0..L (see tocc_bytes)
  void* sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
};

// Optional per-step timing (bfly_timing_enable): a scope records a HIP
// event pair around the launches it encloses when timing is on.
enum StepKind { kStepBin = 0, kStepFirst, kStepSecond, kStepFinal, kNumSteps };
class StepTimer {
 public:
  // stages / inits / switches: work the enclosed launch performs
  StepTimer(int kind, hipStream_t s, int stages = 0, int inits = 0, int switches = 0);
  ~StepTimer();
  StepTimer(const StepTimer&) = delete;
  StepTimer& operator=(const StepTimer&) = delete;

 private:
  int kind_, stages_, inits_, switches_;
  hipStream_t s_;
  hipEvent_t b_ = nullptr;
};
bool timing_on();
// One timed launch: its kind, the work it performed, its duration.
struct LaunchRecord {
  int kind, stages, inits, switches;
  double ms;
};
// Copies up to cap records of the launches collected by the last
// timing_read, in launch order; returns how many there are.
int timing_launches(int cap, LaunchRecord* out);
hipError_t timing_read(double* ms, int64_t* launches, int64_t* stages, int64_t* inits, int64_t* switches);
void timing_set(bool on);

// Bytes of weight storage for one apply.
size_t weight_bytes(const Geo& g, int nrhs, int prec);
// Bytes of the target-box occupancy pyramid (levels 0..L, 2^(d l) boxes at
// level l, one byte each, stored by level, a box at the Morton index of its
// l-digit index), rounded up to whole words.
size_t tocc_bytes(int d, int L);
// Bytes of scratch the leaf-key radix sort needs for n keys of `bits` bits.
hipError_t sort_storage_bytes(int64_t n, int bits, size_t* bytes);

// Everything the level kernels of one apply need (after binning).
struct LevelArgs {
  const Geo* G = nullptr;
  void* W = nullptr;             // weights (FP64 or FP32 complex)
  int nrhs = 1;
  const double* pts_in = nullptr;
  const double* vals_in = nullptr;
  int64_t ld_in = 0;
  const int32_t* perm = nullptr;
  const int32_t* offs = nullptr;
  const int32_t* empty = nullptr;  // device flag: 1 if some leaf holds no input point
  const uint8_t* tocc = nullptr;   // target-box occupancy when targets are sparse, else null
  int64_t n_out = 0;
  const double* pts_out = nullptr;
  double* vals_out = nullptr;
  int64_t ld_out = 0;
  hipStream_t stream = nullptr;
  int ub_force = 0;              // fusion units per workgroup block, every launch (0: see below)
  int ub_first = 0, ub_second = 0;  // per launch kind (0: chosen per launch)
  int rc_one = 0;                // 1: one right-hand side per workgroup (no chunks)
  int k_fuse = 0;                // merge-and-split stages fused per launch, at most (0: by shape)
  // tuning override: stages of each launch, column-space launches then
  // row-space ones (used only when they add up to each half and fit the LDS)
  int split[16] = {0};
  int nsplit = 0;
  size_t lds_budget = 81920;     // bytes of LDS per workgroup (two workgroups per CU)
  // debugging override (single applies): run only the level launches that
  // end within the first stop_stages stages and no final evaluation, so that
  // the weight buffer keeps that level's weights (-1: the whole apply)
  int stop_stages = -1;
};
// Launch-shape limits of one (d, q, phase, precision): the right-hand-side
// chunk of its kernels and the most stages a launch can fuse with chunks
// and with one right-hand side per workgroup.
struct ShapeLimits {
  int rc = 1, kmax_rc = 1, kmax_one = 1;
  // built-in stages per launch of the column-space and row-space halves
  int kcol_rc = 1, krow_rc = 1, kcol_one = 1, krow_one = 1;
};
hipError_t shape_limits(const Geo& g, int prec, ShapeLimits* out);
hipError_t shape_limits_d1(const Geo& g, int prec, ShapeLimits* out);
hipError_t shape_limits_d2(const Geo& g, int prec, ShapeLimits* out);
hipError_t shape_limits_d3(const Geo& g, int prec, ShapeLimits* out);

// Launch shapes of one apply chosen by the autotuner (bfly_tune); zero
// fields keep the built-in choice.
struct TuneParams {
  int ub_first = 0, ub_second = 0, rc_one = 0, nsplit = 0;
  int split[16] = {0};
};
// Tuned shapes for (current device, geometry, nrhs, precision): true and *p
// filled if there is a record.  The first call loads BFLY_TUNE_CACHE.
bool tune_lookup(const Geo& g, int nrhs, int prec, TuneParams* p);
// Record tuned shapes (and write BFLY_TUNE_CACHE if set); ms is the time
// per apply that was measured with them.
hipError_t tune_store(const Geo& g, int nrhs, int prec, const TuneParams& p, double ms);
// Forget every record (tests).
void tune_clear();

hipError_t run_levels_d1(const LevelArgs& la, int prec);
hipError_t run_levels_d2(const LevelArgs& la, int prec);
hipError_t run_levels_d3(const LevelArgs& la, int prec);

// ---- batched applies: many instances, level-synchronous launches ----

// One instance of a batched apply after binning (host side).
struct BatchInst {
  Geo G;
  void* W = nullptr;                 // this instance's weights
  int nrhs = 1;
  const double* pts_in = nullptr;
  const double* vals_in = nullptr;   // complex128 [nrhs][ld_in]
  int64_t ld_in = 0;
  const int32_t* offs = nullptr;     // CSR offsets of this instance's source leaves
  int64_t n_out = 0;
  const double* pts_out = nullptr;
  double* vals_out = nullptr;        // complex128 [nrhs][ld_out]
  int64_t ld_out = 0;
};

// Device descriptor of one (instance, range of right-hand sides) of a
// batched apply; the batched level kernels read it with scalar loads.
struct ItemDesc {
  Geo G;
  void* W;                 // weights, shifted to the first right-hand side of the range
  const double2* vals_in;  // input values, shifted likewise
  double2* vals_out;       // output values, shifted likewise
  const double* pts_in;
  const double* pts_out;
  const int32_t* offs;
  int64_t ld_in, ld_out, n_out;
  int nrhs;                // right-hand sides of the instance
  int chunks;              // chunks of RC right-hand sides in the range
};

// Instances that share d, q, phase and role (forward or adjoint).
struct BatchGroup {
  const BatchInst* inst = nullptr;
  int n = 0;
  const int32_t* perm = nullptr;  // all instances' input points sorted by (instance, leaf)
  const int32_t* empty = nullptr; // device flag: 1 if some leaf of some instance holds no point
  ItemDesc* desc = nullptr;       // device room for 2 n descriptors
  hipStream_t stream = nullptr;
  int k_fuse = 0;
  size_t lds_budget = 81920;
  int ub_force = 0;
};
hipError_t run_batch_d1(const BatchGroup& bg, int prec);
hipError_t run_batch_d2(const BatchGroup& bg, int prec);
hipError_t run_batch_d3(const BatchGroup& bg, int prec);

// Copy n descriptors from host memory to device memory through kernel
// arguments (no host-to-device copy, so the call can be captured).
hipError_t put_items(ItemDesc* dst, const ItemDesc* src, int n, hipStream_t st);

// Input points of one instance for the batched binning.
struct BinInst {
  const double* pts = nullptr;
  int64_t n = 0;
  const Geo* G = nullptr;
  uint32_t leafbase = 0;  // sum of the leaf counts of the instances before it
};
// Bin all instances' input points in one sort: key = leaf base + leaf
// Morton index, value = the point's index within its instance; w.offs gets
// leaves_total + 1 CSR offsets.
hipError_t bin_batch(const BinInst* bi, int n, int64_t n_total, uint64_t leaves_total, const Work& w,
                     hipStream_t st);
// Launch-shape overrides (BFLY_UB, BFLY_KFUSE, BFLY_LDS) for batched applies.
void tune_batch_from_env(BatchGroup& bg);

// Enqueue one apply (binning, initialisation, stages, switch, final
// evaluation) on `stream`.  Inputs were validated by the caller.
// `force` (may be null) gives the launch shapes to use; otherwise the
// tuning table's record for this apply, if any, else the built-in choice.
// BFLY_UB / BFLY_KFUSE / BFLY_LDS / BFLY_KSPLIT override both.
hipError_t run_apply(const Geo& g, int prec, int64_t n_in, const double* pts_in,
                     const double* vals_in, int64_t ld_in, int64_t n_out,
                     const double* pts_out, double* vals_out, int64_t ld_out, int nrhs,
                     const Work& w, hipStream_t stream, const TuneParams* force = nullptr);

}  // namespace bfly
