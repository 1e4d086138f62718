// Device-visible job and task descriptors of the persistent batch kernel.
#pragma once
#include "plan.hpp"

namespace he {

enum PTaskKind : uint32_t { PT_FWD_CT = 0, PT_PT = 1, PT_MAC_INV = 2 };
enum PlainKind : uint32_t { PK_CONV = 0, PK_FC = 1, PK_POLY = 2, PK_CONV_DX = 3 };

// control words: pre-task queue head, error flag, one head per XCD queue of
// dependent tasks (each on its own 128-byte line), then one completion counter
// per job
enum : uint32_t { CTL_HEAD = 0, CTL_ERR = 1, CTL_XQ = 32, CTL_DONE = 32 + 8 * 32 };
constexpr int kXcds = 8;
// polls of a dependency counter before a waiting workgroup gives up and raises
// the error flag (about 1 s at the longest back-off)
constexpr uint32_t kSpinLimit = 1u << 20;

// A task: planes [first, first + count) of the job's array.  kind carries
// PT_WAIT when the job has pre tasks that a dependent task must wait for.  A
// multiply-accumulate task of one plane also carries its output's term range
// [t0, t1) and the planes of its first term's operands (a0 in the transformed
// inputs, b0 in the transformed plaintexts), so it starts its operand loads
// without reading the term lists; t1 < 0: read them (several planes per task).
enum : uint32_t { PT_KIND_MASK = 0xFFu, PT_WAIT = 0x100u };
struct PTask {
  uint32_t kind, job, first, count;
  int32_t t0, t1;
  uint32_t a0, b0;
};

struct PJob {
  const PrimeK *primes;
  const void *tw_fwd, *tw_inv;
  const double *tw_inv_w;   // fp64: the inverse twiddles alone, [L][N]
  const uint64_t *ct_in;
  uint64_t *ct_hat;      // == ct_in when the inputs are already transformed
  const void *plain;
  uint64_t *pt_hat;
  uint64_t *ct_out;
  const int32_t *row, *cti, *pti;
  uint32_t logN, L, n_pre, accumulate;
  uint32_t pkind;
  uint32_t M, C, h, O, S, Cw, cb;
  uint32_t n_in, n_out, n_iw, n_ow, in_ct;
  uint32_t ct_f64;       // fp64 batch: ct_hat holds the batch's own doubles (not the caller's residues)
};

// One job as the task-table builder sees it.
struct JobRef {
  Ctx *ctx;
  const Plan *plan;
  he_job job;
  bool canon_ct = false;   // keep the transformed inputs as canonical residues (read again by later jobs)
};

// Device workspace a job needs inside a persistent launch: transformed inputs
// (unless already transformed) first, at offset 0 as in the per-layer path's
// workspace, then the transformed plaintexts.
size_t job_ws_bytes(const JobRef &j);
// Task table and device job descriptors for `jobs`, with job k's workspace at
// ws[k].  Every pre task precedes every multiply-accumulate task.
// Dependent tasks are split into kXcds contiguous queues, [xq[x], xq[x+1]) in
// the task table, one per XCD; pre tasks are [0, xq[0]).
he_status build_tables(const std::vector<JobRef> &jobs, const std::vector<char *> &ws, int arith, int slab,
                       std::vector<PTask> &tasks, std::vector<PJob> &pjobs, he_batch_info &info,
                       uint32_t xq[kXcds + 1]);

// A compiled variant of the persistent kernel.
struct PVariant {
  int arith, slab, loge, logn_min, logn_max;
  int threads = 0, lds_bytes = 0, wg_per_cu = 1;
};
bool persistent_variant(int arith, uint32_t logn_min, uint32_t logn_max, int pref_loge, PVariant &v);
struct XQ {
  uint32_t b[kXcds + 1];   // queue bounds in the task table
};
// ev0 / ev1 (optional): recorded on `st` right before and after the persistent kernel.
// clear_err: zero the error flag with the other control words (otherwise it
// stays set from earlier launches until the caller clears it).
hipError_t launch_persistent(const PVariant &v, const PTask *tasks, uint32_t n_tasks, const XQ &xq, const PJob *jobs,
                             uint32_t n_jobs, uint32_t *ctl, uint32_t ctl_words, uint32_t grid, uint32_t spin_limit,
                             uint32_t strict, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                             bool clear_err = false);

}  // namespace he
