// batch.hpp -- shared definitions of the batched (persistent-kernel) path.
#pragma once

#include <hip/hip_runtime.h>

#include "desc.hpp"
#include "shapes.hpp"

namespace lsr {

// Group kernels compiled for one local-step model m alone carry the code
// ANY_FIXED + m (see GroupInfo::any_model).
enum : int { ANY_FIXED = 16 };

enum : int { TASK_ROW = 0, TASK_COL = 1 };

// Control block of a group (device, unsigned words).
// CTRL_SPIN and CTRL_EXTRA are set by the host only (zero by default): the
// column tasks' poll limit (0 = about 2 s) and a count added to the row
// blocks a column task waits for (a nonzero value makes every wait give up:
// the failure path, exercised from the host).
enum : int { CTRL_HEAD = 0, CTRL_EXIT = 1, CTRL_NCAV = 2, CTRL_ABORT = 3, CTRL_SPIN = 4, CTRL_EXTRA = 5,
             CTRL_ROWDONE = 16 };

// Optional timestamps of one dispatch: when either event is set the launch
// goes through hipExtLaunchKernelGGL, which records the kernel's own start
// and end on the events (no gaps of events recorded around it).
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

struct KernelVariant {
    // persistent kernel: one launch per round trip
    int (*launch)(int mode, int grid, hipStream_t st, const CavDesc* descs, const int4* tasks, int ntasks,
                  unsigned* ctrl, int chunk, LaunchEvents ev);
    // grouped launch: one launch per pass, one workgroup per task
    int (*launch_pass)(int mode, int kind, hipStream_t st, const CavDesc* descs, const int4* tasks, int ntasks,
                       LaunchEvents ev);
    int (*occupancy)();
    int waves_per_eu;    // register budget the variant was compiled for
    // software-pipelined grouped pass (single-size groups only; else null)
    int (*launch_pipe)(int mode, int kind, hipStream_t st, const CavDesc* descs, const int4* tasks, int ntasks,
                       int grid, LaunchEvents ev);
    int (*occupancy_pipe)(int kind);
};

struct GroupInfo {
    int threads;
    int nsizes;
    int sizes[8];
    ShapeInfo shapes[8];   // the FFT plan of each size
    int alt;               // 0: the sizes' default plans; k > 0: alternative plan k
    int any_model;         // 0: the default local step; 1: each cavity's own local-step
                           // model; 2: also the mirror roughness; ANY_FIXED + m: model m
                           // alone
    int nvariants;
    KernelVariant var[4];
};

// Compiled groups, smallest first; the batch picks, for its sizes, the
// first group that contains all of them (per workgroup size).
int group_count();
const GroupInfo* group_at(int i);

// Row blocks per cavity of size N in the FP32 shapes (0 if unsupported).
int row_blocks(int N);

}  // namespace lsr
