// pc_plain.h -- arguments of the per-iteration ("plain") path of pc_plain.hip.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include "pc_internal.h"

struct PcPlainArgs {
    PcParams p;                 // outputs, model and options shared with the fused path
    const PcGroupDev* g;        // device copy of this group's descriptor
    PcGroupDev g_host;          // host copy (interval)
    const PcJobDev* jobs;       // device: this group's jobs in IC order
    int n_jobs, N, NP, T, S;
    double t2;                  // tol^2
    int64_t Mpad;               // n_jobs * T columns
    double* Y;                  // [NP][9][Mpad]
    double* Y0;                 // [6][Mpad]
    int32_t *active, *dead, *notconv, *valid;   // [Mpad]
    int32_t *job_list, *job_list_out, *job_flag; // [n_jobs]
    int32_t* count;             // [4]: jobs in the current list, jobs in the compacted list,
                                //      jobs with a change above tol (accumulating, then as read)
};

// Workspace bytes of one group on the plain path.
size_t pc_plain_bytes(int NP, int n_jobs, int T);

// Host-side state of one group's propagation on the plain path.  The host loop of
// Sec. 5.4 is cut at its read-backs: pc_plain_begin enqueues the group's work up to the
// first read-back of the active-job count, and each pc_plain_advance, called once that
// read-back has landed in `host`, takes the loop decision and enqueues the work up to the
// next read-back (or the end of the group, after which `done` is set).  One host thread
// can so drive several groups on several streams, polling each stream's read-back.
struct PcPlainRun {
    PcPlainArgs a;
    int32_t* lists[2];          // device: active-job lists (current / compacted)
    int32_t* host;              // pinned host ints (3): the read-back
    void* stream;
    int s = 0, it = 0, cur = 0, count = 0, n_it = 0, status = -1;
    double w2 = 0.0;            // half-length of the current segment
    bool group = false, done = false;
};

// Lay out the group's state in `workspace` and enqueue its work up to the first read-back
// (returns a hipError_t).  host_count: pinned host ints (3).
int pc_plain_begin(PcPlainRun& r, const PcPlainArgs& a, void* workspace, int32_t* host_count, void* stream);
// The read-back enqueued last has completed: decide and enqueue the next part.
int pc_plain_advance(PcPlainRun& r);

// Propagate one group with per-iteration kernels and a host loop that waits on `stream`
// for each read-back (returns a hipError_t).
int pc_run_plain(PcPlainArgs a, void* workspace, int32_t* host_count, void* stream);
