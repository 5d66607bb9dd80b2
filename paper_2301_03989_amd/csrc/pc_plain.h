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

// Propagate one group with per-iteration kernels and a host loop (returns a hipError_t).
// host_count: pinned host ints (3) used for the per-iteration read-back.
int pc_run_plain(PcPlainArgs a, void* workspace, int32_t* host_count, void* stream);
