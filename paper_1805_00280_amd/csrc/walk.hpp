// walk.hpp -- parameter blocks of the walk kernels and the entry points the
// autotuner and the server use.
#pragma once

#include "common.hpp"

namespace n2v {

// Graph view and execution parameters shared by every walk of a launch.
// Execution parameters never change results.
struct Exec {
    DevGraph g;
    uint32_t t_wave;        // rejection moves at degree > t_wave run wave-cooperatively
    uint32_t t_sparse;      // largest deg(t) for the sparse hub path
    uint32_t sparse_ratio;  // cost weight of one search against streaming
    uint32_t t_wg;          // plain form: dense hub moves at degree > t_wg use a whole workgroup
    uint32_t search_ratio;  // dense merges search N(v) in N(t) when N(t)'s range is longer by more
    uint32_t thread_iters;  // persistent form: rejection moves a lane takes before the wave serves pending walks
    uint32_t *cursor;       // walk counter of a single-job launch (taken per launch, zeroed before it)
};

// Parameters of one walk job: a set of walks with the same (L, p, q, seed).
// The common-neighbour multiplier is the constant K = 4.
struct JobCtx {
    uint32_t *out;                 // n x (L+1) rows or null
    uint32_t *cnt;                 // visit counts or null
    unsigned long long *checksum;  // or null
    uint32_t wbase;                // walk id of the job's walk 0, modulo 2^32
    uint32_t L;
    uint32_t k0, k1;               // Philox key = seed
    uint32_t A_ret, A_out;         // 4/p and 4/q
    uint32_t approx_t;             // FN-Approx threshold 1/approx_t (0: exact)
};

// One job of a serving table: its context plus its start ids.
struct alignas(16) JobRec {
    JobCtx c;
    const uint32_t *starts;
    uint32_t n;
};

constexpr uint32_t MAX_TABLE_JOBS = 256;

// A table of jobs as the persistent kernel reads it from device memory.
struct alignas(256) TableHdr {
    uint32_t njobs;
    uint32_t total;                         // sum of the job sizes
    uint32_t cursor;                        // next unassigned walk (0 in the host copy)
    uint32_t jstart[MAX_TABLE_JOBS + 1];    // prefix sums of the job sizes
    JobRec jobs[MAX_TABLE_JOBS];
};

int walk_multipliers(float p, float q, uint32_t *A_ret, uint32_t *A_out);
void make_exec(const n2v_graph *g, const n2v_exec_opts &o, Exec *E);
uint32_t full_grid_blocks(int dev);
int launch_job_table(const Exec &E, const TableHdr *hdr, uint32_t blocks, hipStream_t st);
// One persistent launch of a single job on the graph's walk counters.
int launch_one(const n2v_graph *g, const Exec &E, const JobCtx &c, const uint32_t *starts, uint32_t n,
               const n2v_exec_opts &o, hipStream_t st);

}  // namespace n2v
