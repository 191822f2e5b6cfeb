// Pass kernels generated from a plan and compiled at run time (hipRTC).
//
// The interpreted pass kernels decode every op record on every tile. A
// generated kernel has the op sequence, the register/lane slots, the phase
// layouts, the I/O address constants and the pass flags of one lowered pass
// fixed at compile time; only the matrix entries (and the tile table, source
// and destination) are read at run time, from the same records. All tasks
// whose passes lower to the same structure (for example the tasks of one
// parameterised circuit) share one kernel. The op code is the one of
// qw_dev.h, so a generated kernel rounds exactly as the interpreter does.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "qw_internal.h"

namespace qw {

// Exact structural key of a lowered pass: op types, bit locations, slots,
// phase layouts, flags, tile bits and kernel form. Two passes with the same
// key run the same generated kernel.
std::string jit_pass_key(int n, int m, const HostPass &p, bool use_lds);

// Full HIP source of the generated kernel for a key's pass; `prefetch`
// (0..16, even) is the number of registers of the next tile the persistent
// form loads while working on the current one.
// `stream_loads`: the pass's state loads are non-temporal (its stores always
// are); false for a pass that reads a boundary snapshot other tasks share.
std::string jit_pass_source(int n, int m, const HostPass &p, bool use_lds, int prefetch = 16,
                            const RedPlan *epi = nullptr, bool stream_loads = true);

// Key suffix of a pass kernel with a fused expectation epilogue.
std::string jit_epilogue_key(int n, int m, const HostPass &p, const RedPlan &epi);

struct JitKernel {
    hipFunction_t fn = nullptr;
    bool use_lds = false;
    int m = 0;
    int wg = 0;            // threads per workgroup
    int parts = 1;         // workgroups per tile (flat form)
    int blocks_per_cu = 1; // resident workgroups per CU (LDS form)
    int row_tiles = 1;     // reducers and pass kernels with an expectation
                           // epilogue: tiles per item (a row of kRedRowTiles)
};

// Exact structural key and source of the generated expectation reducer of
// one term group (its terms, register phases and columns are fixed at
// compile time; the state slot, partial-sum array and tile table are read at
// run time).
std::string jit_reduce_key(int n, int m, const TermGroup &g, const RedPlan &rp);
std::string jit_reduce_source(int n, int m, const TermGroup &g, const RedPlan &rp);

// One pass structure of a persistent kernel (all of one m and n).
struct PersistPart {
    const HostPass *pass = nullptr;
    const RedPlan *epi = nullptr;          // fused expectation epilogue
    const std::string *epi_key = nullptr;  // its key suffix
    int n = 0, m = 0;
    bool stream_loads = true;
};

// Key and source of the persistent kernel of a call: every listed pass
// structure in one code object, dispatched per claim (see PSeg).
std::string jit_persist_key(const std::vector<PersistPart> &parts);
std::string jit_persist_source(const std::vector<PersistPart> &parts, int prefetch = 16);

// One requested kernel: its key and what it was computed from (a pass, a
// reducer term group, or the pass structures of a persistent kernel).
struct JitReq {
    std::string key;
    const std::vector<PersistPart> *persist = nullptr;
    const HostPass *pass = nullptr;
    const TermGroup *group = nullptr;
    const RedPlan *rplan = nullptr;
    const RedPlan *epi = nullptr;  // pass kernels: fused expectation epilogue (persistent form)
    int n = 0, m = 0;
    bool use_lds = false;  // pass kernels: persistent LDS form
    bool stream_loads = true;  // pass kernels: non-temporal state loads
};

// Launch a generated reducer over n_descs descriptors of its term group.
hipError_t jit_launch_reduce(hipStream_t st, const JitKernel &k, const ReduceDesc *descs,
                             uint32_t n_descs, uint32_t tiles, uint32_t cu_count, bool tile_major);

// Compiled kernels for the requests on `device`: loaded from memory, from
// the disk cache, or compiled (in parallel). Returns "" or an error message.
std::string jit_get(int device, const std::vector<JitReq> &reqs, std::vector<const JitKernel *> *out);

// True when the kernel of a request is loaded on `device` or its code
// object is in the process or disk cache (no compilation).
bool jit_available(int device, const JitReq &r);

// Compile (or load from the disk cache) the code objects of the requests
// without loading them on a device; no GPU is needed.
std::string jit_precompile(const std::vector<JitReq> &reqs);

// Launch a generated pass kernel over n_descs descriptors (all of its key).
// `tile_major`: the persistent form takes consecutive tiles of one
// descriptor (else the descriptors of one tile) as consecutive items.
hipError_t jit_launch(hipStream_t st, const JitKernel &k, const PassDesc *descs, uint32_t n_descs,
                      uint32_t tiles, int remap, uint32_t cu_count, bool tile_major);

// Launch a persistent kernel over `claims` claims of n_segs segments on
// `grid` workgroups (see PSeg, PDep; sync holds kSyncCounters + descriptor
// count words, zero at launch).
hipError_t jit_launch_persist(hipStream_t st, const JitKernel &k, const PSeg *segs, uint32_t n_segs,
                              const PassDesc *descs, const PDep *deps, uint32_t *sync, uint32_t claims,
                              uint32_t grid, uint32_t spin_limit, uint32_t *host_flag);

// Number of generated kernels compiled (not loaded from cache) and seconds
// spent compiling, since the process started.
void jit_stats(uint64_t *compiled, uint64_t *cache_hits, double *compile_s);

}  // namespace qw
