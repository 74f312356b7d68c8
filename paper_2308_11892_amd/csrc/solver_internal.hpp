// solver_internal.hpp -- the two halves of cptr_setup, for the serving runtime.
//
// cptr_setup = setup_host (validation, host AMG and ILU(0) setup; no device
// call) + setup_device (device layouts and uploads).  measure_device runs the
// device half without touching the device and returns the exact bytes it would
// allocate (in DevArena pieces), so a request can be admitted by its HBM
// footprint before any of it is allocated.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cptr.h"
#include "dev_arena.hpp"

namespace cptr {

// Host half.  On success *out is a handle with no device state.  The handle
// reads A's values in place until drop_input is called: the caller keeps them
// alive until then (setup_device reads them).  With early_stream set (and a
// device handle), the part of the device half that needs only A (its layout,
// the weights, the ILU(0) factors and sweep orders) is built on that stream by
// a second thread while this one builds the AMG hierarchy; the handle then has
// that part when this returns, and setup_device adds the rest.
int setup_host(const cptr_bsr* A, int32_t block_size, const int32_t* elliptic_idx, int32_t n_elliptic,
               const cptr_setup_opts* opts, cptr_solver* out, const hipStream_t* early_stream = nullptr);
// Device bytes setup_device(s, arena, restart, flexible) allocates, counted in
// DevArena pieces.
int measure_device(cptr_solver s, int restart, bool flexible, int64_t* bytes);
// Device half: allocations from `arena` (nullptr: hipMalloc), including the
// solve workspace of (F)GMRES(restart); synchronises `st`.
int setup_device(cptr_solver s, DevArena* arena, int restart, bool flexible, hipStream_t st);
// Frees the device half (back to the arena when there is one); the handle
// returns to its host-only state.
void release_device(cptr_solver s);
// The handle stops reading A's values (call after the last setup_device).
void drop_input(cptr_solver s);
// Device bytes the handle holds now, in DevArena pieces.
int64_t device_bytes(cptr_solver s);
// Message of the last failure on the handle (or of the calling thread's setup).
const char* last_error(cptr_solver s);

}  // namespace cptr
