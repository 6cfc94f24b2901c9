// Entry points of the plan (plan.hip) used by the batch and serving runtime (runtime.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/pkm.h"

namespace pkm_internal {

// Host tables of a multipole request and buffers for up to max_particles objects.
pkm_status prepare(pkm_plan* pl, int ell_max, const double* k_edges, int n_edges, int64_t max_particles);
// Doubles of a result slot of the prepared request (catalog sums + bin sums).
size_t slot_doubles(const pkm_plan* pl);
bool prepared(const pkm_plan* pl);
hipStream_t stream_of(const pkm_plan* pl);
int device_of(const pkm_plan* pl);
int64_t device_bytes(const pkm_plan* pl);
// Changes whenever the plan's device buffers or request tables change.
uint64_t generation(const pkm_plan* pl);
std::string& error_of(pkm_plan* pl);
// One whole estimate of device catalogs, results to a pinned host slot; no allocation, no
// host wait (capturable).
// `timed`: record the plan's per-launch timing events when stage timing is on (never inside
// a graph capture).
pkm_status enqueue(pkm_plan* pl, const pkm_catalog* data, const pkm_catalog* randoms, double* slot, bool timed);
// Multipoles only, of the painted field the plan holds from its last estimate (the same
// catalog, mesh and precision), for the prepared request; the slot gets that estimate's
// catalog sums again.  No allocation, no host wait.
pkm_status enqueue_compute_only(pkm_plan* pl, double* slot);
// Normalise a completed slot into `out` (the prepared ell_max and edges).  PKM_EINVAL
// (reason in *why, `out` untouched) when the normalisation I is not positive.
pkm_status finish(pkm_plan* pl, const double* slot, int64_t nd, int64_t nr, pkm_result* out, std::string* why);
// Device bytes a plan with these parameters would hold for one request (admission control).
int64_t footprint(const pkm_params* p, int ell_max, int n_edges, int64_t n_particles);

}  // namespace pkm_internal
