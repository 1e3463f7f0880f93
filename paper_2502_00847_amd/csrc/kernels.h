// Kernel entry points and their host-side launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "jobs.h"
#include "modarith.h"

namespace secpe {

// Launchers: 'jobs' points to device memory holding n_jobs descriptors.
// max_limbs bounds the limb count of any job in the launch (grid y).
// prof_pass >= 0 brackets that pass (0 = first, 1 = second) with events e0/e1
void launch_ntt(const DevTables& T, bool inverse, const NttJob* jobs, int n_jobs, int max_limbs, hipStream_t s,
                int prof_pass = -1, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_ew(const DevTables& T, const EwJob* jobs, int n_jobs, int max_limbs, hipStream_t s);
void launch_modup(const DevTables& T, const ModUpJob* jobs, int n_jobs, hipStream_t s);
void launch_moddown_conv(const DevTables& T, const ModDownJob* jobs, int n_jobs, hipStream_t s);
void launch_inner(const DevTables& T, const InnerJob* jobs, int n_jobs, int max_ext, hipStream_t s);
void launch_spread_centred(const DevTables& T, const SpreadJob* jobs, int n_jobs, int max_chain, hipStream_t s);
void launch_automorph(const DevTables& T, const AutoJob* jobs, int n_jobs, int max_limbs, hipStream_t s);
void launch_lift(const DevTables& T, const LiftJob* jobs, int n_jobs, const double* ctab, double q0inv_q1, hipStream_t s);
void launch_sample(const DevTables& T, const SampleJob* jobs, int n_jobs, int max_limbs, hipStream_t s);
void launch_int_spread(const DevTables& T, const IntSpreadJob* jobs, int n_jobs, int max_limbs, hipStream_t s);
void launch_encode(const DevTables& T, const EncodeJob* jobs, int n_jobs, hipStream_t s);
void launch_decode(const DevTables& T, const int64_t* m, double* z, int nslots, double inv_scale, hipStream_t s);

}  // namespace secpe
