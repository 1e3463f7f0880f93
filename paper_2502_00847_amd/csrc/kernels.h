// Kernel entry points and their host-side launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "jobs.h"
#include "modarith.h"

namespace secpe {

// Launchers: 'jobs' points to device memory holding n_jobs descriptors.
// max_limbs bounds the limb count of any job in the launch (grid y).
// The NTT runs as ntt_pass_count() launches (1 for N <= 2^12, else 2).
int ntt_pass_count(const DevTables& T);
// tiles_sched: passes run with two tiles per workgroup (where a variant
// exists, N = 2^16): bit 0 forward column pass, bit 1 inverse column pass,
// bit 2 forward row pass.
void launch_ntt_pass(const DevTables& T, bool inverse, const NttJob* jobs, int n_jobs, int max_limbs, int pass,
                     hipStream_t s, int tiles_sched = 0);
void launch_ntt(const DevTables& T, bool inverse, const NttJob* jobs, int n_jobs, int max_limbs, hipStream_t s,
                int tiles_sched = 0);
// For N > 2^12 the key-switch inner product runs fused with the row pass of
// the ModUp outputs' forward NTT (whose column pass ran as an ordinary launch).
bool inner_row_fused(const DevTables& T);
void launch_inner_row(const DevTables& T, const InnerJob* jobs, int n_jobs, int max_ext, hipStream_t s);
// ... and ModUp runs fused with the column pass of that forward NTT; its
// source is the digit-scaled inverse transform (NttJob::ek on the inverse).
// eg: output limbs per workgroup (2 or 4; a tunable)
void launch_modup_col(const DevTables& T, const ModUpJob* jobs, int n_jobs, int max_ext, int eg, hipStream_t s);
// The ModDown's centred conversion fused with the column pass of its outputs'
// forward NTT (source prescaled by the inverse transform: ModDownJob::cinv
// null); the row pass, with the combine as its epilogue, follows as a launch.
// eg: output limbs per workgroup (2 or 4; a tunable)
void launch_moddown_col(const DevTables& T, const ModDownJob* jobs, int n_jobs, int max_chain, int eg,
                        hipStream_t s);
void launch_ew(const DevTables& T, const EwJob* jobs, int n_jobs, int max_limbs, hipStream_t s);
void launch_modup(const DevTables& T, const ModUpJob* jobs, int n_jobs, hipStream_t s);
void launch_moddown_conv(const DevTables& T, const ModDownJob* jobs, int n_jobs, hipStream_t s);
void launch_inner(const DevTables& T, const InnerJob* jobs, int n_jobs, int max_ext, hipStream_t s);
void launch_automorph(const DevTables& T, const AutoJob* jobs, int n_jobs, int max_limbs, hipStream_t s);
void launch_lift(const DevTables& T, const LiftJob* jobs, int n_jobs, const double* ctab, double q0inv_q1, hipStream_t s);
void launch_raise(const DevTables& T, const RaiseJob* jobs, int n_jobs, hipStream_t s);
void launch_bsgs(const DevTables& T, const BsgsJob* jobs, int n_jobs, int max_limbs, hipStream_t s);
void launch_sample(const DevTables& T, const SampleJob* jobs, int n_jobs, int max_limbs, hipStream_t s);
void launch_int_spread(const DevTables& T, const IntSpreadJob* jobs, int n_jobs, int max_limbs, hipStream_t s);
void launch_encode(const DevTables& T, const EncodeJob* jobs, int n_jobs, hipStream_t s);
// phase: -2 zero, -1 scatter, 0 .. log2(2N)-1 FFT stages, 1000 round (FftEncJob)
void launch_fft_enc(const DevTables& T, const FftEncJob* jobs, int n_jobs, int phase, hipStream_t s);
void launch_decode(const DevTables& T, const int64_t* m, double* z, int nslots, double inv_scale, hipStream_t s);

}  // namespace secpe
