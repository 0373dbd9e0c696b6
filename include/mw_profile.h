/*
 * mw_profile.h -- opt-in per-kernel timing of libmw (instrumentation, not a
 * transform).  While enabled, every kernel launch of mw_forward / mw_inverse
 * and the adjoints is bracketed by two hipEventRecord calls on the caller's
 * stream; mw_profile_read() waits for the recorded events and returns the
 * summed duration and launch count of each stage.  Disabled by default; when
 * disabled no event is recorded.
 *
 * Stage ids (index into the output arrays):
 *   0 phi stage, forward        3 contraction, inverse
 *   1 theta stage, forward      4 theta stage, inverse
 *   2 contraction, forward      5 phi stage, inverse
 *   6 contraction, forward adjoint   7 contraction, inverse adjoint
 *   8 other: the inverse's coefficient staging kernel, adjoint Fourier stages,
 *     batched helpers
 */
#ifndef MW_PROFILE_H
#define MW_PROFILE_H

#ifdef __cplusplus
extern "C" {
#endif

#define MW_PROFILE_NSTAGE 9

/* Enable (on != 0) or disable recording; enabling clears previous records. */
int mw_profile_enable(int on);

/* Synchronise the recorded events and write, per stage, the summed kernel time
 * in milliseconds (ms[MW_PROFILE_NSTAGE]) and the number of launches
 * (count[MW_PROFILE_NSTAGE]); clears the records.  Returns an mw_status. */
int mw_profile_read(double* ms, int* count);

/* Name of a stage id ("" if out of range). */
const char* mw_profile_stage_name(int stage);

/* Group size (maps sharing one set of Wigner recursions) that mw_prepare's
 * autotuner chose for the groups that start at band-limit L in mixed-precision
 * calls with `nmaps` maps of band-limit <= L and the given reality; *G = 0 when
 * that shape was not tuned (calls then use the largest size the LDS allows, up
 * to that map count). */
int mw_profile_tuned_group(int L, int reality, int nmaps, int* G);

/* The autotuner's cache: with the environment variable MW_TUNE_CACHE naming a
 * file, mw_prepare reads its entries before tuning and appends what it tunes,
 * one line "gfx950 L reality nmaps G" per shape; lines that do not parse, or
 * name another architecture or an impossible value, are skipped (the shape is
 * then tuned again).  This loads such a file now (host only, no GPU needed)
 * and reports in *entries how many lines it took. */
int mw_profile_tune_cache_load(const char* path, int* entries);

/* Fourier-kernel layout of plans built from now on (a test hook): mode 0 (the
 * default) runs the N2-point transforms in LDS up to N2 = 8192 and splits them
 * into half-length pairs above (band-limits L > 2048); mode 1 splits them for
 * every plan with N2 >= 2048 (L >= 257), so that the split kernels can be
 * compared with the oracle at band-limits it evaluates quickly.  Plans already
 * built keep their layout (plans are cached per band-limit until mw_release).
 * Results agree with the unsplit kernels to rounding. */
int mw_profile_split_fft(int mode);

/* FP64 inverse contraction kernel (a test hook): mode 0 (the default) runs real
 * maps at every band-limit, and complex maps from L = 1024, on the kernel that
 * evaluates each Wigner chain Delta^l_{n,m} with n >= m once for the pairs
 * (m, n) and (n, m) (the symmetry of Sec. III-C), and smaller complex maps on
 * the kernel that runs every (n, m) chain; mode 1 runs every map on the first
 * one, so that it can be compared with the oracle at small band-limits.  Takes
 * effect for the calls that follow; results agree with the default to rounding. */
int mw_profile_inverse_triangle(int mode);

#ifdef __cplusplus
}
#endif

#endif /* MW_PROFILE_H */
