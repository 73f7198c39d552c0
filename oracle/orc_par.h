/*
 * Oracle: parallel cell loops.  TEST INFRASTRUCTURE ONLY.
 *
 * ORC_PARFOR marks a loop over cells or vector entries whose iterations
 * write disjoint outputs and read nothing another iteration writes, so
 * running it on several threads gives exactly the serial result.  Sums
 * (norms, dot products, diagnostics) and the scatter-form transposes are
 * never marked.  The thread count is orc_set_threads' (default 1).
 */
#ifndef ORC_PAR_H
#define ORC_PAR_H
extern int orc_threads;
#define ORC_PARFOR _Pragma("omp parallel for schedule(static) if(orc_threads > 1) num_threads(orc_threads)")
#endif
