/*
 * GRAPE-6-style interface of the direct N-body library (Appendix A).
 *
 * The paper's library keeps the call sequence of the GRAPE-6 library, so an
 * integrator written for GRAPE-6 (the paper's kira runs, Section 4) needs only
 * to be relinked: the host opens the device, hands over j-particles one by one
 * with their predictor data, sets the time to which all j are predicted, then
 * for each group of i-particles starts the force calculation and later
 * collects acceleration, jerk, potential and the nearest neighbour.  Calls
 * with no GPU work in the original are accepted and do nothing.
 *
 * The entry points below carry the names Appendix A lists.  Their argument
 * lists follow the roles of the GRAPE-6 calls but are this library's own (the
 * paper does not print them), so this is a source-level, not binary,
 * counterpart.  Semantics that differ from the paper's library:
 *  - prediction of the j-particles to the requested time runs on the GPU in
 *    float64 (the paper predicted on the host), with the library's Hermite
 *    predictor x + v D + a D^2/2 + j D^3/6, v + a D + j D^2/2, D = t_i - t_j;
 *  - an i-particle whose `index` names a j-particle set at an address below
 *    nj is evaluated at that j-particle's predicted position and velocity, and
 *    that j-particle is excluded from its sums (the interaction with itself);
 *    other i-particles use the given xi, vi and exclude nothing;
 *  - G = 1 (the GRAPE convention); softening enters as eps^2.
 *
 * Every function returns 0 on success or a negative NBODY_ERR_* code (see
 * nbody.h); the detail of the last failure on a cluster is in
 * GPU_last_error.  Host arrays are plain C arrays owned by the caller.  A
 * cluster is not thread-safe.
 */
#ifndef NBODY_GRAPE_H
#define NBODY_GRAPE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Largest cluster id + 1. */
#define NBODY_GRAPE_MAX_CLUSTERS 16

/* Open cluster `clusterid` on HIP device `clusterid` (GPU_open: connect and
 * set up buffers).  Opening an open cluster is a no-op.  NBODY_ERR_ARG for an
 * id outside [0, NBODY_GRAPE_MAX_CLUSTERS); device errors as nbody_create. */
int GPU_open(int clusterid);

/* Release the cluster's device and host memory (GPU_close).  Closing a
 * closed cluster is a no-op. */
int GPU_close(int clusterid);

/* The number of i-particles the host should pass per force call
 * (GPU_npipes).  The GPU has no fixed pipeline count; the value comes from
 * the environment variable NBODY_GRAPE_NPIPES (default 2048), as the paper
 * reads it from a configuration file.  Any ni is accepted by the calls
 * below. */
int GPU_npipes(void);

/* Store j-particle `address` (GPU_set_j_particle): its identity `index`, its
 * time tj, mass, and the position x, velocity v, acceleration a and jerk j at
 * tj (3 doubles each).  The data are buffered on the host and sent to the GPU
 * by the next GPU_set_ti.  Addresses may be set in any order; the j set is
 * addresses 0 .. (highest address set) and unset addresses are massless.
 * NBODY_ERR_ARG for a closed cluster, address < 0 or above 2^31 - 2, NULL
 * vectors, or non-finite data. */
int GPU_set_j_particle(int clusterid, int address, int index, double tj, double mass,
                       const double x[3], const double v[3], const double a[3], const double j[3]);

/* Predict every j-particle to time ti on the device (GPU_set_ti), after
 * sending the buffered j data.  Enqueued; returns without waiting. */
int GPU_set_ti(int clusterid, double ti);

/* Start the force calculation (GPUcalc_firsthalf) of ni i-particles against
 * j addresses 0 .. nj-1 with softening eps2 = eps^2: i-particle k has the
 * identity index[k] and position xi[k], velocity vi[k] (used unless index[k]
 * names a j-particle, see above).  Returns after enqueueing the work; the
 * host arrays may be reused at once.  NBODY_ERR_STATE if GPU_set_ti has not
 * been called since the last GPU_set_j_particle, or a calculation is still
 * pending; NBODY_ERR_ARG for nj outside [0, j set size], ni < 0, NULL arrays
 * with ni > 0, or eps2 < 0. */
int GPUcalc_firsthalf(int clusterid, int nj, int ni, const int index[], const double xi[][3],
                      const double vi[][3], double eps2);

/* Collect the results of the pending calculation (GPUcalc_lasthalf): waits
 * for it, then writes acc[k], jerk[k] (3 doubles each) and pot[k] (the
 * potential, negative) for k < ni.  ni must equal the pending call's.
 * NBODY_ERR_STATE if nothing is pending. */
int GPUcalc_lasthalf(int clusterid, int ni, double acc[][3], double jerk[][3], double pot[]);

/* GPUcalc_lasthalf plus the nearest neighbour of every i-particle (Section
 * 3.3): nnb[k] is the identity (index) of the j-particle at the smallest
 * unsoftened distance, itself excluded, the lowest address among equally
 * close ones; -1 if none.  The calculation must have been started with the
 * nearest neighbour enabled (GPU_set_nn; on by default). */
int GPUcalc_lasthalf2(int clusterid, int ni, double acc[][3], double jerk[][3], double pot[], int nnb[]);

/* Enable (1, the default) or disable (0) the nearest-neighbour search in the
 * following force calculations; without it the pairwise kernel does about
 * 10% less work (Section 3.3). */
int GPU_set_nn(int clusterid, int enable);

/* Arithmetic of the following force calculations: NBODY_PREC_DS_COMP (1,
 * the default) or NBODY_PREC_FP32 (0). */
int GPU_set_precision(int clusterid, int prec);

/* Detail of the last failure on the cluster ("" if none). */
const char *GPU_last_error(int clusterid);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_GRAPE_H */
