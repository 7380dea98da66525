/* internal.h -- helpers shared between the oracle's own translation units.
 * Test infrastructure only (see omc_oracle.h). */
#ifndef OMC_ORACLE_INTERNAL_H
#define OMC_ORACLE_INTERNAL_H
/* Energy-grid position: t = (log2 E - log2 ELO) * (NE-1)/log2(EHI/ELO), clamped
 * to [0, NE-1]; i = min(floor t, NE-2); f = t - i. */
void orc__grid_pos(double E, int* i, double* f);
#endif
