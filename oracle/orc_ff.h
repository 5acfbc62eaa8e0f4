/*
 * orc_ff.h -- Flip-Flop insertion (Section 4.3, Line 8) inside the oracle's
 * round.  TEST INFRASTRUCTURE ONLY (see orc.h); internal to the oracle.
 */
#ifndef ORC_FF_H
#define ORC_FF_H
#include "orc.h"

/* Lines 6 and 8 of a round by Flip-Flop insertion, after the walk of Line 6.
   tloc/tpx/tpy/tkey: per triangle slot, the located triangle (-1 none), the
   circumcenter and its key; mflag: per subsegment, flagged for its midpoint
   (raised further here); sadj: per subsegment, 3*t+edge of its triangles.
   Rewrites the mesh (canonical triangle order), the vertex, subsegment and
   pending arrays, and fills the Line 6/8 fields of st.  0 or an ORC_E_ code. */
int orc_ff_round(orc_mesh *m, const orc_params *prm, const int32_t *tloc, const double *tpx, const double *tpy,
                 const uint64_t *tkey, uint8_t *mflag, const int32_t *sadj, orc_round_stats *st,
                 char *err, int32_t errlen);

/* Replaces the triangles by the canonical CDT of the current vertices and
   subsegments (the state the Flip-Flop rounds keep). */
int orc_ff_canonical(orc_mesh *m, char *err, int32_t errlen);

/* The points S (after Line 6, in key order) of the last Flip-Flop round run
   in this process: coordinates, class (1 midpoint), subsegment or bad
   triangle, claimed triangles (slots before the round), edge of c0 a
   circumcenter lies on (-1 inside), key.  Copies up to cap; returns the
   count.  For tests only. */
int64_t orc_ff_last_points(int64_t cap, double *xy, int32_t *cls, int32_t *id, int32_t *c0, int32_t *c1,
                           int32_t *edge, uint64_t *key);
/* ... and the subsegments flagged for their midpoint when its Line 8 began. */
int64_t orc_ff_last_flagged(int64_t cap, int32_t *ks);
#endif
