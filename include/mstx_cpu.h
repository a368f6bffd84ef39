/*
 * mstx_cpu.h -- host (CPU) implementations of the four Boruvka variants that
 * Durbhakula, arXiv 2005.06913 evaluates on a multicore CPU, for context
 * beside the GPU library (mstx.h).  Built as libmstx_cpu.so with the host
 * compiler; no HIP.
 *
 *   MSTX_CPU_SEQ_PLAIN   Section 2.1 pseudo code: every round every edge is
 *                        examined (two finds), each component keeps its
 *                        lightest outgoing edge, then every component's edge
 *                        is added and the two components are united (the
 *                        larger, by vertex count, keeps its root).
 *   MSTX_CPU_SEQ_COVERED Section 2.1's optimisation: an edge found internal,
 *                        or added to the tree, is marked covered and never
 *                        examined again.
 *   MSTX_CPU_PAR_LOCK    Section 2.2.1: every thread walks all edges (start
 *                        points spread evenly, wrapping around) and keeps the
 *                        minima of the components it owns; a thread unites
 *                        two components only after taking the permission
 *                        word of both (no spinning: on failure the edge waits
 *                        for the next round).
 *   MSTX_CPU_PAR_CAS     Section 2.2.2: as the lock variant, but the union is
 *                        one compare-and-swap of a root's parent pointer from
 *                        itself to the other root; a failed swap leaves the
 *                        edge for the next round.
 * In both parallel variants the root with the larger id is linked under the
 * smaller one (not component2 under component1 as the text has it): the two
 * finds of a union run at different moments, and with a fixed direction a
 * root could be linked under its own descendant, closing a cycle.
 *
 * Edges are compared by the key (w[e], e), so ties are broken by edge index
 * and the tree is the same unique one the GPU library returns.  Phases of a
 * round (reset minima / scan / unite) are separated by thread barriers.
 *
 * Arguments (all HOST pointers, owned by the caller):
 *   variant   one of the MSTX_CPU_* values;
 *   threads   worker threads for the parallel variants (>= 1; ignored by the
 *             sequential ones);
 *   n, m      vertices and edges (0 <= m <= 0xFFFFFFFF); ids in [0, n);
 *   src, dst, w   the edge list (m entries each);
 *   out_in_mst    m bytes, set to 1 for tree edges and 0 otherwise;
 *   out_total     the tree's total weight;
 *   out_rounds    (may be NULL) the number of rounds run.
 * Returns MSTX_OK (tree), MSTX_DISCONNECTED (forest), MSTX_ERR_INVALID_ARG,
 * MSTX_ERR_TOO_LARGE or MSTX_ERR_VERTEX_RANGE (the status codes of mstx.h);
 * outputs are unspecified on a negative status.
 */
#ifndef MSTX_CPU_H
#define MSTX_CPU_H

#include <stdint.h>

#include "mstx.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MSTX_CPU_SEQ_PLAIN = 0,
  MSTX_CPU_SEQ_COVERED = 1,
  MSTX_CPU_PAR_LOCK = 2,
  MSTX_CPU_PAR_CAS = 3
};

int mst_cpu_solve(int variant, int32_t threads, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                  const uint32_t* w, uint8_t* out_in_mst, uint64_t* out_total, int64_t* out_rounds);

/* Name of a variant ("" if out of range). */
const char* mst_cpu_variant_name(int variant);

#ifdef __cplusplus
}
#endif

#endif /* MSTX_CPU_H */
