/* ptg_loadgen.h -- open-loop load generation over the tile server and the plain per-tile
 * path (benchmark support, built as libptg_loadgen.so on top of libptg.so).
 *
 * A stream of n requests with arrival offsets arrival_ns[i] (ns from the start, non-
 * decreasing) is issued at those times by a native thread.  Outputs: done_ns[i], the time
 * (ns from the start) at which the host saw request i complete.  Latency = done - arrival.
 */
#ifndef PTG_LOADGEN_H
#define PTG_LOADGEN_H

#include "ptg.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PTG_LG_DIRECT 0 /* one ptg_fbm_* launch per request as it arrives                  */
#define PTG_LG_GRAPH 1  /* every request that has arrived (up to max_batch) recorded into a */
                        /* ptg_batch and launched as one HIP graph (instantiated once per   */
                        /* batch shape, arguments updated for later batches of that shape); */
                        /* its requests complete together.  Switched off (PTG_EINVAL): a     */
                        /* stream of one-request graphs updated in place ended the process   */
                        /* with a segmentation fault of unknown cause                        */
#define PTG_LG_SOLO 2   /* each request launched alone, one after the other (arrivals        */
                        /* ignored): done_ns[i] receives request i's kernel time (ns)        */
                        /* between two events on the stream; their sum bounds what any       */
                        /* batching of the same requests can save                            */

/* Through server s: requests are submitted at their arrival times (all that have arrived
 * in one ptg_tiles_submit call); completions are taken and released at once, in request
 * order (any_order = 0: when a request waits for bytes held by later requests that
 * completed first, those are taken and released first) or in completion order
 * (any_order = 1, ptg_tiles_wait_any; the server must serve no other client during the
 * call).  done_ns is the server's completion time (t_done_ns); admit_ns (optional) its
 * admission time.  Returns PTG_OK or the first error of the server calls. */
PTG_API int ptg_lg_served(ptg_server *s, const ptg_tile_req *reqs, const int64_t *arrival_ns, int32_t n,
                          int64_t *done_ns, int64_t *admit_ns, int32_t any_order);

/* Through the plain path on a stream of its own: request i writes its dense output into
 * arena (device memory, arena_bytes) at an offset that wraps around in arrival order; the
 * single stream orders the reuse.  stats (optional, 3 entries) receives the number of launch
 * units (requests, or graph launches), and in graph mode the graphs instantiated and the
 * launches that reused an instance with updated arguments.  Returns PTG_OK, PTG_EINVAL,
 * PTG_E2BIG (a request larger than the arena) or PTG_EHIP. */
PTG_API int ptg_lg_plain(const ptg_tile_req *reqs, const int64_t *arrival_ns, int32_t n, void *arena,
                         int64_t arena_bytes, int32_t mode, int32_t max_batch, int64_t *done_ns, int64_t *stats);

#ifdef __cplusplus
}
#endif

#endif
