/*
 * Test hooks of the gsys library: libgsys_testing.so, a library only tests
 * load, linked against libgsys.so (not part of the product ABI).  They let
 * CPU-only tests drive the host service pool through exactly the protocol
 * the GPU uses, without a GPU, and inject faults.
 */
#ifndef GSYS_TESTING_H
#define GSYS_TESTING_H

#include <stdint.h>

#include "gsys.h"

#ifdef __cplusplus
extern "C" {
#endif

/* gsys_test_emulate mode bits */
#define GSYS_EMU_BLOCKING 0x1u  /* blocking calls (the waiter frees the slots)           */
#define GSYS_EMU_LIST     0x2u  /* each group is one descriptor-list request (a group call) */

/*
 * Emulate `threads` GPU wavefronts on host threads, in a context created with
 * GSYS_CFG_NO_DEVICE (else -EINVAL).  Thread w makes `calls_per_thread`
 * pread calls, call k = w * calls_per_thread + i reading `len` bytes at
 * offs[k] into buf_dev + k * len.  Calls go out in groups of `group`
 * (1..64): one fetch-add claims the group's tickets (as a wavefront's ballot
 * does), each call fills its slot, and the group waits on its completion
 * record (section 5's slot protocol).  With GSYS_EMU_LIST a group is one
 * list request carrying `group` descriptors (a work-group call); the list
 * lives at list_dev + 16 * first call of the group.  rets[k] receives each
 * call's return value.  Returns 0, or -ETIMEDOUT if a wait exceeded
 * timeout_ns.
 */
int gsys_test_emulate(gsys_ctx *ctx, uint32_t threads, uint64_t calls_per_thread, uint32_t group,
                      uint32_t mode, int fd, uint64_t buf_dev, uint64_t list_dev, uint32_t len,
                      const uint64_t *offs, int64_t *rets, uint64_t timeout_ns);

/*
 * Publish one raw request (any nr, flags and args) as a single-ticket group
 * and wait for it, in a GSYS_CFG_NO_DEVICE context.  Used to test the
 * whitelist.  *ret receives the result.  Returns 0 or -ETIMEDOUT.
 */
int gsys_test_raw_call(gsys_ctx *ctx, uint16_t nr, uint8_t flags, const uint64_t *args6,
                       int64_t *ret, uint64_t timeout_ns);

/*
 * Claim `n` tickets and publish none of them (a caller that died between
 * claim and publish), in a GSYS_CFG_NO_DEVICE context.  Returns the first
 * ticket.  Used to test shutdown with requests outstanding.
 */
int64_t gsys_test_claim_only(gsys_ctx *ctx, uint32_t n);

/*
 * Drop a registration without gsys_unregister_buffer's outstanding-ticket
 * rule (any context): only the service threads' grace period protects it,
 * so the call returns once no service thread can still use the buffer.
 * Used to test that period with calls in flight.  Errors: -ENOENT.
 */
int gsys_test_unregister_now(gsys_ctx *ctx, uint32_t id);

/* Read-only view of the ring for quiescence checks: copies D control words. */
int gsys_test_ring_ctl(gsys_ctx *ctx, uint64_t *out, uint64_t max);

/*
 * Fault injection: the next `count` requests with call number `nr`, single
 * or descriptor-list, are answered with -err instead of being executed (a
 * list's descriptors are left as the caller wrote them) in any context,
 * device or CPU-only.  count 0 clears it.  Used to check that a caller sees
 * exactly the -errno the host produced, and what it does when a whole call
 * fails.  Returns 0 or -EINVAL.
 */
int gsys_test_inject(gsys_ctx *ctx, uint16_t nr, int32_t err, uint32_t count);

#ifdef __cplusplus
}
#endif

#endif /* GSYS_TESTING_H */
