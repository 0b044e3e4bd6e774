/*
 * gsys wire format: the memory shared by GPU callers and the host service
 * pool.  Plain C, no functions.  Used by the device library and the host pool.
 *
 * The syscall area of the paper (section 5, Fig. 3) holds one 64-byte slot per
 * active work-item with the call number, the slot state, up to six arguments
 * (also reused for the return value), a blocking bit and padding against false
 * sharing.  Here the slots form a ring of D slots claimed by ticket (ticket t
 * uses slot t mod D) instead of being indexed by a hardware work-item id, so
 * the area is sized by the number of calls in flight, not by the number of
 * work-items the GPU can hold.
 *
 * Slot life cycle (section 5, Fig. 4): FREE -> POPULATING -> READY ->
 * PROCESSING -> FINISHED (blocking; the GPU frees the slot after reading the
 * result) or -> FREE (non-blocking; the host frees it).  The control word
 * carries the ticket next to the state, so a slot of one lap of the ring is
 * never taken for the slot of another lap:
 *     ctl = (ticket << 3) | state
 * A slot is free for ticket t when ctl == GSYS_CTL(t, GSYS_ST_FREE).
 */
#ifndef GSYS_ABI_H
#define GSYS_ABI_H

#include <stdint.h>

#define GSYS_ABI_VERSION 3u

/* ---- slot states (low 3 bits of ctl) ---- */
#define GSYS_ST_FREE        0u
#define GSYS_ST_POPULATING  1u
#define GSYS_ST_READY       2u
#define GSYS_ST_PROCESSING  3u
#define GSYS_ST_FINISHED    4u
#define GSYS_CTL(ticket, st) ((((uint64_t)(ticket)) << 3) | (uint64_t)(st))
#define GSYS_CTL_TICKET(ctl) ((uint64_t)(ctl) >> 3)
#define GSYS_CTL_STATE(ctl)  ((uint32_t)((ctl) & 7u))

/* ---- call numbers: the host's x86_64 system-call numbers ---- */
#define GSYS_NR_READ      0
#define GSYS_NR_WRITE     1
#define GSYS_NR_CLOSE     3
#define GSYS_NR_MMAP      9
#define GSYS_NR_MUNMAP   11
#define GSYS_NR_PREAD64  17
#define GSYS_NR_PWRITE64 18
#define GSYS_NR_MADVISE  28
#define GSYS_NR_SENDTO   44
#define GSYS_NR_RECVFROM 45
#define GSYS_NR_OPENAT  257

/* openat paths: the NUL must lie in the first GSYS_PATH_MAX bytes */
#define GSYS_PATH_MAX   256

/* ---- slot flags ---- */
#define GSYS_F_BLOCKING  0x01u  /* the paper's blocking bit */
#define GSYS_F_LIST      0x02u  /* args describe a descriptor list (group call) */
#define GSYS_F_PRODUCER  0x04u  /* role of the call under relaxed ordering */
#define GSYS_F_STRONG    0x08u  /* strong ordering was requested */
#define GSYS_F_GRAN_SHIFT 4     /* 2 bits: 0 work-item, 1 work-group, 2 kernel */
#define GSYS_F_GRAN_MASK 0x30u
#define GSYS_GRAN_WI     0u
#define GSYS_GRAN_WG     1u
#define GSYS_GRAN_KERNEL 2u

/* One 64-byte slot. */
typedef struct gsys_slot {
    uint64_t ctl;        /* (ticket << 3) | state                                   */
    uint16_t nr;         /* GSYS_NR_*                                               */
    uint8_t  flags;      /* GSYS_F_*                                                */
    uint8_t  grp_n;      /* size of the claim group this ticket belongs to (1..64)  */
    uint32_t grp_off;    /* ticket minus the group's first ticket                  */
    uint64_t args[6];    /* call arguments; args[0] receives the return value      */
} gsys_slot;

/*
 * Completion record, indexed by ticket mod C (C = max(4 D, 65536)).  A
 * blocking call's record cannot be lapped (its slot is freed only after the
 * GPU read the result, and C > D); a non-blocking call's slot is freed by
 * the host, so its record is reused once ticket t + C is claimed, and a
 * device wait that finds it reused reports -EOVERFLOW.  The host writes
 * `ret` of ticket t into comp[t mod C].ret and counts finished members of a
 * claim group with head h in comp[h mod C].stamp = (h << 8) | count.
 * A GPU waiter of group h is done when stamp == (h << 8) | grp_n.
 */
typedef struct gsys_comp {
    int64_t  ret;
    uint64_t stamp;
} gsys_comp;
#define GSYS_STAMP(head, count) ((((uint64_t)(head)) << 8) | (uint64_t)(count))

/*
 * Descriptor of one file transfer inside a list call (pread / pwrite):
 * transfer `len_ret` bytes between file offset `off` and buffer address
 * base + buf_off, where base is args[3] of the slot.  The host replaces
 * len_ret with the call's return value (bytes moved, or -errno), as the
 * slot's args field is reused for the return value.
 * List slot args: [0] fd, [1] list address, [2] count, [3] base address.
 * The list call's own result is the bytes moved by all its descriptors once
 * the host has run the list, whatever their individual results; a negative
 * result means the list never ran (refused as a whole, an injected fault,
 * or a device-side -ETIMEDOUT / -ESHUTDOWN) and every descriptor still holds
 * what the caller wrote.
 */
typedef struct gsys_iodesc {
    uint64_t off;
    uint32_t buf_off;
    int32_t  len_ret;
} gsys_iodesc;

/*
 * Descriptor of one datagram inside a list call (recvfrom / sendto) on an
 * IPv4 UDP socket.  recvfrom fills `addr` with the sender; sendto sends to
 * `addr`.  len_ret as above.  List slot args as for gsys_iodesc, plus
 * [4] per-call flags (MSG_DONTWAIT is always added by the host for recvfrom).
 */
typedef struct gsys_netdesc {
    uint32_t buf_off;
    int32_t  len_ret;
    uint32_t addr_len;
    uint32_t pad;
    uint8_t  addr[16];   /* struct sockaddr_in */
} gsys_netdesc;

/* Device context: what a kernel needs to issue calls. */
typedef struct gsys_dev_ctx {
    gsys_slot *ring;                 /* D slots, host-coherent                   */
    gsys_comp *comp;                 /* C records, host-coherent                 */
    unsigned long long *tail;        /* device memory: next ticket               */
    const uint64_t *retired_lo;      /* host-coherent: every ticket below has retired
                                        (maintained by the host for drain statistics) */
    uint64_t ring_mask;              /* D - 1                                    */
    uint64_t comp_mask;              /* C - 1                                    */
    uint64_t timeout_ticks;          /* device watchdog, 100 MHz ticks (0 = none) */
    uint32_t sleep_max;              /* backoff cap for s_sleep                  */
    uint32_t flags;
    uint64_t arena;                  /* reserved range for GPU mmap (0 = none)   */
    uint64_t arena_bytes;
    uint64_t doorbell;               /* interrupt signal handle (0 = pollers spin) */
    const uint64_t *sleepers;        /* host-coherent: pollers blocked on it      */
    uint64_t ksites;                 /* device: kernel-granularity call sites (16 B each),
                                        cleared by gsys_launch before every launch */
    uint32_t n_ksites;
    uint32_t pad;
} gsys_dev_ctx;

#define GSYS_ETIMEDOUT_RET (-110)    /* -ETIMEDOUT */
#define GSYS_ESHUTDOWN_RET (-108)    /* -ESHUTDOWN */
#define GSYS_EOVERFLOW_RET (-75)     /* -EOVERFLOW: completion record was lapped */
#define GSYS_EINVAL_RET (-22)        /* -EINVAL */
#define GSYS_NOT_WAITED    (-115)    /* -EINPROGRESS: this lane did not wait */

#endif /* GSYS_ABI_H */
