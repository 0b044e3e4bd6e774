"""GPU parity of the FNV-1a-64 chain itself, over items of every length.

The kernel-split entry point (gsys_fnv4k_consume) hashes bytes that are
already in memory, with a length chosen per item, so a wavefront can be
given any mix of lengths: every residue of the 16-byte loads and of the
256- and 128-byte tile steps, empty and single-byte items, error returns,
items longer than a tile step, and ragged last wavefronts, in work-groups
of 64 to 1024 (256- and 128-byte steps) with bytes in device or host
memory.  Every result must equal the oracle's FNV-1a-64 bit for bit, and
items with a length <= 0 hash nothing."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_06965_amd as g
    ctx = g.Context(ring_slots=1 << 10, device_timeout_ns=60_000_000_000)
    yield g, ctx
    assert ctx.shutdown() == 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lengths(item_bytes, seed):
    """Per-wavefront length patterns (64 items each), then a ragged tail."""
    rng = np.random.default_rng([170506965, 90, item_bytes, seed])
    cap = min(item_bytes, 4096)
    w = []
    w.append(np.full(64, cap))                                   # uniform, full
    w.append(np.arange(64))                                      # 0..63: every residue
    w.append(cap - np.arange(64))                                # cap..cap-63
    w.append(np.zeros(64))                                       # nothing to hash
    one = np.zeros(64)
    one[37] = 1
    w.append(one)                                                # one lane, one byte
    w.append(rng.integers(0, cap + 1, 64))                       # random up to the cap
    w.append(np.where(rng.random(64) < 0.3, -rng.integers(1, 30, 64),
                      rng.integers(1, cap + 1, 64)))             # some errors (ret < 0)
    w.append(16 * rng.integers(0, cap // 16 + 1, 64))            # multiples of 16
    w.append(rng.integers(cap - 300, cap + 1, 64))               # near the cap
    w.append(rng.integers(0, item_bytes + 1, 64))                # up to the item size
    if item_bytes > 4096:
        w.append(np.full(64, item_bytes))                        # longer than 4 KiB
        mix = rng.integers(0, 4097, 64)
        mix[5] = 4097                                            # one long item
        w.append(mix)
    tail = rng.integers(0, item_bytes + 1, 29)                   # ragged last wavefront
    return np.concatenate(w + [tail]).astype(np.int64)


def run_case(g, ctx, item_bytes, wg, grid=0, host=False, seed=0):
    import torch
    from paper_1705_06965_amd.fnv import consume
    lens = lengths(item_bytes, seed)
    n = len(lens)
    rng = np.random.default_rng([170506965, 91, item_bytes, seed])
    data = rng.integers(0, 256, n * item_bytes, dtype=np.uint8)
    if host:
        buf = ctx.host_alloc(n * item_bytes)
        buf.array[:n * item_bytes] = data
        staging, keep = buf.dev, buf
    else:
        keep = torch.from_numpy(data).cuda()
        staging = keep.data_ptr()
    rets = torch.from_numpy(lens).cuda()
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    say("fnv chain item_bytes", item_bytes, "wg", wg, "grid", grid, "host", host, "n", n)
    consume(ctx, staging, rets, item_bytes, out, wg_size=wg, grid=grid)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint64)
    want = np.array([oracle.fnv1a64(data[i * item_bytes:i * item_bytes + max(0, min(int(lens[i]),
                                                                                 item_bytes))])
                     for i in range(n)], dtype=np.uint64)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "items %s (lengths %s) differ" % (bad[:8].tolist(),
                                                            lens[bad[:8]].tolist())
    del keep


@pytest.mark.parametrize("item_bytes,wg", [(4096, 256), (4096, 64), (4096, 128), (8192, 256),
                                           (64, 256), (4096, 1024), (8192, 512)])
def test_chain_matches_oracle(gs, item_bytes, wg):
    g, ctx = gs
    run_case(g, ctx, item_bytes, wg)


def test_chain_grid_stride_and_host_staging(gs):
    """Fewer work-groups than batches (grid-stride loop), bytes in host memory."""
    g, ctx = gs
    run_case(g, ctx, 4096, 256, grid=2, host=True, seed=1)
    run_case(g, ctx, 4096, 64, grid=3, seed=2)
