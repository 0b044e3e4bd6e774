"""Host-side pieces of the word-search driver (no GPU)."""
import numpy as np

from paper_1705_06965_amd.wordscan import chunk_table, staging_bytes


def test_chunk_table_covers_files_exactly():
    sizes = [0, 1, 4096, 4097, 10_000_000, 3]
    t = chunk_table([3, 4, 5, 6, 7, 8], sizes, 1 << 20)
    for f, size in enumerate(sizes):
        rows = t[t["file"] == f]
        assert int(rows["len"].sum()) == size
        if size:
            assert rows["off"][0] == 0
            assert (rows["off"][1:] == rows["off"][:-1] + rows["len"][:-1]).all()
            assert (rows["len"] <= 1 << 20).all() and (rows["len"] > 0).all()
        else:
            assert len(rows) == 0
    assert (t["fd"][t["file"] == 4] == 7).all()


def test_staging_bytes_rounds_to_16():
    assert staging_bytes(13, 1) == 80
    assert staging_bytes(1 << 20, 2) == 2 * ((1 << 20) + 64)


def test_empty_chunk_table_is_a_valid_call():
    """A corpus of empty files has no chunks: gsys_wordscan takes a null
    chunk table with n_chunks == 0 in every form (it only zeroes the counts,
    which needs the device: -ENODEV on a CPU-only context), and refuses a
    null table that claims chunks."""
    import errno

    import paper_1705_06965_amd as g
    c = g.Context(flags=g.CFG_NO_DEVICE | g.CFG_NO_PIN, service_threads=1)
    try:
        st = c.host_alloc(staging_bytes(4096, 2))

        def call(chunks, n_chunks, form, passes=1):
            return g.lib.gsys_wordscan(c.h, chunks, n_chunks, 4096, 0x1000, 0x2000, 1, 0x3000, 3,
                                       st.dev, st.nbytes, form, passes, None)
        for form in (g.PLAIN, g.PERSISTENT, g.GRAPH):
            assert call(0, 0, form) == -errno.ENODEV
            assert call(0, 1, form) == -errno.EINVAL
        assert call(0, 0, g.PERSISTENT, passes=3) == -errno.ENODEV
        st.free()
    finally:
        c.shutdown()
