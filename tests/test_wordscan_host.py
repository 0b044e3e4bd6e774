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
