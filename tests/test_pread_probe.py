"""Host read capacity probe (gsys_host_pread_rate) on the CPU: the bytes it
copies are the file's, ranges land in slot i mod n_slots, bad arguments and
failing preads are reported."""
import ctypes as C
import errno
import os

import numpy as np
import pytest

import paper_1705_06965_amd as g

MIB = 1 << 20


@pytest.fixture(scope="module")
def datafile(tmpdata):
    p = os.path.join(tmpdata, "probe.bin")
    data = np.random.default_rng([170506965, 9]).bytes(6 * MIB + 1234)
    with open(p, "wb") as f:
        f.write(data)
    fd = os.open(p, os.O_RDONLY)
    yield fd, data
    os.close(fd)


def probe(fds, offs, lens, buf, slot, n_slots, threads=3, reps=2):
    fds = np.ascontiguousarray(fds, dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.uint64)
    lens = np.ascontiguousarray(lens, dtype=np.uint32)
    out = C.c_double(-1.0)
    rc = g.lib.gsys_host_pread_rate(fds.ctypes.data, offs.ctypes.data, lens.ctypes.data,
                                    len(lens), buf.ctypes.data, slot, n_slots, threads, reps,
                                    C.byref(out))
    return rc, out.value


def test_every_range_lands_in_its_slot(datafile):
    fd, data = datafile
    offs = [0, MIB, 2 * MIB + 7, 5 * MIB, 6 * MIB]   # the last one reaches EOF (short)
    lens = [MIB, 4096, 65, MIB, MIB]
    slot = MIB + 64
    buf = np.zeros(slot * len(lens), dtype=np.uint8)
    rc, gbps = probe([fd] * len(lens), offs, lens, buf, slot, len(lens))
    assert rc == 0 and gbps > 0
    for i, (o, n) in enumerate(zip(offs, lens)):
        want = data[o:o + n]
        assert bytes(buf[i * slot:i * slot + len(want)]) == want, i


def test_slots_wrap(datafile):
    fd, data = datafile
    offs = [k * 4096 for k in range(10)]
    slot = 4096
    buf = np.zeros(slot * 3, dtype=np.uint8)
    rc, _ = probe([fd] * 10, offs, [4096] * 10, buf, slot, 3)
    assert rc == 0
    for s in range(3):
        got = bytes(buf[s * slot:(s + 1) * slot])
        assert got in [data[o:o + 4096] for i, o in enumerate(offs) if i % 3 == s], s


def test_refusals(datafile):
    fd, _ = datafile
    buf = np.zeros(8192, dtype=np.uint8)
    assert probe([fd], [0], [8193], buf, 8192, 1)[0] == -errno.EINVAL   # longer than a slot
    assert probe([fd], [0], [4096], buf, 8192, 1, threads=0)[0] == -errno.EINVAL
    assert probe([fd], [0], [4096], buf, 8192, 0)[0] == -errno.EINVAL
    assert probe([fd], [0], [4096], buf, 8192, 1, reps=0)[0] == -errno.EINVAL
    assert probe([-1], [0], [4096], buf, 8192, 1)[0] == -errno.EBADF


def test_runs_of_ranges(datafile):
    """Many short ranges (claimed 256 at a time) all land in their slots."""
    fd, data = datafile
    n = 4096
    offs = (np.arange(n, dtype=np.uint64) * np.uint64(1531)) % np.uint64(6 * MIB)
    lens = (np.arange(n, dtype=np.uint32) % 61) + 1
    slot = 64
    buf = np.zeros(slot * n, dtype=np.uint8)
    rc, gbps = probe([fd] * n, offs, lens, buf, slot, n, threads=2)
    assert rc == 0 and gbps > 0
    for i in range(n):
        o, k = int(offs[i]), int(lens[i])
        assert bytes(buf[i * slot:i * slot + k]) == data[o:o + k], i


def test_out_of_descriptors_falls_back_to_the_callers(datafile, tmp_path):
    """With too few descriptors for a private copy of every file in every
    thread (a low RLIMIT_NOFILE, in a child process), the probe reads through
    the caller's descriptors instead, as the pool's pollers do, and the bytes
    are still the file's."""
    import subprocess
    import sys
    fd, data = datafile
    path = os.readlink("/proc/self/fd/%d" % fd)
    code = """
import ctypes as C, os, resource, sys
import numpy as np
sys.path.insert(0, %r)
import paper_1705_06965_amd as g
fds = [os.open(%r, os.O_RDONLY) for _ in range(24)]
resource.setrlimit(resource.RLIMIT_NOFILE, (max(fds) + 12, resource.getrlimit(resource.RLIMIT_NOFILE)[1]))
n = 96
f = np.array([fds[i %% 24] for i in range(n)], dtype=np.int32)
o = (np.arange(n, dtype=np.uint64) * 4096)
l = np.full(n, 4096, dtype=np.uint32)
buf = np.zeros(n * 4096, dtype=np.uint8)
out = C.c_double()
rc = g.lib.gsys_host_pread_rate(f.ctypes.data, o.ctypes.data, l.ctypes.data, n, buf.ctypes.data,
                                4096, n, 8, 1, C.byref(out))
want = open(%r, "rb").read(n * 4096)
print(rc, bytes(buf) == want)
""" % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))), path, path)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split()[-2:] == ["0", "True"], r.stdout
