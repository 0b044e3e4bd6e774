"""Key-value workload pieces that run on the CPU: the native load generator
against the oracle's CPU UDP server, and the heap padding."""
import socket
import struct
import threading

import numpy as np

import oracle
import synth
from paper_1705_06965_amd.kv import loadgen, make_requests, padded_heap


def test_padded_heap_moves_every_value():
    kv = synth.kv_set(n_keys=500, n_req=10)
    poff, ph = padded_heap(kv.val_off, kv.val_len, kv.heap)
    assert (poff % 16 == 0).all()
    for i in range(0, 500, 7):
        a, ln = int(kv.val_off[i]), int(kv.val_len[i])
        assert ph[int(poff[i]):int(poff[i]) + ln].tobytes() == kv.heap[a:a + ln].tobytes()


def test_loadgen_against_oracle_server():
    kv = synth.kv_set(n_keys=3000, n_req=6000, miss_every=32)
    ix = oracle.KVIndex(kv.keys, kv.val_off, kv.val_len, kv.heap)
    srv = socket.socket(socket.AF_INET, socket.SOCK_DGRAM)
    srv.setsockopt(socket.SOL_SOCKET, socket.SO_RCVBUF, 8 << 20)
    srv.bind(("127.0.0.1", 0))
    # blocking socket with a kernel receive timeout: the C server returns
    # after 0.3 s without traffic
    srv.setsockopt(socket.SOL_SOCKET, socket.SO_RCVTIMEO, struct.pack("ll", 0, 300000))
    port = srv.getsockname()[1]
    served = []
    th = threading.Thread(target=lambda: served.append(ix.serve(srv.fileno(), 1 << 40)))
    th.start()
    reqs = make_requests(kv.req_keys)
    # two malformed requests: wrong op, short datagram handled as status 2
    reqs[5, 8] = 7
    got, replies, rlen, lat, rt = loadgen(port, reqs, threads=3, window=32)
    th.join()
    assert got == len(reqs)
    for k in range(len(reqs)):
        want = ix.reply(reqs[k].tobytes())
        assert rlen[k] == len(want)
        assert replies[k, :rlen[k]].tobytes() == want
    assert served[0] >= len(reqs)
    assert (lat > 0).all()
    ix.close()
    srv.close()
