// UDP load generator for the key-value GET server: the CPU load generator of
// the network case study (section 7.3), which sends datagrams to the server
// and receives its answers.  Client threads each own a loopback socket and a
// contiguous slice of the requests, keep up to `window` of them outstanding,
// match replies to requests by id (request k carries id k + 1), and
// retransmit a request whose reply has not come within rto_ns (UDP may drop
// datagrams; a GET is idempotent, so a duplicate reply is identical).
// Requests go out and replies come in up to kBatch datagrams per kernel call
// (sendmmsg / recvmmsg), so that the generator is not what bounds a server.
#include <arpa/inet.h>
#include <errno.h>
#include <netinet/in.h>
#include <poll.h>
#include <string.h>
#include <sys/socket.h>
#include <time.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "gsys.h"

namespace {

constexpr uint32_t kBatch = 64;

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Slice {
  uint64_t lo, hi;
  uint64_t completed = 0, retransmits = 0;
  int err = 0;
};

void client(uint32_t port, const uint8_t* reqs, uint32_t req_len, Slice* sl, uint32_t window,
            uint64_t rto_ns, uint64_t deadline, uint8_t* replies, uint32_t stride,
            uint32_t* reply_len, uint64_t* lat_ns) {
  int fd = socket(AF_INET, SOCK_DGRAM, 0);
  if (fd < 0) {
    sl->err = -errno;
    return;
  }
  int big = 8 << 20;
  setsockopt(fd, SOL_SOCKET, SO_RCVBUF, &big, sizeof big);
  setsockopt(fd, SOL_SOCKET, SO_SNDBUF, &big, sizeof big);
  sockaddr_in me{};
  me.sin_family = AF_INET;
  me.sin_addr.s_addr = htonl(INADDR_LOOPBACK);
  me.sin_port = 0;
  if (bind(fd, (sockaddr*)&me, sizeof me) != 0) {
    sl->err = -errno;
    close(fd);
    return;
  }
  sockaddr_in srv{};
  srv.sin_family = AF_INET;
  srv.sin_addr.s_addr = htonl(INADDR_LOOPBACK);
  srv.sin_port = htons((uint16_t)port);
  const uint64_t n = sl->hi - sl->lo;
  std::vector<uint8_t> state(n, 0);        // 0 unsent, 1 outstanding, 2 done
  std::vector<uint64_t> t_first(n, 0), t_last(n, 0);
  uint64_t next = 0, oldest = 0, outstanding = 0, done = 0;
  const uint32_t rsz = std::max<uint32_t>(stride, 2048);
  std::vector<uint8_t> rbuf((size_t)rsz * kBatch);
  mmsghdr mm[kBatch];
  iovec iov[kBatch];
  while (done < n) {
    const uint64_t t = now_ns();
    if (t > deadline) {
      sl->err = -ETIMEDOUT;
      break;
    }
    // new requests
    while (outstanding < window && next < n) {
      const uint32_t m = (uint32_t)std::min<uint64_t>({kBatch, window - outstanding, n - next});
      for (uint32_t j = 0; j < m; ++j) {
        const uint64_t k = sl->lo + next + j;
        iov[j].iov_base = const_cast<uint8_t*>(reqs + k * req_len);
        iov[j].iov_len = req_len;
        memset(&mm[j], 0, sizeof mm[j]);
        mm[j].msg_hdr.msg_name = &srv;
        mm[j].msg_hdr.msg_namelen = sizeof srv;
        mm[j].msg_hdr.msg_iov = &iov[j];
        mm[j].msg_hdr.msg_iovlen = 1;
      }
      const int sent = sendmmsg(fd, mm, m, 0);
      if (sent < 0) {
        if (errno == EAGAIN || errno == ENOBUFS) break;
        sl->err = -errno;
        close(fd);
        return;
      }
      const uint64_t t1 = now_ns();
      for (int j = 0; j < sent; ++j) {
        state[next] = 1;
        t_first[next] = t_last[next] = t1;
        ++next;
        ++outstanding;
      }
      if ((uint32_t)sent < m) break;
    }
    // replies
    bool any = false;
    for (;;) {
      for (uint32_t j = 0; j < kBatch; ++j) {
        iov[j].iov_base = rbuf.data() + (size_t)j * rsz;
        iov[j].iov_len = rsz;
        memset(&mm[j], 0, sizeof mm[j]);
        mm[j].msg_hdr.msg_iov = &iov[j];
        mm[j].msg_hdr.msg_iovlen = 1;
      }
      const int got = recvmmsg(fd, mm, kBatch, MSG_DONTWAIT, nullptr);
      if (got <= 0) break;
      any = true;
      const uint64_t t1 = now_ns();
      for (int j = 0; j < got; ++j) {
        const uint8_t* rb = rbuf.data() + (size_t)j * rsz;
        const uint32_t r = mm[j].msg_len;
        if (r < 16) continue;
        uint64_t id;
        memcpy(&id, rb, 8);
        if (id == 0) continue;
        const uint64_t k = id - 1;
        if (k < sl->lo || k >= sl->hi) continue;
        const uint64_t i = k - sl->lo;
        if (state[i] != 1) continue;  // duplicate
        state[i] = 2;
        const uint32_t len = std::min<uint32_t>(r, stride);
        memcpy(replies + k * (uint64_t)stride, rb, len);
        reply_len[k] = r;
        if (lat_ns) lat_ns[k] = t1 - t_first[i];
        --outstanding;
        ++done;
      }
      if ((uint32_t)got < kBatch) break;
    }
    while (oldest < next && state[oldest] == 2) ++oldest;
    if (!any) {
      // retransmit what has waited too long, then wait for the socket
      const uint64_t t2 = now_ns();
      for (uint64_t i = oldest; i < next; ++i) {
        if (state[i] == 1 && t2 - t_last[i] > rto_ns) {
          const uint64_t k = sl->lo + i;
          if (sendto(fd, reqs + k * req_len, req_len, 0, (sockaddr*)&srv, sizeof srv) >= 0) {
            t_last[i] = t2;
            ++sl->retransmits;
          }
        }
      }
      pollfd p{fd, POLLIN, 0};
      poll(&p, 1, 1);
    }
  }
  sl->completed = done;
  close(fd);
}

}  // namespace

extern "C" int64_t gsys_kv_loadgen(uint32_t server_port, const uint8_t* reqs, uint32_t req_len,
                                   uint64_t n, uint32_t threads, uint32_t window, uint64_t rto_ns,
                                   uint64_t timeout_ns, uint8_t* replies, uint32_t reply_stride,
                                   uint32_t* reply_len, uint64_t* lat_ns, uint64_t* retransmits) {
  if (!reqs || !replies || !reply_len || !req_len || !threads || !window || reply_stride < 16)
    return -EINVAL;
  if (!n) return 0;
  const uint64_t deadline = now_ns() + (timeout_ns ? timeout_ns : 60000000000ull);
  std::vector<Slice> sl(threads);
  std::vector<std::thread> th;
  for (uint32_t t = 0; t < threads; ++t) {
    sl[t].lo = n * t / threads;
    sl[t].hi = n * (t + 1) / threads;
    th.emplace_back(client, server_port, reqs, req_len, &sl[t], window, rto_ns ? rto_ns : 20000000ull,
                    deadline, replies, reply_stride, reply_len, lat_ns);
  }
  for (auto& x : th) x.join();
  int64_t total = 0;
  uint64_t rt = 0;
  int err = 0;
  for (auto& s : sl) {
    total += (int64_t)s.completed;
    rt += s.retransmits;
    if (s.err && !err) err = s.err;
  }
  if (retransmits) *retransmits = rt;
  return err && total < (int64_t)n ? err : total;
}
