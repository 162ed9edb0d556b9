// Host test of the request server's bookkeeping (server_book.hpp): the
// first-fit pool allocator and the ticket board.  Built with g++ and the
// address sanitizer by tests/test_server_book_host.py.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <random>
#include <thread>
#include <vector>

#include "server_book.hpp"

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);  \
      exit(1);                                                          \
    }                                                                   \
  } while (0)

struct FakeJob {
  bool done = false;
  int value = 0;
};

static void test_pool() {
  const size_t cap = 64 * psk::kAlign;
  psk::PoolAlloc pa(cap);
  std::vector<char> owner(cap / psk::kAlign, 0);  // live blocks, by 256-byte unit
  std::vector<std::pair<size_t, size_t>> live;
  std::mt19937 rng(7);
  size_t used = 0, peak = 0;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 2) {
      const size_t bytes = 1 + rng() % (8 * psk::kAlign);
      const size_t off = pa.alloc(bytes);
      const size_t units = (bytes + psk::kAlign - 1) / psk::kAlign;
      if (off == SIZE_MAX) {
        // refused only if no free run of that many units exists
        size_t run = 0, best = 0;
        for (char o : owner) {
          run = o ? 0 : run + 1;
          if (run > best) best = run;
        }
        CHECK(best < units);
        continue;
      }
      CHECK(off % psk::kAlign == 0 && off + units * psk::kAlign <= cap);
      for (size_t u = off / psk::kAlign; u < off / psk::kAlign + units; ++u) {
        CHECK(!owner[u]);
        owner[u] = 1;
      }
      live.push_back({off, units});
      used += units * psk::kAlign;
      if (used > peak) peak = used;
    } else {
      const size_t k = rng() % live.size();
      pa.release(live[k].first);
      for (size_t u = live[k].first / psk::kAlign; u < live[k].first / psk::kAlign + live[k].second;
           ++u)
        owner[u] = 0;
      used -= live[k].second * psk::kAlign;
      live[k] = live.back();
      live.pop_back();
    }
    CHECK(pa.used() == used);
  }
  CHECK(pa.peak() == peak);
  for (auto &b : live) pa.release(b.first);
  CHECK(pa.used() == 0);
  CHECK(pa.alloc(cap) == 0);  // everything coalesced back into one range
}

static void test_tickets_single_wait_and_poll() {
  std::mutex mu;
  psk::TicketBoard<FakeJob> board;
  FakeJob *j = new FakeJob();
  int64_t t;
  {
    std::lock_guard<std::mutex> lk(mu);
    t = board.add(j);
  }
  int got = -99;
  {
    std::lock_guard<std::mutex> lk(mu);
    CHECK(board.poll(t, [&](const FakeJob &x) { got = x.value; }) == board.kPending);
    CHECK(board.poll(t + 100, [&](const FakeJob &) {}) == board.kUnknown);
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    j->value = 42;
    j->done = true;
    board.completed();
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    CHECK(board.poll(t, [&](const FakeJob &x) { got = x.value; }) == board.kOk);
    CHECK(got == 42);
    CHECK(board.poll(t, [&](const FakeJob &) {}) == board.kUnknown);
    CHECK(board.size() == 0);
  }
}

// Two threads wait on one ticket while a worker finishes it: exactly one
// gets the result, the other is refused at once; a poll during the wait is
// refused too.  Under the address sanitizer a shared, freed job would fault.
static void test_tickets_two_waiters() {
  for (int rep = 0; rep < 200; ++rep) {
    std::mutex mu;
    psk::TicketBoard<FakeJob> board;
    FakeJob *j = new FakeJob();
    int64_t t;
    {
      std::lock_guard<std::mutex> lk(mu);
      t = board.add(j);
    }
    std::atomic<int> ok{0}, refused{0}, values{0};
    // the second waiter is refused: kClaimed while the first still waits,
    // kUnknown if it arrives after the first has taken the result (a late
    // thread start; both are PSK_EINVAL at the server's interface)
    auto waiter = [&] {
      std::unique_lock<std::mutex> lk(mu);
      int v = -1;
      const int rc = board.wait(lk, t, [&](const FakeJob &x) { v = x.value; });
      if (rc == board.kOk) {
        ++ok;
        values += v;
      } else if (rc == board.kClaimed || rc == board.kUnknown) {
        ++refused;
      }
    };
    std::thread w1(waiter), w2(waiter);
    std::this_thread::sleep_for(std::chrono::microseconds(50 + rep % 7 * 20));
    {
      std::lock_guard<std::mutex> lk(mu);
      const int prc = board.poll(t, [&](const FakeJob &) {});
      CHECK(prc == board.kClaimed || prc == board.kPending);
      j->value = 7;
      j->done = true;
      board.completed();
    }
    w1.join();
    w2.join();
    CHECK(ok == 1);
    CHECK(refused == 1);
    CHECK(values == 7);
    CHECK(board.size() == 0);
  }
}

static void test_clear_deletes_jobs() {
  psk::TicketBoard<FakeJob> board;
  for (int i = 0; i < 5; ++i) board.add(new FakeJob());
  CHECK(board.size() == 5);
  board.clear();
  CHECK(board.size() == 0);
}

int main() {
  test_pool();
  test_tickets_single_wait_and_poll();
  test_tickets_two_waiters();
  test_clear_deletes_jobs();
  printf("server_book ok\n");
  return 0;
}
