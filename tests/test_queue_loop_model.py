"""Host model of the barrier sequence of the tile-pair pass's persistent loop.

The workgroup's four waves are four threads sharing the loop's LDS fields
(`bi`, `bn`: the next prefetched entry and the number prefetched; `q`: the
entry being worked on).  Wave 0 refills the batch of prefetched queue
entries (its lane 0 writes `bn` and `bi` before the refill barrier), thread 0
pops the next entry before the post-pop barrier, and a hardware barrier only
counts arrivals: it does not know which `__syncthreads()` each wave reached.

The model replays two interleavings in which one wave is slow:

* it reaches the loop top after wave 0 has already rewritten `bn` / `bi` in
  its refill;
* it reaches the loop top after thread 0 has already popped the next entry
  (no refill due), leaving `bi == bn`.

With the refill predicate read from `bi` / `bn` at the loop top (the earlier
kernel), the slow wave takes a different barrier sequence from the rest of
the block: one barrier generation mixes two barrier sites, and from then on
waves work on different queue entries in the same iteration (the tile pair
staged from two different pops).  With the predicate latched by every wave
between the post-pop barrier and the end-of-iteration barrier (the committed
kernel), every generation joins the same site and every wave sees the same
sequence of entries, in both interleavings.
"""
import threading

import pytest

QUEUE = 7      # queue entries
QB = 2         # entries per refill
WAVES = 4


class SiteBarrier:
    """A barrier that counts arrivals like s_barrier and records, per
    generation, the site each thread arrived from."""

    def __init__(self, n, timeout=2.0):
        self.n, self.timeout = n, timeout
        self.cv = threading.Condition()
        self.count, self.gen = 0, 0
        self.sites = {}
        self.broken = False

    def wait(self, site):
        with self.cv:
            if self.broken:
                raise RuntimeError("broken")
            g = self.gen
            self.sites.setdefault(g, []).append(site)
            self.count += 1
            if self.count == self.n:
                self.count = 0
                self.gen += 1
                self.cv.notify_all()
                return
            if not self.cv.wait_for(lambda: self.gen != g or self.broken, self.timeout):
                self.broken = True
                self.cv.notify_all()
                raise RuntimeError("barrier never completed")
            if self.broken:
                raise RuntimeError("broken")


def run_block(latched, slow_at):
    """Run one workgroup over the queue; `slow_at` = ("refill" | "pop", k):
    wave 1 reaches the loop top of iteration k only after wave 0's refill
    writes / thread 0's pop of that iteration."""
    S = {"bi": 0, "bn": 0, "q": -2, "bq0": 0, "next": 0}
    bar = SiteBarrier(WAVES)
    event = threading.Event()
    staged = {w: [] for w in range(WAVES)}
    errors = []

    def refill():
        q0 = S["next"]
        S["next"] += QB
        S["bq0"] = q0
        S["bn"] = max(0, min(QB, QUEUE - q0))
        S["bi"] = 0

    def pop():
        if S["bi"] >= S["bn"]:
            S["q"] = -1
            return
        S["q"] = S["bq0"] + S["bi"]
        S["bi"] += 1

    def wave(w):
        need_refill = True
        it = 0
        try:
            while True:
                if w == 1 and it == slow_at[1]:
                    event.wait(1.0)
                refill_now = need_refill if latched else S["bi"] >= S["bn"]
                if refill_now:
                    if w == 0:
                        refill()
                        if slow_at[0] == "refill" and it == slow_at[1]:
                            event.set()
                    bar.wait("refill")
                if w == 0:
                    pop()
                    if slow_at[0] == "pop" and it == slow_at[1]:
                        event.set()
                bar.wait("pop")
                if S["q"] < 0:
                    break
                if latched:
                    need_refill = S["bi"] >= S["bn"]
                staged[w].append(S["q"])
                bar.wait("work")
                bar.wait("end")
                it += 1
        except RuntimeError as e:
            errors.append((w, str(e)))

    ts = [threading.Thread(target=wave, args=(w,)) for w in range(WAVES)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(10.0)
    mixed = [g for g, s in bar.sites.items() if len(set(s)) > 1]
    return mixed, staged, errors


# iterations at which wave 0 refills (QB entries per batch): 0, 2, 4, ...;
# iterations with no refill due: 1, 3, ...
@pytest.mark.parametrize("slow_at", [("refill", 2), ("refill", 4), ("pop", 1), ("pop", 3)])
def test_loop_top_predicate_skews_the_barriers(slow_at):
    mixed, staged, errors = run_block(latched=False, slow_at=slow_at)
    # a barrier generation joins different sites, or the block deadlocks, or
    # waves work on different entries
    diverged = any(staged[w] != staged[0] for w in range(WAVES))
    assert mixed or errors or diverged, (mixed, staged, errors)


@pytest.mark.parametrize("slow_at", [("refill", 2), ("refill", 4), ("pop", 1), ("pop", 3),
                                     ("none", -1)])
def test_latched_predicate_keeps_the_barriers_in_step(slow_at):
    mixed, staged, errors = run_block(latched=True, slow_at=slow_at)
    assert not mixed and not errors, (mixed, errors)
    for w in range(WAVES):
        assert staged[w] == list(range(QUEUE)), (w, staged[w])
