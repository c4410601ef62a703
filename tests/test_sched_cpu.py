"""The serving scheduler's policy on the CPU: the scheduling core of the
library driven through callbacks with a simulated device and clock
(gfc_sched_*).  No GPU is touched."""

import numpy as np
import pytest


class FakeDevice:
    """Simulated clock and device: a batch of n stamps launched at time t
    finishes at t + base + n * per_stamp."""

    def __init__(self, base=1e-3, per_stamp=1e-6, fail_keys=(), poll_fail=()):
        self.t = 0.0
        self.base, self.per_stamp = base, per_stamp
        self.launched = {}      # batch -> dict
        self.released = []
        self.fail_tickets = set(fail_keys)
        self.poll_fail = set(poll_fail)

    def now(self):
        return self.t

    def launch(self, batch, stream, tickets, n_stamps):
        self.launched[batch] = dict(stream=stream, tickets=list(tickets), n=n_stamps, t0=self.t,
                                    t1=self.t + self.base + n_stamps * self.per_stamp)
        return 1 if self.fail_tickets.intersection(tickets) else 0

    def poll(self, batch):
        b = self.launched[batch]
        if self.poll_fail.intersection(b["tickets"]):
            return -1
        return 1 if self.t >= b["t1"] else 0

    def release(self, batch):
        self.released.append(batch)


def make(dev, budget, n_streams=1, max_batch=1 << 20):
    from paper_2012_15797_amd.serving import Scheduler

    return Scheduler(dev.now, dev.launch, dev.poll, dev.release, budget, n_streams, max_batch)


def finish_all(dev, s, ticks=100, dt=1e-3):
    for _ in range(ticks):
        dev.t += dt
        s.step()


def test_admission_is_strict_fifo_under_the_budget():
    dev = FakeDevice()
    s = make(dev, budget=100, n_streams=4)
    t = [s.submit(1, 10, b) for b in (60, 30, 50, 10)]
    s.step()
    assert [s.query(x)[0] for x in t] == ["launched", "launched", "pending", "pending"]
    assert s.usage() == (90, 2)
    dev.t = 1.0
    s.step()
    assert s.query(t[0])[0] == "done"
    s.release(t[0])
    s.step()
    assert s.query(t[2])[0] in ("admitted", "launched") and s.query(t[3])[0] in ("admitted", "launched")
    assert s.usage()[0] == 90
    s.close()


def test_oversized_request_is_rejected():
    from paper_2012_15797_amd import GfcError

    dev = FakeDevice()
    s = make(dev, budget=100)
    with pytest.raises(GfcError) as e:
        s.submit(1, 1, 101)
    assert e.value.status == -6
    s.close()


def test_batches_share_a_key_and_keep_arrival_order():
    dev = FakeDevice()
    s = make(dev, budget=1 << 30, n_streams=1)
    a = s.submit(1, 5, 10)
    b = s.submit(2, 5, 10)
    c = s.submit(1, 7, 10)
    d = s.submit(1, 3, 10)
    s.step()
    (bid, rec), = dev.launched.items()
    assert rec["tickets"] == [a, c, d] and rec["n"] == 15
    assert s.query(b)[0] == "admitted"
    dev.t = 1.0
    s.step()
    assert s.query(b)[0] == "launched" and len(dev.launched) == 2
    s.close()


def test_max_batch_stamps_caps_fusion():
    dev = FakeDevice()
    s = make(dev, budget=1 << 30, n_streams=1, max_batch=100)
    t = [s.submit(1, n, 1) for n in (60, 30, 20)]
    s.step()
    assert list(dev.launched.values())[0]["tickets"] == t[:2]
    finish_all(dev, s, ticks=5)
    assert [r["tickets"] for r in dev.launched.values()] == [t[:2], t[2:]]
    s.close()


def test_plain_mode_launches_each_request_alone():
    dev = FakeDevice()
    s = make(dev, budget=1 << 30, n_streams=1, max_batch=0)
    t = [s.submit(1, 4, 1) for _ in range(5)]
    finish_all(dev, s, ticks=20)
    assert [r["tickets"] for r in dev.launched.values()] == [[x] for x in t]
    assert s.stats()["launches"] == 5
    s.close()


def test_one_batch_in_flight_per_stream_and_continuous_batching():
    dev = FakeDevice(base=10e-3)
    s = make(dev, budget=1 << 30, n_streams=2)
    first = [s.submit(k, 10, 1) for k in (1, 2, 3)]
    s.step()
    assert len(dev.launched) == 2          # two streams busy, third key waits
    assert s.query(first[2])[0] == "admitted"
    # arrivals while both streams are busy are admitted and fused later
    dev.t = 2e-3
    late = [s.submit(3, 10, 1) for _ in range(4)]
    s.step()
    assert len(dev.launched) == 2
    dev.t = 20e-3
    s.step()
    third = list(dev.launched.values())[2]
    assert third["tickets"] == [first[2], *late]
    s.close()


def test_latency_percentiles_on_simulated_clock():
    dev = FakeDevice(base=0.0, per_stamp=1e-3)
    s = make(dev, budget=1 << 30, n_streams=1, max_batch=0)
    sizes = np.arange(1, 101)
    t = [s.submit(1, int(n), 1) for n in sizes]
    finish_all(dev, s, ticks=6000, dt=1e-3)
    assert all(s.query(x)[0] == "done" for x in t)
    st = s.stats()
    assert st["done"] == 100 and st["launches"] == 100
    # every request waited for the ones before it: latency_i ~ sum(sizes[:i+1]) ms
    # (plus at most one 1 ms clock tick per request for the reaping granularity)
    lat = np.cumsum(sizes).astype(float)
    assert lat[49] - 1e-6 <= st["p50_ms"] <= lat[49] + 50 + 1e-6
    assert lat[98] - 1e-6 <= st["p99_ms"] <= lat[98] + 99 + 1e-6
    assert lat[99] - 1e-6 <= st["max_ms"] <= lat[99] + 100 + 1e-6
    s.close()


def test_failed_launch_and_failed_batch_are_isolated():
    dev = FakeDevice()
    s = make(dev, budget=1000, n_streams=1)
    good = s.submit(1, 3, 100)
    bad = s.submit(2, 3, 100)
    dev.fail_tickets = {bad}
    finish_all(dev, s, ticks=10)
    assert s.query(good)[0] == "done"
    assert s.query(bad)[0] == "failed"
    s.release(good)
    s.release(bad)
    assert s.usage() == (0, 0)
    s.close()


def test_release_before_completion_is_refused():
    from paper_2012_15797_amd import GfcError

    dev = FakeDevice(base=1.0)
    s = make(dev, budget=1000)
    t = s.submit(1, 3, 10)
    s.step()
    with pytest.raises(GfcError) as e:
        s.release(t)
    assert e.value.status == -5
    dev.t = 2.0
    s.step()
    s.release(t)
    assert dev.released, "batch memory must be released once its requests are"
    s.close()


def test_device_error_on_poll_fails_only_that_batch():
    dev = FakeDevice()
    s = make(dev, budget=1000, n_streams=2)
    a = s.submit(1, 2, 10)
    b = s.submit(2, 2, 10)
    dev.poll_fail = {b}
    finish_all(dev, s, ticks=5)
    assert s.query(a)[0] == "done" and s.query(b)[0] == "failed"
    s.close()
