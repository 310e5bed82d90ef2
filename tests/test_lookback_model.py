"""A model of the cross-segment look-back (the decoupled look-back of the transcode
kernels) under the dispatch the hardware allows, run on the CPU.

The machine: 8 XCDs with a few workgroup slots each.  Two kernels run at once; each
kernel's workgroup i goes to XCD i mod 8, and each XCD dispatches each kernel's
workgroups in index order, but is free to interleave the two kernels.  An adversarial
dispatcher fills XCD x with kernel (x mod 2)'s workgroups first.  A resident workgroup
publishes its aggregate, then walks back over its predecessors' status words (an
inclusive prefix ends the walk); a predecessor that has published nothing after
`patience` polls gets its aggregate recomputed by the waiting workgroup (which costs it
`cost` steps), as lookback_wave does.

Checked: with the recompute every workgroup of both kernels finishes and every
exclusive prefix equals the plain sum of the aggregates before it; without it (infinite
patience) the same dispatch deadlocks, so the model does reach the case the recompute
exists for.
"""
import itertools

import numpy as np
import pytest

N_XCD = 8


class Kernel:
    def __init__(self, n, rng):
        self.n = n
        self.agg = rng.integers(0, 1000, n)
        self.status = [None] * n  # None, ("A", aggregate) or ("P", inclusive prefix)
        self.excl = [None] * n
        self.next_per_xcd = {x: x for x in range(N_XCD)}  # next index each XCD dispatches


class Workgroup:
    def __init__(self, kern, i, patience, cost):
        self.k, self.i = kern, i
        self.patience, self.cost = patience, cost
        self.state = "publish"
        self.top = i - 1
        self.excl = 0
        self.polls = 0
        self.busy = 0
        self.fixed = {}

    def step(self):
        """One time step; returns True when the workgroup has finished."""
        k = self.k
        if self.busy:
            self.busy -= 1
            return False
        if self.state == "publish":
            k.status[self.i] = ("P", k.agg[0]) if self.i == 0 else ("A", k.agg[self.i])
            if self.i == 0:
                k.excl[0] = 0
                return True
            self.state = "look"
            return False
        # one poll of the window (the model takes the whole remaining walk as the window)
        while self.top >= 0:
            st = self.fixed.get(self.top) or k.status[self.top]
            if st is None:
                self.polls += 1
                if self.polls >= self.patience:
                    # recompute the missing aggregate from the input
                    v = k.agg[self.top]
                    self.fixed[self.top] = ("P", v) if self.top == 0 else ("A", v)
                    self.busy = self.cost
                    self.polls = 0
                return False
            self.excl += st[1]
            self.top -= 1
            if st[0] == "P":
                break
        k.excl[self.i] = self.excl
        k.status[self.i] = ("P", self.excl + k.agg[self.i])
        return True


def simulate(n_per_kernel, slots, patience, cost=3, max_steps=200_000, seed=0):
    rng = np.random.default_rng(seed)
    kernels = [Kernel(n_per_kernel, rng), Kernel(n_per_kernel, rng)]
    resident = {x: [] for x in range(N_XCD)}
    done = 0
    total = 2 * n_per_kernel
    last_progress = 0
    for t in itertools.count():
        # dispatch: XCD x prefers kernel x % 2, then the other (in index order per kernel)
        for x in range(N_XCD):
            for kk in (x % 2, 1 - x % 2):
                k = kernels[kk]
                while len(resident[x]) < slots and k.next_per_xcd[x] < k.n:
                    resident[x].append(Workgroup(k, k.next_per_xcd[x], patience, cost))
                    k.next_per_xcd[x] += N_XCD
        progressed = False
        for x in range(N_XCD):
            keep = []
            for wg in resident[x]:
                if wg.step():
                    done += 1
                    progressed = True
                else:
                    keep.append(wg)
            resident[x] = keep
        if progressed:
            last_progress = t
        if done == total:
            return kernels, t
        if t - last_progress > 10_000 or t > max_steps:
            return None, t


def test_every_wait_ends_with_recompute():
    for seed in range(5):
        kernels, steps = simulate(n_per_kernel=400, slots=6, patience=64, seed=seed)
        assert kernels is not None, "stuck at step %d" % steps
        for k in kernels:
            want = np.concatenate([[0], np.cumsum(k.agg)[:-1]])
            assert list(k.excl) == list(want)
            assert k.status[-1] == ("P", int(np.sum(k.agg)))


def test_same_dispatch_deadlocks_without_recompute():
    kernels, steps = simulate(n_per_kernel=400, slots=6, patience=float("inf"))
    assert kernels is None


@pytest.mark.parametrize("slots", [1, 2, 16])
def test_single_kernel_any_residency(slots):
    """One kernel alone: in-order dispatch already guarantees progress; the recompute
    leaves the prefixes unchanged."""
    rng = np.random.default_rng(slots)
    k = Kernel(300, rng)
    resident = {x: [] for x in range(N_XCD)}
    done = 0
    for _ in range(100_000):
        for x in range(N_XCD):
            while len(resident[x]) < slots and k.next_per_xcd[x] < k.n:
                resident[x].append(Workgroup(k, k.next_per_xcd[x], 4, 2))
                k.next_per_xcd[x] += N_XCD
        for x in range(N_XCD):
            keep = []
            for wg in resident[x]:
                if wg.step():
                    done += 1
                else:
                    keep.append(wg)
            resident[x] = keep
        if done == k.n:
            break
    assert done == k.n
    assert list(k.excl) == list(np.concatenate([[0], np.cumsum(k.agg)[:-1]]))
