"""Device memory reserved once and carved into blocks, for the serving loop.

A serving loop that allocates each job's buffers from PyTorch's caching
allocator runs into that allocator's per-stream caches: jobs run on different
streams, a block freed by one stream is kept for that stream, and with jobs
of widely varying sizes the reserved memory climbs to the device's limit.
The allocator then frees every cached block, synchronizing the device, and
that stall lasts seconds.  Here the loop reserves its budget once, and every
job's buffers are carved from that one reservation:

- `DeviceArena`: best fit over the free holes, placed at the low or the high
  end of the chosen hole, holes merged on release; offsets aligned to 256
  bytes.  Pure bookkeeping: it never touches the device after the one
  allocation that backs it.
- `Slab`: one arena block handed out by bumping a cursor, released as a whole.
  A job holds a few slabs of different lifetimes.  If a slab's first
  estimate is short, the excess comes from the arena as blocks of its own
  (`DeviceArena.spills` counts them) rather than failing the job.

The caller keeps a block until the device work that uses it has completed
(for instance until an event recorded after that work has been reached):
the arena does not track streams.
"""
from __future__ import annotations

import bisect

import torch

ALIGN = 256


def aligned(nbytes: int, align: int = ALIGN) -> int:
    return (max(int(nbytes), 1) + align - 1) // align * align


class DeviceArena:
    """`nbytes` of device memory (one allocation), carved into blocks."""

    def __init__(self, nbytes: int, device="cuda", align: int = ALIGN):
        self.align = int(align)
        self.size = int(nbytes) // self.align * self.align
        if self.size <= 0:
            raise ValueError("an arena needs at least %d bytes" % self.align)
        self.device = torch.device(device)
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=self.device)
        self._offs = [0]          # free holes: offsets (sorted) and sizes
        self._lens = [self.size]
        self._live = {}           # offset -> size of every block handed out
        self.spills = 0
        self.peak = 0

    # ---- bookkeeping
    @property
    def used(self) -> int:
        return self.size - sum(self._lens)

    def largest_hole(self) -> int:
        return max(self._lens, default=0)

    def holes(self) -> list[tuple[int, int]]:
        return list(zip(self._offs, self._lens))

    def _best(self, need: int, lens) -> int:
        best, best_len = -1, None
        for i, n in enumerate(lens):
            if n >= need and (best_len is None or n < best_len):
                best, best_len = i, n
        return best

    def fits(self, sizes) -> bool:
        """Whether blocks of these sizes can all be placed now (best fit, in the order given)."""
        lens = list(self._lens)
        for s in sizes:
            need = aligned(s, self.align)
            i = self._best(need, lens)
            if i < 0:
                return False
            lens[i] -= need
        return True

    def alloc(self, nbytes: int, high: bool = False) -> int | None:
        """Offset of a new block of at least nbytes (None if no hole holds it): the smallest hole
        that fits, its low end (or its high end with `high`)."""
        need = aligned(nbytes, self.align)
        i = self._best(need, self._lens)
        if i < 0:
            return None
        off, n = self._offs[i], self._lens[i]
        if high:
            block = off + n - need
            self._lens[i] = n - need
        else:
            block = off
            self._offs[i] = off + need
            self._lens[i] = n - need
        if self._lens[i] == 0:
            del self._offs[i], self._lens[i]
        self._live[block] = need
        self.peak = max(self.peak, self.used)
        return block

    def release(self, off: int):
        need = self._live.pop(off)
        i = bisect.bisect_left(self._offs, off)
        # merge with the hole before and the hole after
        if i > 0 and self._offs[i - 1] + self._lens[i - 1] == off:
            i -= 1
            self._lens[i] += need
        else:
            self._offs.insert(i, off)
            self._lens.insert(i, need)
        if i + 1 < len(self._offs) and self._offs[i] + self._lens[i] == self._offs[i + 1]:
            self._lens[i] += self._lens[i + 1]
            del self._offs[i + 1], self._lens[i + 1]

    def view(self, off: int, nbytes: int, dtype=torch.uint8) -> torch.Tensor:
        """A 1-D tensor of dtype over [off, off + nbytes) of the arena."""
        esz = torch.empty((), dtype=dtype).element_size()
        if off % esz or nbytes % esz:
            raise ValueError("offset and size must be multiples of the element size")
        return self.buf[off:off + nbytes].view(dtype)


class Slab:
    """One arena block of `nbytes`, handed out in aligned pieces (`empty`), released as a whole."""

    def __init__(self, arena: DeviceArena, nbytes: int, high: bool = False):
        self.arena = arena
        self.size = aligned(nbytes, arena.align)
        self.off = arena.alloc(self.size, high=high)
        if self.off is None:
            raise MemoryError("no hole of %d bytes in the arena (largest %d)" % (self.size, arena.largest_hole()))
        self.cursor = 0
        self._extra = []

    def empty(self, n: int, dtype) -> torch.Tensor:
        """An uninitialized 1-D tensor of max(n, 1) elements of dtype."""
        esz = torch.empty((), dtype=dtype).element_size()
        nbytes = max(int(n), 1) * esz
        need = aligned(nbytes, self.arena.align)
        if self.off is None:
            raise RuntimeError("slab already released")
        if self.cursor + need <= self.size:
            off = self.off + self.cursor
            self.cursor += need
        else:  # the estimate was short: a block of its own, released with the slab
            off = self.arena.alloc(need)
            if off is None:
                raise MemoryError("slab overflow and no hole of %d bytes in the arena" % need)
            self.arena.spills += 1
            self._extra.append(off)
        return self.arena.view(off, nbytes, dtype)

    def zeros(self, n: int, dtype) -> torch.Tensor:
        return self.empty(n, dtype).zero_()

    def release(self):
        if self.off is None:
            return
        self.arena.release(self.off)
        for off in self._extra:
            self.arena.release(off)
        self.off, self._extra = None, []
