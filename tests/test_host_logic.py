"""Host-side logic of the library that needs no GPU.

The server admits requests by device bytes and component slots with a
first-fit range allocator (csrc/range_alloc.h).  A tiny driver built with
g++ replays random allocate/release sequences and must agree, call for call,
with a straightforward Python model of first fit over a sorted free list.
"""
import os
import random
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_14335_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "range_alloc.h"
int main() {
  mpld::RangeAlloc a;
  char op;
  long long x, y;
  while (std::scanf(" %c %lld %lld", &op, &x, &y) == 3) {
    if (op == 'r') { a.reset(x); std::printf("ok\n"); }
    else if (op == 'a') {
      const long long off = a.alloc(x, y);
      std::printf("%lld %lld\n", off, (long long)a.used());
    }
    else if (op == 'f') { a.release(x, y); std::printf("%lld\n", (long long)a.used()); }
  }
  return 0;
}
"""


class Model:
    def __init__(self, cap):
        self.free = [[0, cap]] if cap > 0 else []
        self.used = 0

    def alloc(self, length, align):
        for i, (beg, size) in enumerate(self.free):
            start = (beg + align - 1) // align * align
            end = beg + size
            if start + length > end:
                continue
            del self.free[i]
            pieces = []
            if start > beg:
                pieces.append([beg, start - beg])
            if start + length < end:
                pieces.append([start + length, end - start - length])
            self.free[i:i] = pieces
            self.used += length
            return start
        return -1

    def release(self, off, length):
        self.used -= length
        self.free.append([off, length])
        self.free.sort()
        merged = []
        for beg, size in self.free:
            if merged and merged[-1][0] + merged[-1][1] == beg:
                merged[-1][1] += size
            else:
                merged.append([beg, size])
        self.free = merged


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("ra")
    src = d / "ra.cpp"
    src.write_text(DRIVER)
    exe = d / "ra"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)])
    return str(exe)


@pytest.mark.parametrize("seed", range(4))
def test_range_alloc_matches_first_fit_model(driver, seed):
    rng = random.Random(seed)
    cap = rng.choice([4096, 1 << 20])
    ops = [("r", cap, 0)]
    model = Model(cap)
    expect = ["ok"]
    live = []
    for _ in range(600):
        if live and rng.random() < 0.45:
            off, length = live.pop(rng.randrange(len(live)))
            ops.append(("f", off, length))
            model.release(off, length)
            expect.append(str(model.used))
        else:
            length = rng.randint(1, cap // 8)
            align = rng.choice([1, 8, 256])
            ops.append(("a", length, align))
            got = model.alloc(length, align)
            expect.append(f"{got} {model.used}")
            if got >= 0:
                live.append((got, length))
    inp = "\n".join(f"{o} {x} {y}" for o, x, y in ops) + "\n"
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    assert out[: len(expect)] == expect
    # everything released: one free range again, nothing used
    for off, length in live:
        model.release(off, length)
    assert model.free == [[0, cap]] and model.used == 0
