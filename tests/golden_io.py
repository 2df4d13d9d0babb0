"""Reader for the small text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    n = source = tau = None
    tail, head, w, expect, dist, cells = [], [], [], [], None, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            key, vals = line[0], [int(x) for x in line[1:]]
            if key == "n":
                n = vals[0]
            elif key == "source":
                source = vals[0]
            elif key == "tau":
                tau = vals[0]
            elif key == "arc":
                tail.append(vals[0]); head.append(vals[1]); w.append(vals[2])
            elif key == "edge":
                tail += [vals[0], vals[1]]; head += [vals[1], vals[0]]; w += [vals[2], vals[2]]
            elif key == "expect":
                expect.append((vals[0], vals[1]))
            elif key == "dist":
                dist = np.array(vals, dtype=np.uint64)
            elif key == "cells":
                cells = np.array(vals, dtype=np.uint32)
    return dict(n=n, source=source, tau=tau,
                tail=np.array(tail, dtype=np.uint32), head=np.array(head, dtype=np.uint32),
                w=np.array(w, dtype=np.uint32),
                expect=np.array(sorted(expect), dtype=np.uint32).reshape(-1, 2),
                dist=dist, cells=cells)
