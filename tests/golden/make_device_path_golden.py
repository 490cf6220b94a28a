"""Write tests/golden/device_path_bc.txt: the oracle's betweenness (Algorithm 1,
ordered pairs) of the graph that tests/c_api/device_path.cpp builds -- a
60-cycle with a chord (i, i+30 mod 60) for every i that is a multiple of 7,
and pendants 60, 61 on vertex 5 and 62 on vertex 33.  Calls only oracle/.

    python tests/golden/make_device_path_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def graph():
    n = 63
    adj = [set() for _ in range(n)]

    def add(a, b):
        adj[a].add(b)
        adj[b].add(a)

    for i in range(60):
        add(i, (i + 1) % 60)
    for i in range(0, 60, 7):
        add(i, (i + 30) % 60)
    add(60, 5)
    add(61, 5)
    add(62, 33)
    rp = np.zeros(n + 1, np.int32)
    col = []
    for v in range(n):
        nb = sorted(adj[v])
        rp[v + 1] = rp[v] + len(nb)
        col.extend(nb)
    return n, rp, np.array(col, np.int32)


def main():
    n, rp, col = graph()
    bc = oracle.bc_plain(n, rp, col, threads=1)
    with open(os.path.join(HERE, "device_path_bc.txt"), "w") as f:
        f.write("# oracle betweenness (Algorithm 1, ordered pairs) of the device_path.cpp graph, one value per vertex\n")
        f.write(f"{n}\n")
        for x in bc:
            f.write(f"{float(x)!r}\n")


if __name__ == "__main__":
    main()
