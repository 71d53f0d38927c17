"""Quadtree partitions and their refinement (Sec. 6.1 "Quadtree Partition", Sec. 6.2 "Refining
Quadtree Partition", Sec. 6.3 "4d Partition"), pointer-based, in plain Python.

TEST INFRASTRUCTURE (see the package docstring): only tests/, smoke() and bench.py's
cpu_baseline leg may use it.

A forest of R quadtrees over the unit square (R = 1 for the 2-D screen partition; one
tree per top-level grid cell for the 4-D partition, each over the two direction
coordinates). The regions are the leaves. Nodes are numbered in creation order: the roots
0..R-1, then the four children of every split, in the order the splits are made.

* lookup: descend from the root; at a node with square [x0, x0 + s) x [y0, y0 + s) the
  child is (x >= x0 + s/2) + 2 (y >= y0 + s/2); points outside [0, 1]^2, or NaN, have no
  region (-1);
* refinement: the leaves visited more than M_split times since the last refinement split
  into four, in increasing node order; children do not split in the same refinement; a
  split child inherits the parent's scaling parameter lambda as it is and n_k / 4 as its
  number of updates (rounded down and kept >= 1 so that the step size stays finite; the
  paper does not say), with an empty pending window (A = 0, i = 0); every visit counter
  then restarts from 0. When the node storage (capacity) cannot hold all splits, only the
  first ones in node order are made. Leaves at MAX_DEPTH do not split (so every square
  corner is exact in float32, and lookups decide the same way in float32 and float64).
"""

import math

import numpy as np

MAX_DEPTH = 20


class Node:
    __slots__ = ("index", "depth", "x0", "y0", "children", "visits")

    def __init__(self, index, depth, x0, y0):
        self.index = index
        self.depth = depth
        self.x0 = x0      # lower corner; the side is 2^-depth
        self.y0 = y0
        self.children = None
        self.visits = 0

    @property
    def side(self):
        return 0.5 ** self.depth


class Forest:
    def __init__(self, n_roots, capacity):
        if capacity < n_roots:
            raise ValueError("capacity below the number of roots")
        self.capacity = capacity
        self.nodes = [Node(i, 0, 0.0, 0.0) for i in range(n_roots)]
        self.n_roots = n_roots

    def leaves(self):
        return [n for n in self.nodes if n.children is None]

    def lookup(self, root, x, y, count=True):
        """Leaf index of point (x, y) in tree `root`, or -1."""
        if root < 0 or root >= self.n_roots:
            return -1
        if not (0.0 <= x <= 1.0 and 0.0 <= y <= 1.0):  # also rejects NaN
            return -1
        node = self.nodes[root]
        while node.children is not None:
            h = node.side / 2
            q = int(x >= node.x0 + h) + 2 * int(y >= node.y0 + h)
            node = node.children[q]
        if count:
            node.visits += 1
        return node.index

    def lookup_many(self, root, x, y, count=True):
        """lookup() of many points at once: every point descends one level per step, so
        the half side h is the same for all points at a step. root: int array (or None for
        tree 0), x, y: float arrays. Returns int64 leaf indices (-1 where none)."""
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        root = np.zeros(x.shape, dtype=np.int64) if root is None else np.asarray(root, dtype=np.int64)
        child = np.asarray(self.child_array(), dtype=np.int64)
        valid = (root >= 0) & (root < self.n_roots) & (x >= 0) & (x <= 1) & (y >= 0) & (y <= 1)
        node = np.where(valid, root, 0)
        x0 = np.zeros(x.shape)
        y0 = np.zeros(x.shape)
        h = 0.5
        for _ in range(MAX_DEPTH + 1):
            first = child[node]
            inner = valid & (first >= 0)
            if not inner.any():
                break
            right = x >= x0 + h
            top = y >= y0 + h
            node = np.where(inner, first + right + 2 * top, node)
            x0 = np.where(inner & right, x0 + h, x0)
            y0 = np.where(inner & top, y0 + h, y0)
            h /= 2
        leaf = np.where(valid, node, -1)
        if count:
            hits = np.bincount(leaf[valid], minlength=len(self.nodes))
            for n, c in zip(self.nodes, hits.tolist()):
                n.visits += c
        return leaf

    def visits_array(self):
        return [n.visits for n in self.nodes]

    def corners(self):
        """(x0, y0, side) of every node, in node order."""
        return [(n.x0, n.y0, n.side) for n in self.nodes]

    def refine(self, m_split, state=None):
        """One refinement pass; `state` (oracle.region_adapt state arrays indexed by node,
        length >= capacity) receives the children's inherited parameters. Returns the
        number of splits."""
        splitting = [n for n in self.nodes if n.children is None and n.visits > m_split and n.depth < MAX_DEPTH]
        room = (self.capacity - len(self.nodes)) // 4
        splitting = splitting[:room]
        for parent in splitting:
            h = parent.side / 2
            kids = []
            for q in range(4):
                c = Node(len(self.nodes), parent.depth + 1, parent.x0 + h * (q & 1), parent.y0 + h * (q >> 1))
                self.nodes.append(c)
                kids.append(c)
                if state is not None:
                    state["lambda"][c.index] = state["lambda"][parent.index]
                    state["updates"][c.index] = max(1, int(state["updates"][parent.index]) // 4)
                    state["acc"][c.index] = 0.0
                    state["visits"][c.index] = 0
            parent.children = kids
        for n in self.nodes:
            n.visits = 0
        return len(splitting)

    def child_array(self):
        """First child index per node (-1 for a leaf), the layout the GPU keeps."""
        return [-1 if n.children is None else n.children[0].index for n in self.nodes]

    def depth_array(self):
        return [n.depth for n in self.nodes]

    def area(self):
        """Total area of the leaves (each tree covers area 1)."""
        return math.fsum(n.side * n.side for n in self.leaves())
