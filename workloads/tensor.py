"""Block-sparse tensor container shared by the input generators, the oracle and
the device binding.

This module only stores data. It performs no contraction, factorisation or
any other step of the boundary-MPS method.

Layout
------
A tensor has ``nlegs`` legs. Leg ``l`` is split into ``nsect`` sectors; sector
``s`` carries an integer label tuple (``nlab`` integers) and a dimension.
Each leg also has a direction ``dir`` (+1 or -1) used by abelian flux rules.

Blocks are dense sub-arrays, one per present sector tuple. Block ``i`` covers
the sectors ``blocks[i, :]`` (one sector index per leg) and is stored
row-major (last leg fastest) at ``data[offsets[i] : offsets[i] + size_i]``.
A dense tensor is the special case of one sector per leg and one block.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class Leg:
    labels: np.ndarray          # int32 [nsect, nlab]
    dims: np.ndarray            # int32 [nsect]
    dir: int = 1

    @staticmethod
    def make(pairs, dir=1):
        """``pairs`` is a list of (label_tuple, dim)."""
        labs = np.array([tuple(np.atleast_1d(p[0])) for p in pairs], dtype=np.int32)
        if labs.ndim == 1:
            labs = labs[:, None]
        dims = np.array([int(p[1]) for p in pairs], dtype=np.int32)
        return Leg(labs, dims, int(dir))

    @staticmethod
    def dense(dim, dir=1, label=0):
        return Leg.make([((label,), dim)], dir)

    @property
    def nsect(self):
        return int(self.dims.shape[0])

    @property
    def total(self):
        return int(self.dims.sum())

    def flipped(self):
        return Leg(self.labels.copy(), self.dims.copy(), -self.dir)

    def same_sectors(self, other) -> bool:
        return (self.labels.shape == other.labels.shape
                and np.array_equal(self.labels, other.labels)
                and np.array_equal(self.dims, other.dims))


@dataclass
class Tensor:
    legs: list
    blocks: np.ndarray          # int32 [nblocks, nlegs]
    offsets: np.ndarray         # int64 [nblocks]
    data: np.ndarray            # float64 [nelem]
    _index: dict = field(default=None, repr=False, compare=False)

    @property
    def nlegs(self):
        return len(self.legs)

    @property
    def nblocks(self):
        return int(self.blocks.shape[0])

    def block_shape(self, i):
        return tuple(int(self.legs[l].dims[s]) for l, s in enumerate(self.blocks[i]))

    def block(self, i):
        shp = self.block_shape(i)
        n = int(np.prod(shp)) if shp else 1
        o = int(self.offsets[i])
        return self.data[o:o + n].reshape(shp)

    def find(self, sect_tuple):
        if self._index is None:
            self._index = {tuple(int(v) for v in b): i for i, b in enumerate(self.blocks)}
        return self._index.get(tuple(int(v) for v in sect_tuple))

    def to_dict(self):
        """dict: sector tuple -> ndarray view."""
        return {tuple(int(v) for v in b): self.block(i) for i, b in enumerate(self.blocks)}

    @staticmethod
    def from_blocks(legs, block_list, arrays=None, dtype=np.float64):
        """Build a tensor from an ordered list of sector tuples.

        ``arrays`` (optional) gives the data of each block; otherwise zeros.
        """
        blocks = np.array(block_list, dtype=np.int32).reshape(len(block_list), len(legs))
        sizes = []
        for b in blocks:
            sizes.append(int(np.prod([legs[l].dims[s] for l, s in enumerate(b)])) if len(legs) else 1)
        offsets = np.zeros(len(sizes), dtype=np.int64)
        if sizes:
            offsets[1:] = np.cumsum(sizes)[:-1]
        data = np.zeros(int(sum(sizes)), dtype=dtype)
        t = Tensor(list(legs), blocks, offsets, data)
        if arrays is not None:
            for i, a in enumerate(arrays):
                t.block(i)[...] = a
        return t

    def copy(self):
        return Tensor([Leg(l.labels.copy(), l.dims.copy(), l.dir) for l in self.legs],
                      self.blocks.copy(), self.offsets.copy(), self.data.copy())

    def dense_shape(self):
        return tuple(l.total for l in self.legs)

    def to_dense(self):
        """Embed the blocks into a dense array (sectors laid out in order)."""
        starts = [np.concatenate([[0], np.cumsum(l.dims)[:-1]]).astype(np.int64) for l in self.legs]
        out = np.zeros(self.dense_shape())
        for i, b in enumerate(self.blocks):
            sl = tuple(slice(int(starts[l][s]), int(starts[l][s] + self.legs[l].dims[s]))
                       for l, s in enumerate(b))
            out[sl] = self.block(i)
        return out


def dense_tensor(array, dirs=None):
    """Wrap a dense ndarray as a one-block tensor."""
    array = np.asarray(array, dtype=np.float64)
    dirs = dirs or [1] * array.ndim
    legs = [Leg.dense(n, d) for n, d in zip(array.shape, dirs)]
    return Tensor.from_blocks(legs, [tuple([0] * array.ndim)], [array])
