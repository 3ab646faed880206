"""Helpers shared by the GPU tests: device <-> host transfers of packed arrays
(marshalling only) and oracle references."""
import sys

import numpy as np

from paper_1609_00061_amd import inputs, pa


def note(*msg):
    """Print the case before a GPU step (flushed), so a failure names it."""
    print("[gpu]", *msg, flush=True)
    sys.stdout.flush()


def to_device(arr):
    import torch
    return torch.from_numpy(pa.pack_bits(arr).copy()).cuda()


def to_host(t, dims):
    import torch
    torch.cuda.synchronize()
    return pa.unpack_bits(t.cpu().numpy(), dims)


def random_relation(seed, arity, degree=3):
    rng = inputs.SplitMix64(seed)
    return inputs.Relation(tuple(range(arity)), degree, rng.normals(inputs.n_monomials(arity, degree)))
