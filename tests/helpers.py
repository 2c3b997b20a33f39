"""Shared glue for the parity tests: build a GPU table and the matching
oracle configuration, move seeded keys between host and device, and read back
raw table images."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2406_09255_amd as cpht
import synth


def oracle_cfg(t: "cpht.Table") -> oracle.Cfg:
    c = t.config
    return oracle.Cfg(scheme=c.scheme, w=c.key_bits, log2_slots0=c.log2_slots0, log2_slots1=c.log2_slots1,
                      B0=c.bucket0, B1=c.bucket1, s0=c.slot_bits0, s1=c.slot_bits1, H=c.n_hash,
                      C=c.max_chain, compact=c.compact, log2_lists=c.log2_lists, pool_slabs=c.pool_slabs,
                      pad=0, seed=c.seed)


def oracle_table(t: "cpht.Table") -> oracle.Table:
    c = t.config
    return oracle.Table(c.scheme, c.key_bits, c.log2_slots0, c.bucket0, c.slot_bits0,
                        log2_slots1=c.log2_slots1, B1=c.bucket1, s1=c.slot_bits1, H=c.n_hash,
                        C=c.max_chain, compact=bool(c.compact), seed=c.seed, log2_lists=c.log2_lists,
                        pool_slabs=c.pool_slabs)


def to_dev(keys: torch.Tensor, w: int, device) -> torch.Tensor:
    return synth.to_words(keys, w).to(device).contiguous()


def host_u64(keys: torch.Tensor) -> np.ndarray:
    return synth.from_words(keys.cpu()).numpy().astype(np.uint64)


def images(t: "cpht.Table"):
    return [t.export(x) for x in range(t.nimages)]


def check_table(t: "cpht.Table"):
    """Checker invariants on the GPU table; returns the decoded key set."""
    imgs = images(t)
    ok, msg, keys = oracle.check_images(oracle_cfg(t), *imgs)
    assert ok, f"table checker: {msg}"
    return keys
