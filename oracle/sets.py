"""Plain set semantics of a batch of hash-table operations.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Below the load at which a table first answers FULL, every correct table
computes exactly this (Theorem 1 (c), (d) of Appendix A and the corollary
that closes it: at most one find-or-put of a key returns PUT, the others
return FOUND).  No hashing is involved; numpy's sort, unique and isin are the
only library steps.
"""
from __future__ import annotations

import numpy as np

PUT, FOUND, FULL = 1, 2, 3


def as_set(keys) -> np.ndarray:
    """Sorted distinct keys."""
    return np.unique(np.asarray(keys, dtype=np.uint64))


def find(S: np.ndarray, queries) -> np.ndarray:
    """Membership: 1 where the query is in S, else 0."""
    q = np.asarray(queries, dtype=np.uint64)
    return np.isin(q, S).astype(np.uint8)


def insert(S: np.ndarray, keys):
    """Operations applied in index order to the set S.

    Returns (outcomes, S_after): FOUND for keys already in S or inserted by an
    earlier operation of the batch, PUT for the first occurrence of every
    other key."""
    k = np.asarray(keys, dtype=np.uint64)
    out = np.full(k.size, FOUND, np.uint8)
    _, first = np.unique(k, return_index=True)
    first = np.sort(first)
    new_first = first[~np.isin(k[first], S)]
    out[new_first] = PUT
    return out, np.union1d(S, k)


def insert_values(M: dict, keys, values):
    """Map find-or-put applied in index order to the dictionary M (key ->
    value): a key not in M is stored with the value of this operation (PUT),
    a key already in M keeps its value (FOUND).  Returns the answers; M is
    updated in place."""
    out = np.empty(len(keys), np.uint8)
    for i, (k, v) in enumerate(zip((int(x) for x in keys), (int(x) for x in values))):
        if k in M:
            out[i] = FOUND
        else:
            M[k] = v
            out[i] = PUT
    return out


def find_values(M: dict, keys):
    """Map lookup: (found, value) per key; value 0 where not found."""
    found = np.array([int(k) in M for k in keys], dtype=np.uint8)
    vals = np.array([M.get(int(k), 0) for k in keys], dtype=np.uint64)
    return found, vals


def delete(S: np.ndarray, keys):
    """Deletions applied in index order to S.

    Returns (answers, S_after): 1 at the first occurrence of every key of S
    (that operation removes it), 0 for keys not in S and for repeats."""
    k = np.asarray(keys, dtype=np.uint64)
    out = np.zeros(k.size, np.uint8)
    _, first = np.unique(k, return_index=True)
    hit = first[np.isin(k[first], S)]
    out[hit] = 1
    return out, np.setdiff1d(S, k)


def mixed(S: np.ndarray, keys, ops):
    """Finds (op 0) and inserts (op 1) applied in index order to S.

    Returns (answers, S_after, racy): answers are the sequential results (0/1
    for finds, PUT/FOUND for inserts); racy marks finds whose key is absent
    from S but inserted somewhere in this batch.  Under concurrent execution
    such a find may answer either way; every other answer is fixed."""
    k = np.asarray(keys, dtype=np.uint64)
    o = np.asarray(ops, dtype=np.uint8)
    ins = o == 1
    out = np.zeros(k.size, np.uint8)
    # sequential answer for a find at position p: key in S, or inserted at some q < p
    inserted_keys = k[ins]
    ins_pos = np.nonzero(ins)[0]
    # first insert position of every inserted key
    uk, first_idx = np.unique(inserted_keys, return_index=True)
    first_pos = ins_pos[first_idx]
    in_S = np.isin(k, S)
    pos_of = np.searchsorted(uk, k)
    pos_of = np.minimum(pos_of, max(0, uk.size - 1))
    has_ins = (uk.size > 0) & (uk[pos_of] == k) if uk.size else np.zeros(k.size, bool)
    earliest = np.where(has_ins, first_pos[pos_of] if uk.size else 0, np.iinfo(np.int64).max)
    idx = np.arange(k.size)
    finds = ~ins
    out[finds] = (in_S[finds] | (earliest[finds] < idx[finds])).astype(np.uint8)
    racy = finds & ~in_S & has_ins
    ins_out, S_after = insert(S, inserted_keys)
    out[ins] = ins_out
    return out, S_after, racy


def check_insert_outcomes(S_before: np.ndarray, keys, outcomes) -> tuple[bool, str]:
    """Check concurrent insert outcomes against the set semantics.

    Which occurrence of a duplicated new key is the PUT depends on timing, so
    the comparison is per distinct key: a key already in S_before must be
    FOUND every time; any other key must be PUT exactly once and FOUND for all
    its other occurrences."""
    k = np.asarray(keys, dtype=np.uint64)
    r = np.asarray(outcomes, dtype=np.uint8)
    if k.size != r.size:
        return False, "size mismatch"
    bad = ~np.isin(r, [PUT, FOUND])
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        return False, f"op {i}: outcome {int(r[i])} is neither PUT nor FOUND"
    old = np.isin(k, S_before)
    if (r[old] != FOUND).any():
        i = int(np.nonzero(old & (r != FOUND))[0][0])
        return False, f"op {i}: key already present but outcome {int(r[i])}"
    uk, inv = np.unique(k, return_inverse=True)
    puts = np.bincount(inv, weights=(r == PUT).astype(np.float64), minlength=uk.size)
    new_keys = ~np.isin(uk, S_before)
    want = np.where(new_keys, 1, 0)
    if (puts != want).any():
        j = int(np.nonzero(puts != want)[0][0])
        return False, f"key {int(uk[j])}: {int(puts[j])} PUT outcomes, expected {int(want[j])}"
    return True, ""
