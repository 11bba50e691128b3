"""Association of decoded hits with the generator's truth (test helper).

The decoder orders the valid words of a bank by word value, keeping bank order for equal words.
Sorting the generator's (bank, word) pairs the same way gives, for every decoded hit, the raw word
it came from and therefore its truth record.
"""
import numpy as np


def word_bank_ids(bank_offsets):
    counts = np.diff(bank_offsets.astype(np.int64))
    return np.repeat(np.arange(counts.shape[0], dtype=np.int64), counts)


def decoded_word_index(words, bank_offsets):
    """Index into `words` of each decoded hit, in decoded order."""
    bank = word_bank_ids(bank_offsets)
    valid = np.nonzero(words & 0xF)[0]
    key = (bank[valid] << 16) | words[valid].astype(np.int64)
    return valid[np.argsort(key, kind="stable")]


def decoded_truth(batch):
    """Per decoded hit: truth track id (>=0 VELO track, -1 noise, -2 hidden) and measured u."""
    wi = decoded_word_index(batch.words, batch.bank_offsets)
    return batch.truth["track"][wi], batch.truth["u_meas"][wi], wi
