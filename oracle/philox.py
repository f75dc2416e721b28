"""Philox4x64-10 counter-based generator, written from its published definition.

TEST INFRASTRUCTURE ONLY: part of the CPU oracle. Nothing in the product path
may import this module.

Definition followed: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3" (SC'11), section 3.2 (the Philox S-box: two 64x64->128-bit
multiplies per round, hi/lo halves XORed with the other counter words and the
round key; key bumped by the Weyl constants between rounds), with the
multipliers and Weyl constants of that paper's Philox4x64.

Stream convention used by the simulator (one 64-bit word per measure/reset
event, per shot):
    word(seed, shot, e) = philox4x64_10(ctr=(e//4 + 1, 0, 0, 0), key=(seed, shot))[e % 4]
i.e. the e-th output of ``numpy.random.Philox(key=[seed, shot]).random_raw()``,
which advances its counter before producing its first block. The uniform
variate is u = (word >> 11) * 2**-53, in [0, 1). Depolarizing noise draws use
their own counters (noise_word), independent of the event stream.
"""

MASK64 = (1 << 64) - 1

# Philox4x64 round multipliers and Weyl key increments (Salmon et al. 2011).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B


def _mulhilo(a, b):
    p = a * b
    return (p >> 64) & MASK64, p & MASK64


def philox4x64(ctr, key, rounds=10):
    """One Philox4x64-R block: 4 counter words, 2 key words -> 4 output words."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in ctr)
    k0, k1 = (int(x) & MASK64 for x in key)
    for _ in range(rounds):
        hi0, lo0 = _mulhilo(PHILOX_M0, c0)
        hi1, lo1 = _mulhilo(PHILOX_M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + PHILOX_W0) & MASK64
        k1 = (k1 + PHILOX_W1) & MASK64
    return [c0, c1, c2, c3]


def event_word(seed, shot, event):
    """The 64-bit word a shot consumes at its ``event``-th measure/reset."""
    block = philox4x64((event // 4 + 1, 0, 0, 0), (seed, shot))
    return block[event % 4]


def noise_word(seed, shot, sid, loop_code, operand):
    """The word of one depolarizing draw: counter (sid, loop_code, operand, 1),
    output word 0. The fourth counter word is 1 here and 0 in every event
    counter, so noise draws never coincide with measurement/reset draws."""
    return philox4x64((sid, loop_code, operand, 1), (seed, shot))[0]


def word_to_uniform(word):
    """53-bit uniform in [0, 1): the top 53 bits of the word times 2**-53."""
    return float(word >> 11) * (2.0 ** -53)


class ShotStream:
    """Sequential per-shot stream; caches one 4-word block at a time."""

    def __init__(self, seed, shot):
        self.seed = int(seed) & MASK64
        self.shot = int(shot) & MASK64
        self.event = 0
        self._block_index = -1
        self._block = None

    def next_word(self):
        b = self.event // 4
        if b != self._block_index:
            self._block = philox4x64((b + 1, 0, 0, 0), (self.seed, self.shot))
            self._block_index = b
        w = self._block[self.event % 4]
        self.event += 1
        return w

    def next_uniform(self):
        return word_to_uniform(self.next_word())
