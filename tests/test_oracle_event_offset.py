"""Pin of the oracle's first_event option: a product-state program measured
block by block, each block starting its draws where the earlier blocks' draws
end, gives the same shot as the whole program."""
import workloads as W
from oracle import sim


def test_blockwise_draws_equal_whole_program():
    full, blocks, offs = W.separable_brickwork(seed=9, n=9, blocks=3, layers=6)
    full += "bit[9] f;\nf = measure q;\n"
    for shot in range(6):
        whole = sim.run_shot(full, seed=4, shot=shot)
        bits, record, prob = [], [], 1.0
        for src, off in zip(blocks, offs):
            w = int(src.split("qubit[")[1].split("]")[0])
            o = sim.run_shot(src + f"bit[{w}] f;\nf = measure q;\n", seed=4, shot=shot, first_event=off)
            bits += o.cbits
            record += o.record
            prob *= o.record_prob
        assert bits == whole.cbits and record == whole.record
        assert abs(prob - whole.record_prob) < 1e-12
