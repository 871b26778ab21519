"""Write skip_gap_edge.txt: a gamete whose geometric-gap crossover walk
consumes the word 0xFFFFFFFF while a crossover is still to follow.

Crossovers at independent boundaries (Supplementary S2, "Genetics") are
drawn as geometric gaps by inversion, gap = min{k : x < T_k} with
T_k = floor((1 - (1-r)^(k+1)) 2^32).  For r = 0.09 and L = 1024 the table
reaches 2^32 inside the genome, so a word of 0xFFFFFFFF must give the index
of that entry.
The search uses only the oracle: its Philox words and its table.  Run from
the repository root: python tests/golden/make_skip_gap_edge.py
"""
import os
import sys
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

SEED, C3, R, L, SLOTS = 7, 0, 0.09, 1024, 4096
CHUNK = 32  # generations per search task
X = 0xFFFFFFFF


def main():
    found = []
    lock = threading.Lock()
    nxt = [1000]

    def worker():
        while True:
            with lock:
                if found:
                    return
                t0 = nxt[0]
                nxt[0] += CHUNK
            hit = oracle.find_gap_word(SEED, C3, R, L, SLOTS, t0, t0 + CHUNK, X)
            if hit:
                with lock:
                    found.append(hit)
                return

    threads = [threading.Thread(target=worker) for _ in range(os.cpu_count() or 4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    # the earliest hit among the chunks that finished
    t, j, stream, word, b = min(found)
    gap = oracle.skip_gap(R, L, X)
    with open(os.path.join(HERE, "skip_gap_edge.txt"), "w") as f:
        f.write("# Gamete whose geometric-gap walk reads the word 0xFFFFFFFF with a crossover still to follow\n")
        f.write("# (Supplementary S2, Genetics: independent crossovers, geometric gaps by inversion).\n")
        f.write("# Written by tests/golden/make_skip_gap_edge.py from the oracle's Philox words and table.\n")
        f.write("# seed c3 r n_loci slots generation slot stream word_index boundary_before gap\n")
        f.write(f"{SEED} {C3} {R} {L} {SLOTS} {t} {j} {stream} {word} {b} {gap}\n")
    print(t, j, stream, word, b, gap)


if __name__ == "__main__":
    main()
