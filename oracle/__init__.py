"""FP64 CPU oracle for KNN-graph-supported k-means (Deng & Zhao, "Fast k-means
based on KNN Graph", arXiv 1705.01813).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library and imports
nothing from it.

Every function is a plain, slow restatement of the paper (and of the readings
listed in the design notes where the paper is silent), computed in float64 from
the same float32 input array the GPU consumes.  Modules:

* ``rng``       counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) and
                Floyd's distinct sampling (Bentley & Floyd, CACM 1987).
* ``twomeans``  Alg. 1 (two-means tree) as a level-synchronous balanced
                bisection.
* ``gkmeans``   Alg. 2 in its Lloyd form (the paper's "GK-means^-", Sec. 4.2):
                candidate collection, restricted argmin, centroid update
                (Eqn. 1 means), distortion (Eqn. 4) and the Eqn. 2 identity, fit.
* ``knng``      Alg. 3 (KNN graph construction): random initial lists,
                intra-cluster exhaustive comparison and list update.
* ``exact``     textbook references used as pins: brute-force KNN and
                exhaustive Lloyd assignment.
* ``metrics``   gap masks, label agreement, graph recall.

Pin status per function is recorded in each module's docstring.
"""
