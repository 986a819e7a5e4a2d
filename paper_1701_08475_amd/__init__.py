"""MI355X-native kNN-graph construction by repeated two-means bisection
(Zhao, Yang, Deng, arXiv 1701.08475, Sec. 3.1, Algorithm 1).

Importing the package loads nothing; ``paper_1701_08475_amd.knng`` binds the
HIP library ``libknng.so`` on first use and raises if it is missing.
"""
