"""FP64 CPU oracle of the non-smooth Newton step -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg import this
package.  It shares no code with the GPU library.
"""
