"""CPU oracle of the QoZ hot path.

TEST INFRASTRUCTURE ONLY: a plain, single-threaded C++ implementation of the
predictor, quantizer, Huffman stage, stream, metrics and tuner, used to check
the GPU library.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import it.
"""
