"""MI355X-native HDD partial inverse (hierarchical domain decomposition).

The product is the HIP library libhdd.so behind the C ABI in include/hdd.h;
`paper_1708_02207_amd.hdd` is its Python binding.
"""
