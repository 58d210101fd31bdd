// Host driver for the sanitizer test: calls nf_create on every model
// description file named on the command line (both precision modes) and
// prints one line "<file> <mode> <code>" per call. Built with the same
// sanitizers as the host-only library it links.
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

#include "../../include/nufold.h"

int main(int argc, char** argv) {
  for (int i = 1; i < argc; ++i) {
    std::ifstream f(argv[i], std::ios::binary);
    if (!f) {
      std::printf("%s cannot-open\n", argv[i]);
      return 2;
    }
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    for (int mode = NF_M64; mode <= NF_M32; ++mode) {
      nf_ctx* ctx = nullptr;
      const int code = nf_create(&ctx, text.c_str(), mode, nullptr);
      if (ctx) nf_destroy(ctx);
      std::printf("%s %d %d\n", argv[i], mode, code);
    }
  }
  return 0;
}
